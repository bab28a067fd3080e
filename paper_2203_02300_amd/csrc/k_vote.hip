// k_vote.hip -- disparity refinement by region vote (Eq. 4, Sec. 4.3).
//
// One pass: every valid pixel p takes the disparity with the most votes in
// its stage-1 cross region N_p (for each y' on p's vertical arm, the pixels
// of (x, y')'s horizontal segment); equal counts go to the smallest
// disparity.  Invalid pixels (-1) neither vote nor change.  Passes read only
// the previous pass's map.
//
// Layout: one wavefront per 8 x 8 pixel tile.  The tile's votes plus a kLMax
// apron on every side (42 x 42 int16) and the horizontal arms of the tile
// columns over the apron rows go to LDS; every lane then counts its own
// region into its own D counters (16-bit, lane-interleaved so that the 64
// lanes' counters of one disparity are 128 contiguous bytes: no bank
// conflicts whatever the disparities).  Runs of equal votes along a segment
// are added as one count.  All counts are integers, so the result does not
// depend on the order of the additions.
#include "dco_device.h"

namespace {

constexpr int kVT = 8;                // tile side
constexpr int kVR = kVT + 2 * kLMax;  // staged side
constexpr int kVStride = kVR + 2;

struct VoteLds {
    int16_t d[kVR][kVStride];      // votes of the staged region (-1: none)
    uint8_t l[kVR][kVT], r[kVR][kVT];  // horizontal arms of the tile columns
};

// din: H x W int16; valid (first pass only, else null): H x W uint8; a vote
// outside [0, D) counts as invalid.  dout: H x W int16, -1 where invalid.
__global__ __launch_bounds__(64) void k_vote(const int16_t* __restrict__ din,
                                             const uint8_t* __restrict__ valid,
                                             const uint32_t* __restrict__ arms, int W, int H,
                                             int D, int16_t* __restrict__ dout) {
    __shared__ VoteLds S;
    extern __shared__ __align__(16) uint16_t hist[];  // [D][64]
    const int lane = threadIdx.x, tx = lane & (kVT - 1), ty = lane / kVT;
    const int x0 = blockIdx.x * kVT, y0 = blockIdx.y * kVT;
    for (int i = lane; i < kVR * kVR; i += 64) {
        const int ry = i / kVR, rx = i - ry * kVR;
        const int x = x0 - kLMax + rx, y = y0 - kLMax + ry;
        int v = -1;
        if (x >= 0 && x < W && y >= 0 && y < H) {
            const size_t q = (size_t)y * W + x;
            const int dv = din[q];
            if ((valid == nullptr || valid[q]) && dv >= 0 && dv < D) v = dv;
        }
        S.d[ry][rx] = (int16_t)v;
    }
    for (int i = lane; i < kVR * kVT; i += 64) {
        const int ry = i / kVT, cx = i - ry * kVT;
        const int x = x0 + cx, y = y0 - kLMax + ry;
        const uint32_t a = x < W && y >= 0 && y < H ? arms[(size_t)y * W + x] : 0u;
        S.l[ry][cx] = (uint8_t)(a & 0xff);
        S.r[ry][cx] = (uint8_t)((a >> 8) & 0xff);
    }
    for (int i = lane; i < D * 8; i += 64) reinterpret_cast<uint4*>(hist)[i] = make_uint4(0, 0, 0, 0);
    __syncthreads();

    const int x = x0 + tx, y = y0 + ty;
    const bool in = x < W && y < H;
    const int mine = S.d[ty + kLMax][tx + kLMax];
    const uint32_t a = in ? arms[(size_t)y * W + x] : 0u;
    const int u = (a >> 16) & 0xff, dn = a >> 24;
    int cur = -1, run = 0;
    for (int k = -kLMax; k <= kLMax; ++k) {
        const bool rowin = mine >= 0 && k >= -u && k <= dn;
        if (!__any(rowin)) continue;  // uniform
        const int ry = ty + kLMax + k;
        const int lo = rowin ? -(int)S.l[ry][tx] : 1, hi = rowin ? (int)S.r[ry][tx] : 0;
        const int16_t* row = &S.d[ry][tx + kLMax];
#pragma unroll
        for (int j = -kLMax; j <= kLMax; ++j) {
            const int v = row[j];
            const bool take = j >= lo && j <= hi && v >= 0;
            if (take && v != cur) {
                if (run > 0) hist[cur * 64 + lane] += (uint16_t)run;
                cur = v;
                run = 0;
            }
            run += take ? 1 : 0;
        }
    }
    if (run > 0) hist[cur * 64 + lane] += (uint16_t)run;
    int best = 0, bc = -1;
    if (mine >= 0)
        for (int d = 0; d < D; ++d) {
            const int c = hist[d * 64 + lane];
            if (c > bc) {
                bc = c;
                best = d;
            }
        }
    if (in) dout[(size_t)y * W + x] = (int16_t)(mine >= 0 ? best : -1);
}

// Output of a voted map: disp = dv + the parabola offset at dv (Eq. 3's
// sub-pixel step on the aggregated costs) and valid = 1 where dv is in
// [0, D) (and valid_in, when given, is set); else disp = 0, valid = 0.
// valid may alias valid_in; dv_out (optional) gets dv, or -1 where invalid.
__global__ __launch_bounds__(256) void k_vote_finish(const int16_t* dv, const uint8_t* valid_in,
                                                     const float* __restrict__ agg, int P, int D,
                                                     int subpixel, float* __restrict__ disp,
                                                     uint8_t* valid, int16_t* dv_out) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= P) return;
    const int d = dv[i];
    const bool ok = (valid_in == nullptr || valid_in[i]) && d >= 0 && d < D;
    float out = 0.0f;
    if (ok) {
        float del = 0.0f;
        if (subpixel && d > 0 && d < D - 1)
            del = dco::subpixel_delta(agg[(size_t)(d - 1) * P + i], agg[(size_t)d * P + i],
                                      agg[(size_t)(d + 1) * P + i], d, D);
        out = (float)d + del;
    }
    disp[i] = out;
    valid[i] = (uint8_t)ok;
    if (dv_out) dv_out[i] = (int16_t)(ok ? d : -1);
}

}  // namespace

size_t vote_lds_bytes(int D) { return (size_t)D * 64 * sizeof(uint16_t); }

hipError_t launch_vote(const int16_t* dL, const uint8_t* valid, const uint32_t* arms, int W, int H,
                       int D, int iters, int16_t* buf0, int16_t* buf1, const int16_t** result,
                       hipStream_t st) {
    const dim3 grid((W + kVT - 1) / kVT, (H + kVT - 1) / kVT);
    const int16_t* src = dL;
    const uint8_t* mask = valid;
    int16_t* bufs[2] = {buf0, buf1};
    for (int it = 0; it < iters; ++it) {
        int16_t* dst = bufs[it & 1];
        hipLaunchKernelGGL(k_vote, grid, dim3(64), vote_lds_bytes(D), st, src, mask, arms, W, H,
                           D, dst);
        src = dst;
        mask = nullptr;
    }
    *result = src;
    return hipGetLastError();
}

hipError_t launch_vote_finish(const int16_t* dv, const uint8_t* valid_in, const float* agg, int W,
                              int H, int D, int subpixel, float* disp, uint8_t* valid,
                              int16_t* dv_out, hipStream_t st) {
    const int P = W * H;
    hipLaunchKernelGGL(k_vote_finish, dim3((P + 255) / 256), dim3(256), 0, st, dv, valid_in, agg,
                       P, D, subpixel, disp, valid, dv_out);
    return hipGetLastError();
}
