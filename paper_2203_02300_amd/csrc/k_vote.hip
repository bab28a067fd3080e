// k_vote.hip -- disparity refinement by region vote (Eq. 4, Sec. 4.3).
//
// One pass: every valid pixel p takes the disparity with the most votes in
// its stage-1 cross region N_p (for each y' on p's vertical arm, the pixels
// of (x, y')'s horizontal segment); equal counts go to the smallest
// disparity.  Invalid pixels (-1) neither vote nor change.  Passes read only
// the previous pass's map.
//
// Layout: one workgroup of eight wavefronts per 16 x 32 pixel tile (16
// columns, 32 rows), one thread per pixel.  The tile's votes plus a kLMax
// apron on every side (66 rows x 50 columns of int16) and the horizontal arms
// of the tile columns over the apron rows go to LDS, and each staged row is
// run-length coded once (runs of equal votes: start column, value, and the
// run of each column).  A pixel's region is the union of the horizontal
// segments of the rows on its vertical arm, and the segment of (column, row)
// is the same for every pixel whose arm covers that row; so the votes are
// counted once per segment: for a window of kVBins disparities at a time,
// each of the 66 x 16 segments adds, for every run it meets, the overlap
// length to its own counters; the counters are then prefix-summed down each
// tile column, and a pixel reads its counts as the difference of two prefix
// rows (the ends of its vertical arm).  Counters are 16-bit, two per 32-bit
// word (a count is at most 67 rows x 35 columns, so packed sums and
// differences never carry between the halves).
// The windows step from the smallest to the largest vote staged for the
// tile; a strict running maximum keeps the smallest disparity among equal
// counts.  All counts are integers, so the result does not depend on the
// order of the additions.
#include "dco_device.h"

namespace {

constexpr int kVTW = 16, kVTH = 32;         // tile width and height
constexpr int kVThreads = kVTW * kVTH;      // one thread per tile pixel
constexpr int kVWaves = kVThreads / 64;
constexpr int kVRW = kVTW + 2 * kLMax;      // staged width
constexpr int kVRH = kVTH + 2 * kLMax;      // staged height
constexpr int kVStride = kVRW + 2;

constexpr int kVBins = 16;               // disparities per counter window
constexpr int kVWords = kVBins / 2;      // two 16-bit counters per word
constexpr int kVWordStride = kVWords + 1;  // per tile column (odd: no bank conflicts)
constexpr int kVSegs = kVRH * kVTW;      // segments: staged rows x tile columns
constexpr int kVStage = (kVRW * kVRH + kVThreads - 1) / kVThreads;
constexpr int kVArms = (kVRH * kVTW + kVThreads - 1) / kVThreads;
static_assert(kVBins % 2 == 0 && (kVRH + 1) * 35 < 65536, "packed 16-bit counters");
static_assert((kVTW & (kVTW - 1)) == 0, "tile width a power of two");

struct VoteLds {
    // cnt[r][c][k]: for tile column c and the window's bins 2k, 2k + 1, the
    // votes over the segments of staged rows 0 .. r - 1 (row 0: none)
    uint32_t cnt[kVRH + 1][kVTW][kVWordStride];
    int16_t d[kVRH][kVStride];    // votes of the staged region (-1: none)
    int16_t rv[kVRH][kVRW];       // value of run k of each staged row
    uint8_t rs[kVRH][kVRW + 2];   // run of each column
    uint8_t st[kVRH][kVRW + 2];   // start column of run k; st[nruns] = kVRW
    uint8_t l[kVRH][kVTW], r[kVRH][kVTW];  // horizontal arms of the tile columns
    int lo[kVWaves], hi[kVWaves];      // vote range seen by each wavefront
};

__device__ inline int wave_min(int v) {
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ inline int wave_max(int v) {
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

// din: H x W int16; valid (first pass only, else null): H x W uint8; a vote
// outside [0, D) counts as invalid.  dout: H x W int16, -1 where invalid.
__global__ __launch_bounds__(kVThreads) void k_vote(const int16_t* __restrict__ din,
                                                    const uint8_t* __restrict__ valid,
                                                    const uint32_t* __restrict__ arms, int W,
                                                    int H, int D, int16_t* __restrict__ dout) {
    __shared__ __align__(16) VoteLds S;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int tx = tid & (kVTW - 1), ty = tid / kVTW;
    const int x0 = blockIdx.x * kVTW, y0 = blockIdx.y * kVTH;
    {   // stage the votes: every load issued before any is used (clamped addresses)
        int dv[kVStage];
        bool ok[kVStage];
#pragma unroll
        for (int t = 0; t < kVStage; ++t) {
            const int i = min(tid + kVThreads * t, kVRW * kVRH - 1);
            const int ry = i / kVRW, rx = i - ry * kVRW;
            const int x = x0 - kLMax + rx, y = y0 - kLMax + ry;
            ok[t] = x >= 0 && x < W && y >= 0 && y < H;
            const size_t q = (size_t)min(max(y, 0), H - 1) * W + min(max(x, 0), W - 1);
            dv[t] = din[q];
            if (valid) ok[t] = ok[t] && valid[q] != 0;
        }
        int lo = D, hi = -1;
#pragma unroll
        for (int t = 0; t < kVStage; ++t) {
            const int i = tid + kVThreads * t;
            const int v = ok[t] && dv[t] >= 0 && dv[t] < D ? dv[t] : -1;
            if (i < kVRW * kVRH) {
                const int ry = i / kVRW;
                S.d[ry][i - ry * kVRW] = (int16_t)v;
                if (v >= 0) {
                    lo = min(lo, v);
                    hi = max(hi, v);
                }
            }
        }
        lo = wave_min(lo);
        hi = wave_max(hi);
        if (lane == 0) {
            S.lo[w] = lo;
            S.hi[w] = hi;
        }
    }
    {   // horizontal arms of the tile columns (loads issued together, clamped)
        uint32_t av[kVArms];
#pragma unroll
        for (int t = 0; t < kVArms; ++t) {
            const int i = min(tid + kVThreads * t, kVRH * kVTW - 1);
            const int ry = i / kVTW, cx = i - ry * kVTW;
            const int x = min(x0 + cx, W - 1), y = min(max(y0 - kLMax + ry, 0), H - 1);
            av[t] = arms[(size_t)y * W + x];
        }
#pragma unroll
        for (int t = 0; t < kVArms; ++t) {
            const int i = tid + kVThreads * t;
            const int ry = i / kVTW, cx = i - ry * kVTW;
            const int x = x0 + cx, y = y0 - kLMax + ry;
            const uint32_t a = x < W && y >= 0 && y < H ? av[t] : 0u;
            if (i < kVRH * kVTW) {
                S.l[ry][cx] = (uint8_t)min(a & 0xff, (uint32_t)kLMax);
                S.r[ry][cx] = (uint8_t)min((a >> 8) & 0xff, (uint32_t)kLMax);
            }
        }
    }
    __syncthreads();
    int vlo = S.lo[0], vhi = S.hi[0];  // the tile's vote range (empty when vhi < vlo)
#pragma unroll
    for (int k = 1; k < kVWaves; ++k) {
        vlo = min(vlo, S.lo[k]);
        vhi = max(vhi, S.hi[k]);
    }
    if (tid < kVRH) {  // run-length code staged row `tid`
        int n = 0, prev = 0;
#pragma unroll 5
        for (int c = 0; c < kVRW; ++c) {
            const int v = S.d[tid][c];
            if (c == 0 || v != prev) {
                S.st[tid][n] = (uint8_t)c;
                S.rv[tid][n] = (int16_t)v;
                ++n;
                prev = v;
            }
            S.rs[tid][c] = (uint8_t)(n - 1);
        }
        S.st[tid][n] = (uint8_t)kVRW;
    }
    __syncthreads();

    const int x = x0 + tx, y = y0 + ty;
    const bool in = x < W && y < H;
    const int mine = S.d[ty + kLMax][tx + kLMax];
    const uint32_t a = in ? arms[(size_t)y * W + x] : 0u;
    const int u = min((int)((a >> 16) & 0xff), kLMax), dn = min((int)(a >> 24), kLMax);
    // this pixel's vertical arm in staged rows: prefix rows r0 (before it)
    // and r1 (through its last row)
    const int r0 = ty + kLMax - u, r1 = ty + kLMax + dn + 1;
    int best = 0, bc = -1;
    for (int base = vlo; base <= vhi; base += kVBins) {  // uniform
        const int nb = min(kVBins, vhi - base + 1);      // bins past vhi get no votes
        // 1. each segment's counts (one thread per segment; row 0 is zero)
        for (int i = tid; i < kVTW * kVWords; i += kVThreads)
            S.cnt[0][i / kVWords][i % kVWords] = 0u;
        for (int sg = tid; sg < kVSegs; sg += kVThreads) {
            const int ry = sg / kVTW, cx = sg - ry * kVTW;
            uint32_t* c = S.cnt[ry + 1][cx];
#pragma unroll
            for (int k = 0; k < kVWords; ++k) c[k] = 0u;
            uint16_t* c16 = reinterpret_cast<uint16_t*>(c);
            const int lo = cx + kLMax - S.l[ry][cx], hi = cx + kLMax + S.r[ry][cx];
            const int k1 = S.rs[ry][hi];
            for (int j = S.rs[ry][lo]; j <= k1; ++j) {
                const int b = S.rv[ry][j] - base;
                if (b >= 0 && b < nb) {
                    const int s0 = max((int)S.st[ry][j], lo);
                    const int s1 = min((int)S.st[ry][j + 1] - 1, hi);
                    c16[b] = (uint16_t)(c16[b] + (s1 - s0 + 1));
                }
            }
        }
        __syncthreads();
        // 2. prefix sums down each tile column, a (column, word) per thread
        for (int i = tid; i < kVTW * kVWords; i += kVThreads) {
            const int cx = i / kVWords, k = i % kVWords;
            uint32_t run = 0u;
#pragma unroll 11
            for (int ry = 1; ry <= kVRH; ++ry) {
                run += S.cnt[ry][cx][k];
                S.cnt[ry][cx][k] = run;
            }
        }
        __syncthreads();
        // 3. this pixel's counts: two prefix rows per word
        if (mine >= 0) {
            for (int k = 0; 2 * k < nb; ++k) {
                const uint32_t w = S.cnt[r1][tx][k] - S.cnt[r0][tx][k];
                const int c0 = (int)(w & 0xffffu), c1 = (int)(w >> 16);
                if (c0 > bc) {
                    bc = c0;
                    best = base + 2 * k;
                }
                if (2 * k + 1 < nb && c1 > bc) {
                    bc = c1;
                    best = base + 2 * k + 1;
                }
            }
        }
        __syncthreads();
    }
    if (in) dout[(size_t)y * W + x] = (int16_t)(mine >= 0 ? best : -1);
}

// Output of a voted map: disp = dv + the parabola offset at dv (Eq. 3's
// sub-pixel step on the aggregated costs) and valid = 1 where dv is in
// [0, D) (and valid_in, when given, is set); else disp = 0, valid = 0.
// valid may alias valid_in; dv_out (optional) gets dv, or -1 where invalid.
__global__ __launch_bounds__(256) void k_vote_finish(const int16_t* dv, const uint8_t* valid_in,
                                                     const float* __restrict__ agg, int paired,
                                                     int P, int D, int subpixel,
                                                     float* __restrict__ disp, uint8_t* valid,
                                                     int16_t* dv_out) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= P) return;
    const int d = dv[i];
    const bool ok = (valid_in == nullptr || valid_in[i]) && d >= 0 && d < D;
    float out = 0.0f;
    if (ok) {
        float del = 0.0f;
        if (subpixel && d > 0 && d < D - 1) {
            if (paired)
                del = dco::subpixel_delta(dco::paired_at(agg, P, D, d - 1, i),
                                          dco::paired_at(agg, P, D, d, i),
                                          dco::paired_at(agg, P, D, d + 1, i), d, D);
            else
                del = dco::subpixel_delta(agg[(size_t)(d - 1) * P + i], agg[(size_t)d * P + i],
                                          agg[(size_t)(d + 1) * P + i], d, D);
        }
        out = (float)d + del;
    }
    disp[i] = out;
    valid[i] = (uint8_t)ok;
    if (dv_out) dv_out[i] = (int16_t)(ok ? d : -1);
}

}  // namespace

hipError_t launch_vote(const int16_t* dL, const uint8_t* valid, const uint32_t* arms, int W, int H,
                       int D, int iters, int16_t* buf0, int16_t* buf1, const int16_t** result,
                       hipStream_t st) {
    const dim3 grid((W + kVTW - 1) / kVTW, (H + kVTH - 1) / kVTH);
    const int16_t* src = dL;
    const uint8_t* mask = valid;
    int16_t* bufs[2] = {buf0, buf1};
    for (int it = 0; it < iters; ++it) {
        int16_t* dst = bufs[it & 1];
        hipLaunchKernelGGL(k_vote, grid, dim3(kVThreads), 0, st, src, mask, arms, W, H, D, dst);
        src = dst;
        mask = nullptr;
    }
    *result = src;
    return hipGetLastError();
}

hipError_t launch_vote_finish(const int16_t* dv, const uint8_t* valid_in, const float* agg,
                              bool paired, int W, int H, int D, int subpixel, float* disp,
                              uint8_t* valid, int16_t* dv_out, hipStream_t st) {
    const int P = W * H;
    hipLaunchKernelGGL(k_vote_finish, dim3((P + 255) / 256), dim3(256), 0, st, dv, valid_in, agg,
                       (int)paired, P, D, subpixel, disp, valid, dv_out);
    return hipGetLastError();
}
