// k_aggregate.hip -- aggregation over the adaptive cross region (Eq. 2),
// applied as two stages (horizontal-then-vertical, then
// vertical-then-horizontal), in exact integer arithmetic.
//
// Work decomposition: one workgroup = one disparity slice x one column strip.
// The strip's 256 threads own 256 consecutive columns: 2*kLMax apron columns
// on each side and kStripOut output columns in the middle.  The workgroup
// streams down the image rows, so the vertical apron costs nothing; the
// horizontal apron is re-read from L2.
//
// Per row the four range sums are
//   H1: E1 = row range sum of q             (block prefix scan + 2 LDS reads)
//   V1: S1 = column range sum of E1         (per-column ring of prefix sums)
//       a1 = floor((S1 + N1/2) / N1)        (exact multiply-shift division)
//   V2: E2 = column range sum of a1         (second per-column ring)
//   H2: S2 = row range sum of E2            (block prefix scan + 2 LDS reads)
//       out = RN(S2 / N2) * 2^-20           (reciprocal + one FMA correction)
// Each ring keeps the last kRing column-prefix rows of one column; only the
// thread owning that column touches it, so ring traffic needs no barrier.
// Rows are handled in chunks of kRowChunk so that the two block scans of a
// chunk cost four barriers in total.  The pipeline lags: V1 finalises row
// y - kLMax and H2 row y - 2 kLMax - 1 while H1 consumes row y.
//
// Every sum is an integer (differences of prefix sums taken mod 2^32 are exact
// because every true range sum is below 2^31), so the result does not depend
// on summation order and equals the oracle bit for bit.
//
// The same kernel body also serves the one-call matcher: with kFused the raw
// cost q of Eq. 1 is computed on the fly from the images and census codes
// instead of being read from a cost volume.
#include "dco_internal.h"

namespace {

constexpr int kRingCols = kStripThreads - 2 * kLMax;  // ring columns used: 222
constexpr int kRingStride = 224;
constexpr int kPB = kStripThreads + 4;                // prefix row stride (P[-1] at 0)

// Inclusive prefix sum over a wavefront of 64 lanes with DPP row shifts and
// the row broadcasts of the gfx9 family (wrap-around uint32 arithmetic).
__device__ inline uint32_t wave_incl_scan(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);  // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return v;
}

// Inclusive scan of K rows at once across the 256 threads of the block.
// Writes P(t) to pb[k][t + 1] and 0 to pb[k][0].  Two barriers; on return
// every thread sees every row's prefix.
template <int K>
__device__ inline void block_scan_rows(uint32_t (&v)[K], uint32_t (*pb)[kPB],
                                       uint32_t (*ws)[4]) {
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        v[k] = wave_incl_scan(v[k]);
        if (lane == 63) ws[k][w] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const uint4 s = *reinterpret_cast<const uint4*>(ws[k]);
        uint32_t off = 0;
        if (w > 0) off += s.x;
        if (w > 1) off += s.y;
        if (w > 2) off += s.z;
        pb[k][t + 1] = v[k] + off;
        if (t == 0) pb[k][0] = 0;
    }
    __syncthreads();
}

__device__ inline int ring_slot(int slot_y, int back) {  // slot of row (y - back), 0 <= back < kRing
    int s = slot_y - back;
    return s < 0 ? s + kRing : s;
}

// RN((float)s / N) given (N, RN(1/N)).  Exact: q0 = RN(s * y) is within two
// ulps of s/N, r = s - q0 * N is then exact, and s/N is never a float
// midpoint for integer N, so RN(q0 + r * y) = RN(s / N).
__device__ inline float div_rn(uint32_t s, float2 nv) {
    const float a = (float)s;
    const float q0 = a * nv.y;
    const float r = __builtin_fmaf(-q0, nv.x, a);
    return __builtin_fmaf(r, nv.y, q0);
}

__device__ inline uint32_t div_half_up(uint32_t s, DivInt dv) {
    const uint64_t n = (uint64_t)(s + (dv.half_sh & 0xffffu));
    return (uint32_t)((n * dv.m) >> (dv.half_sh >> 16));
}

// Work item of block b, remapped so that the blocks one XCD runs (round-robin
// block -> XCD dispatch) get consecutive items: neighbouring strips of the
// same slice share their apron columns in that XCD's L2.
__device__ inline int xcd_work_item(int b, int n) {
    const int xcd = b & 7, i = b >> 3;
    const int per = n >> 3, rem = n & 7;
    return xcd < rem ? xcd * (per + 1) + i : rem * (per + 1) + (xcd - rem) * per + i;
}

struct AggArgs {
    const float* cost;         // staged: D x H x W raw costs
    const uint32_t* rgbL;      // fused: packed RGB of both views
    const uint32_t* rgbR;
    const uint64_t* cenL;      // fused: census codes
    const uint64_t* cenR;
    const float* tabA;         // fused: Eq. 1 tables
    const float* tabC;
    const float* alpha;
    const float* beta;
    const uint32_t* arms;      // packed arms of the reference view
    const DivInt* div1;
    const float2* div2;
    float* out;                // D x H x W
    int W, H, D, nstrips, ref, L1;
};

template <int ITERS, bool kFused>
__global__ __launch_bounds__(kStripThreads, 2) void k_agg_stream(AggArgs A) {
    __shared__ uint32_t ring1[kRing][kRingStride];
    __shared__ uint32_t ring2[ITERS == 2 ? kRing : 1][kRingStride];
    __shared__ uint32_t pbuf[2][kRowChunk][kPB];
    __shared__ __attribute__((aligned(16))) uint32_t wsum[2][kRowChunk][4];
    __shared__ float s_tabA[kFused ? 768 : 1];
    __shared__ float s_tabC[kFused ? 65 : 1];
    __shared__ float s_ab[kFused ? 2 * (kLMax + 1) : 1];

    const int W = A.W, H = A.H;
    const int t = threadIdx.x;
    const int work = xcd_work_item(blockIdx.x, A.nstrips * A.D);
    const int d = work / A.nstrips, strip = work - d * A.nstrips;
    const int x0 = strip * kStripOut;
    const int c = x0 - 2 * kLMax + t;
    const bool in_img = c >= 0 && c < W;
    const int j = t - kLMax;
    const bool ring_thr = j >= 0 && j < kRingCols && in_img;
    const bool out_thr = t >= 2 * kLMax && t < 2 * kLMax + kStripOut && c < W;
    const size_t slice = (size_t)W * H;
    float* out = A.out + (size_t)d * slice;
    const float* cost = kFused ? nullptr : A.cost + (size_t)d * slice;

    if (kFused) {
        for (int i = t; i < 766; i += kStripThreads) s_tabA[i] = A.tabA[i];
        if (t < 65) s_tabC[t] = A.tabC[t];
        if (t <= A.L1) {
            s_ab[t] = A.alpha[t];
            s_ab[kLMax + 1 + t] = A.beta[t];
        }
    }
    if (j >= 0 && j < kRingCols) {
        ring1[kRing - 1][j] = 0;  // column prefix of row -1
        if (ITERS == 2) ring2[kRing - 1][j] = 0;
    }
    // partner column for the fused raw cost
    const int cp = A.ref == 0 ? c - d : c + d;
    const bool par_ok = in_img && cp >= 0 && cp < W;
    const uint32_t* Iref = A.ref == 0 ? A.rgbL : A.rgbR;
    const uint32_t* Ipar = A.ref == 0 ? A.rgbR : A.rgbL;
    const uint64_t* Cref = A.ref == 0 ? A.cenL : A.cenR;
    const uint64_t* Cpar = A.ref == 0 ? A.cenR : A.cenL;
    __syncthreads();

    uint32_t cp1 = 0, cp2 = 0;
    int slot = 0;  // ring slot of row y
    const int nsteps = ITERS == 2 ? H + 2 * kLMax + 1 : H + kLMax;
    for (int yc = 0; yc < nsteps; yc += kRowChunk) {
        uint32_t q[kRowChunk], armA[kRowChunk], armB[kRowChunk], armC[kRowChunk];
        DivInt dv1[kRowChunk];
        float2 dv2[kRowChunk];
#pragma unroll
        for (int k = 0; k < kRowChunk; ++k) {
            const int y = yc + k, y1 = y - kLMax, y2 = y - 2 * kLMax - 1;
            q[k] = 0;
            armA[k] = 0;
            armB[k] = 0;
            armC[k] = 0;
            dv1[k] = DivInt{0, 0};
            dv2[k] = make_float2(1.f, 1.f);
            if (in_img && y < H) {
                const size_t pix = (size_t)y * W + c;
                armA[k] = A.arms[pix];
                if (kFused) {
                    if (par_ok) {
                        const uint32_t a = armA[k];
                        const int lmin = min(min((int)(a & 0xff), (int)((a >> 8) & 0xff)),
                                             min((int)((a >> 16) & 0xff), (int)(a >> 24)));
                        const size_t ppix = (size_t)y * W + cp;
                        const uint32_t s = __builtin_amdgcn_sad_u8(Iref[pix], Ipar[ppix], 0u);
                        const int h = __popcll(Cref[pix] ^ Cpar[ppix]);
                        const float qa = __builtin_rintf(s_ab[lmin] * s_tabA[s]);
                        const float qc = __builtin_rintf(s_ab[kLMax + 1 + lmin] * s_tabC[h]);
                        q[k] = (uint32_t)qa + (uint32_t)qc;
                    } else {
                        q[k] = 1u << 20;
                    }
                } else {
                    q[k] = (uint32_t)(cost[pix] * 1048576.0f);
                }
            }
            if (in_img && y1 >= 0 && y1 < H) {
                const size_t pix = (size_t)y1 * W + c;
                armB[k] = A.arms[pix];
                dv1[k] = A.div1[pix];
                if (ITERS == 1) dv2[k] = A.div2[pix];
            }
            if (ITERS == 2 && in_img && y2 >= 0 && y2 < H) {
                const size_t pix = (size_t)y2 * W + c;
                armC[k] = A.arms[pix];
                dv2[k] = A.div2[pix];
            }
        }
        block_scan_rows<kRowChunk>(q, pbuf[0], wsum[0]);

        uint32_t e2[kRowChunk];
#pragma unroll
        for (int k = 0; k < kRowChunk; ++k) {
            const int y = yc + k, y1 = y - kLMax, y2 = y - 2 * kLMax - 1;
            e2[k] = 0;
            if (ring_thr) {
                if (y < H) {  // H1: E1 of row y, push its column prefix
                    const int l = armA[k] & 0xff, r = (armA[k] >> 8) & 0xff;
                    const uint32_t e1 = pbuf[0][k][t + r + 1] - pbuf[0][k][t - l];
                    cp1 += e1;
                    ring1[slot][j] = cp1;
                }
                if (ITERS == 2 && y2 >= 0 && y2 < H) {  // V2: E2 of row y2 (rows y2-u-1 .. y2+dn)
                    // row y2 + dn is 2*kLMax+1-dn rows behind y; row y2-u-1 is kRing+u
                    // rows behind y, i.e. in the slot of row y - u
                    const int u = (armC[k] >> 16) & 0xff, dn = armC[k] >> 24;
                    e2[k] = ring2[ring_slot(slot, 2 * kLMax + 1 - dn)][j] -
                            ring2[ring_slot(slot, u)][j];
                }
                if (y1 >= 0 && y1 < H) {  // V1: S1 of row y1 (rows y1-u-1 .. y1+dn)
                    const int u = (armB[k] >> 16) & 0xff, dn = armB[k] >> 24;
                    const uint32_t s1 = ring1[ring_slot(slot, kLMax - dn)][j] -
                                        ring1[ring_slot(slot, kLMax + u + 1)][j];
                    if (ITERS == 2) {
                        cp2 += div_half_up(s1, dv1[k]);
                        ring2[ring_slot(slot, kLMax)][j] = cp2;
                    } else if (out_thr) {
                        out[(size_t)y1 * W + c] = div_rn(s1, dv2[k]) * 0x1p-20f;
                    }
                }
            }
            slot = slot + 1 == kRing ? 0 : slot + 1;
        }
        if (ITERS == 2) {
            block_scan_rows<kRowChunk>(e2, pbuf[1], wsum[1]);
#pragma unroll
            for (int k = 0; k < kRowChunk; ++k) {
                const int y2 = yc + k - 2 * kLMax - 1;
                if (out_thr && y2 >= 0 && y2 < H) {  // H2: S2 of row y2
                    const int l = armC[k] & 0xff, r = (armC[k] >> 8) & 0xff;
                    const uint32_t s2 = pbuf[1][k][t + r + 1] - pbuf[1][k][t - l];
                    out[(size_t)y2 * W + c] = div_rn(s2, dv2[k]) * 0x1p-20f;
                }
            }
        }
    }
}

template <int ITERS, bool kFused>
hipError_t launch_stream(const AggArgs& a, hipStream_t st) {
    const int nblk = a.nstrips * a.D;
    hipLaunchKernelGGL((k_agg_stream<ITERS, kFused>), dim3(nblk), dim3(kStripThreads), 0, st, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_aggregate(const float* cost, const uint32_t* arms, const DivInt* div1,
                            const float2* div2, int W, int H, int D, int iters, float* out,
                            hipStream_t st) {
    AggArgs a{};
    a.cost = cost;
    a.arms = arms;
    a.div1 = div1;
    a.div2 = div2;
    a.out = out;
    a.W = W;
    a.H = H;
    a.D = D;
    a.nstrips = (W + kStripOut - 1) / kStripOut;
    return iters == 1 ? launch_stream<1, false>(a, st) : launch_stream<2, false>(a, st);
}

hipError_t launch_cost_aggregate(int ref, const uint32_t* rgbL, const uint32_t* rgbR,
                                 const uint64_t* cenL, const uint64_t* cenR,
                                 const uint32_t* arms, const DivInt* div1, const float2* div2,
                                 int W, int H, int D, int iters, const float* tabA,
                                 const float* tabC, const float* alpha, const float* beta,
                                 int L1, float* out, hipStream_t st) {
    AggArgs a{};
    a.rgbL = rgbL;
    a.rgbR = rgbR;
    a.cenL = cenL;
    a.cenR = cenR;
    a.tabA = tabA;
    a.tabC = tabC;
    a.alpha = alpha;
    a.beta = beta;
    a.arms = arms;
    a.div1 = div1;
    a.div2 = div2;
    a.out = out;
    a.W = W;
    a.H = H;
    a.D = D;
    a.ref = ref;
    a.L1 = L1;
    a.nstrips = (W + kStripOut - 1) / kStripOut;
    return iters == 1 ? launch_stream<1, true>(a, st) : launch_stream<2, true>(a, st);
}
