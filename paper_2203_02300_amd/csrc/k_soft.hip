// k_soft.hip -- differentiable soft-argmin form of the matcher (left view).
//
// Forward, per pair b, disparity d, pixel p (all float):
//   c(p,d)  = alpha_p (1 - exp(-(s/3)/lambda_AD)) + (1 - alpha_p)(1 - exp(-h/lambda_census))
//             (Eq. 1; c = 1 where the partner pixel x - d is outside the image)
//   E1 = row range sum of c       a1 = (column range sum of E1) / N1     (Eq. 2, stage 1)
//   E2 = column range sum of a1   A2 = (row range sum of E2) / N2         (Eq. 2, stage 2)
//   dhat = sum_d d softmax_d(-A2 / T),  lse = log sum_d exp(-A2 / T)
// Every range sum is a difference of two FP64 prefix sums (along the row, or
// running down the column), so it is within one FP32 rounding of the exact
// sum of its FP32 terms.  Every sum runs in a fixed order, so results are
// bit-reproducible.
//
// Backward, given g = dLoss/d dhat:
//   G_A2  = g w (dhat - d) / T,   dLoss/dT = sum g w (d - dhat) A2 / T^2
// then the adjoint of each range sum: an output that summed a range hands its
// adjoint back to every pixel of that range.  The first row adjoint scatters
// each G(x) into a 64-bit fixed-point difference array over the row (integer
// adds, so their order does not matter); column adjoints are FP64 difference
// arrays streamed down each column by one thread.  The last row adjoint is
// never formed: with
// E1 = H c,  sum_p (H^T G)(p) dc/dlambda(p) = sum_x G(x) (H dc/dlambda)(x),
// so the row range sums of the two cost derivatives are dotted with G:
//   dLoss/dlambda_AD     = sum G_E1 . H (alpha d(1 - exp(-(s/3)/lambda_AD))/dlambda_AD)
//   dLoss/dlambda_census = sum G_E1 . H ((1 - alpha) d(1 - exp(-h/lambda_census))/dlambda_census)
// with fixed-order two-level reductions.  The only atomics are LDS adds whose
// result does not depend on their order (integers), or that one thread makes
// to its own column in program order.
//
// Layout: volumes are B x D x H x W float in handle scratch; arms and the
// packed pixels (census, RGB, L_min) are per pair B x H x W.  Row passes run
// one wavefront per image row with its FP64 prefix in LDS; column passes one
// thread per column, streaming down the rows with a ring of FP64 sums in LDS.
#include <type_traits>

#include "dco_internal.h"

namespace {


struct SoftGeom {
    const uint32_t* arms;  // B x H x W packed arms of the left view
    const float* n1;       // B x H x W stage-1 region counts
    const float* n2;       // B x H x W stage-2 region counts
    int B, W, H, D;
};

__device__ inline int arm(uint32_t a, int k) { return (a >> (8 * k)) & 0xff; }

// Tables of Eq. 1 for the current theta, and their lambda derivatives:
// tab[0..765] = 1 - exp(-(s/3)/lambda_AD),   tab[768..1533] = d/dlambda_AD
// tab[1536..1600] = 1 - exp(-h/lambda_c),    tab[1664..1728] = d/dlambda_c
__global__ void k_soft_tables(const float* __restrict__ theta, float* __restrict__ tab) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const float la = theta[0], lc = theta[1];
    if (i < 766) {
        const float x = (float)i / 3.0f;
        const float e = expf(-x / la);
        tab[i] = -expm1f(-x / la);
        tab[768 + i] = -e * x / (la * la);
    } else if (i >= 768 && i < 768 + 65) {
        const int h = i - 768;
        const float e = expf(-(float)h / lc);
        tab[1536 + h] = -expm1f(-(float)h / lc);
        tab[1664 + h] = -e * (float)h / (lc * lc);
    }
}

// Region pixel counts of the left view (as floats) for every pair: one
// block per 64 x 4 tile.  The row lengths l + r + 1 of the tile's columns
// over kLMax rows above and below, and the column lengths u + dn + 1 of the
// tile's rows over kLMax columns left and right, go to LDS (0 outside the
// image, where no arm reaches); each count is then a sum of LDS entries.
constexpr int kCntTW = 64, kCntTH = 4;
__global__ __launch_bounds__(256) void k_soft_counts(SoftGeom g, float* __restrict__ n1,
                                                     float* __restrict__ n2) {
    constexpr int CH = kCntTH + 2 * kLMax, RW = kCntTW + 2 * kLMax;
    __shared__ uint8_t hl[CH][kCntTW];  // l + r + 1 down each tile column
    __shared__ uint8_t vl[kCntTH][RW];  // u + dn + 1 along each tile row
    const int t = threadIdx.x, b = blockIdx.z;
    const int x0 = blockIdx.x * kCntTW, y0 = blockIdx.y * kCntTH;
    const uint32_t* A = g.arms + (size_t)b * g.W * g.H;
    for (int k = t; k < CH * kCntTW; k += 256) {
        const int r = k / kCntTW, c = k - r * kCntTW;
        const int x = x0 + c, y = y0 - kLMax + r;
        const bool in = x < g.W && y >= 0 && y < g.H;
        const uint32_t q = in ? A[(size_t)y * g.W + x] : 0u;
        hl[r][c] = in ? (uint8_t)(arm(q, 0) + arm(q, 1) + 1) : 0;
    }
    for (int k = t; k < kCntTH * RW; k += 256) {
        const int r = k / RW, c = k - r * RW;
        const int x = x0 - kLMax + c, y = y0 + r;
        const bool in = x >= 0 && x < g.W && y < g.H;
        const uint32_t q = in ? A[(size_t)y * g.W + x] : 0u;
        vl[r][c] = in ? (uint8_t)(arm(q, 2) + arm(q, 3) + 1) : 0;
    }
    __syncthreads();
    const int tx = t & (kCntTW - 1), ty = t / kCntTW;
    const int x = x0 + tx, y = y0 + ty;
    if (x >= g.W || y >= g.H) return;
    const uint32_t a = A[(size_t)y * g.W + x];
    int s1 = 0, s2 = 0;
    for (int k = -arm(a, 2); k <= arm(a, 3); ++k) s1 += hl[ty + kLMax + k][tx];
    for (int k = -arm(a, 0); k <= arm(a, 1); ++k) s2 += vl[ty][tx + kLMax + k];
    const size_t i = (size_t)b * g.W * g.H + (size_t)y * g.W + x;
    n1[i] = (float)s1;
    n2[i] = (float)s2;
}

// Eq. 1 tables of the current theta in LDS: the k_soft_tables layout, then
// alpha_L for L = 0 .. kLMax.
constexpr int kTabFloats = 1792;
constexpr size_t kTabLds = (kTabFloats + 32) * sizeof(float);

struct SoftImg {
    const uint4* pixL;   // B x H x W packed pixels: census lo, census hi,
    const uint4* pixR;   //   RGB, 8 L_min
    const float* alpha;  // alpha_L, L = 0..kLMax
    const float* tab;    // k_soft_tables output
};

__device__ inline void load_tables(const SoftImg& im, float* lds) {
    for (int i = threadIdx.x; i < kTabFloats; i += blockDim.x) lds[i] = im.tab[i];
    if (threadIdx.x <= kLMax) lds[kTabFloats + threadIdx.x] = im.alpha[threadIdx.x];
    __syncthreads();
}

// Raw cost c of Eq. 1 for reference pixel a and partner pixel b (and, with
// kDeriv, its lambda_AD and lambda_census derivatives); c = 1 and zero
// derivatives when the partner lies outside the image.
template <bool kDeriv>
__device__ inline void cost_px(uint4 a, uint4 b, bool inside, const float* tab, float& c,
                               float& dca, float& dcc) {
    const uint32_t s = __builtin_amdgcn_sad_u8(a.z, b.z, 0u);
    const int h = __popcll(((uint64_t)a.y << 32 | a.x) ^ ((uint64_t)b.y << 32 | b.x));
    const float al = tab[kTabFloats + (a.w >> 3)];
    const float v = al * tab[s] + (1.0f - al) * tab[1536 + h];
    c = inside ? v : 1.0f;
    if (kDeriv) {
        const float va = al * tab[768 + s], vc = (1.0f - al) * tab[1664 + h];
        dca = inside ? va : 0.0f;
        dcc = inside ? vc : 0.0f;
    }
}

// Row passes: one wavefront per image row, kRowWaves wavefronts per
// workgroup, each with its own LDS slice (no workgroup barriers after the
// table load) and kRowsPerWave rows in turn.  Row ids run over (b, y, d)
// with d fastest, so the rows that run together share one image row (its
// pixels, arms and counts stay in cache across the disparities).  Outside
// the prefix phase (which has its own layout, see prefix_row) lane `lane`
// handles columns lane + 64 k; loads are issued
// kRowBatch columns at a time with clamped (always valid) addresses.
constexpr int kRowWaves = 4;
constexpr int kRowsPerWave = 4;
constexpr int kRowBatch = 8;

// Runs body(nb, x0) over a row of W columns in batches of 64 NB columns
// (NB = decltype(nb)::value): batches of kMax while they fit, then of 2, then
// of 1 (the last may run past W; the body masks those lanes).  A row of 640
// columns takes one batch of 8 and one of 2, not two of 8.
template <int kMax = kRowBatch, typename Body>
__device__ inline void over_row(int W, Body body) {
    int x0 = 0;
    for (; x0 + 64 * kMax <= W; x0 += 64 * kMax) body(std::integral_constant<int, kMax>{}, x0);
    for (; x0 + 64 * 2 <= W; x0 += 64 * 2) body(std::integral_constant<int, 2>{}, x0);
    for (; x0 < W; x0 += 64) body(std::integral_constant<int, 1>{}, x0);
}

// Workgroup index in the row order of workgroup b of n: the workgroups one
// XCD runs (round-robin dispatch, b mod 8) take a contiguous run, so the
// workgroups that share an image row share that XCD's L2.
__device__ inline int xcd_block(int b, int n) {
    const int xcd = b & 7, i = b >> 3;
    const int per = n >> 3, rem = n & 7;
    return xcd < rem ? xcd * (per + 1) + i : rem * (per + 1) + (xcd - rem) * per + i;
}

__device__ inline void row_of(int rid, int D, int H, int& b, int& d, int& y) {
    d = rid % D;
    const int by = rid / D;
    y = by % H;
    b = by / H;
}

template <unsigned Ctrl, unsigned RowMask>
__device__ inline double dpp_f64(double v) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, Ctrl, RowMask,
                                                              0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), Ctrl,
                                                              RowMask, 0xf, false);
    return __builtin_bit_cast(double, (uint64_t)hi << 32 | lo);
}

__device__ inline double readlane_f64(double v, int l) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
    return __builtin_bit_cast(double, (uint64_t)hi << 32 | lo);
}

// FP64 inclusive scan across the wavefront (lane L gets v(0) + ... + v(L)):
// DPP row shifts 1, 2, 4, 8, then the row broadcasts of lanes 15 and 31.
__device__ inline double wave_scan_f64(double v) {
    v += dpp_f64<0x111, 0xf>(v);
    v += dpp_f64<0x112, 0xf>(v);
    v += dpp_f64<0x114, 0xf>(v);
    v += dpp_f64<0x118, 0xf>(v);
    v += dpp_f64<0x142, 0xa>(v);
    v += dpp_f64<0x143, 0xc>(v);
    return v;
}

// The same scan and lane read on exact 64-bit integers.
template <unsigned Ctrl, unsigned RowMask>
__device__ inline long long dpp_i64(long long v) {
    const uint64_t u = (uint64_t)v;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, Ctrl, RowMask,
                                                              0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), Ctrl,
                                                              RowMask, 0xf, false);
    return (long long)((uint64_t)hi << 32 | lo);
}

__device__ inline long long wave_scan_i64(long long v) {
    v += dpp_i64<0x111, 0xf>(v);
    v += dpp_i64<0x112, 0xf>(v);
    v += dpp_i64<0x114, 0xf>(v);
    v += dpp_i64<0x118, 0xf>(v);
    v += dpp_i64<0x142, 0xa>(v);
    v += dpp_i64<0x143, 0xc>(v);
    return v;
}

__device__ inline long long readlane_i64(long long v, int l) {
    const uint64_t u = (uint64_t)v;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
    return (long long)((uint64_t)hi << 32 | lo);
}

// The prefix phase of a row pass works on 256-column chunks in which lane
// `lane` owns the four consecutive columns x0 + 4 lane .. x0 + 4 lane + 3:
// a lane prefixes its four values in FP64, one wavefront scan over the lane
// totals places them, so a chunk costs one FP64 scan per four columns instead
// of one per column.
constexpr int kPreChunk = 256;

// Writes P[x + k + 1] (x = the lane's first column, k < 4, x + k < W) for one
// chunk from the lane's four values (zero past the row's end), given the
// row's sum before the chunk; returns the row's sum up to the chunk's end.
__device__ inline double chunk_prefix(const float (&v)[4], int x, int W, double carry, double* P) {
    double s[4];
    s[0] = (double)v[0];
#pragma unroll
    for (int k = 1; k < 4; ++k) s[k] = s[k - 1] + (double)v[k];
    const double inc = wave_scan_f64(s[3]);
    const double base = carry + (inc - s[3]);
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (x + k < W) P[x + k + 1] = base + s[k];
    return carry + readlane_f64(inc, 63);
}

// Moves the chunk's values c (lane `lane` holding columns x0 + 64 j + lane)
// through the wavefront's LDS stage into the four-consecutive-columns layout.
__device__ inline void restage(const float (&c)[4], float* stage, float (&v)[4]) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int j = 0; j < 4; ++j) stage[64 * j + lane] = c[j];
    __builtin_amdgcn_wave_barrier();
    const float4 q = *reinterpret_cast<const float4*>(stage + 4 * lane);
    v[0] = q.x;
    v[1] = q.y;
    v[2] = q.z;
    v[3] = q.w;
    __builtin_amdgcn_wave_barrier();  // the stage is rewritten next
}

// FP64 prefixes of the wavefront's row (W <= 2048): P[0] = 0 and
// P[x + 1] = v(0) + ... + v(x), where v is (kCost) the raw cost of Eq. 1 of
// row y for disparity d, or (kDeriv) its lambda_AD derivative, with the
// lambda_census derivative prefixed into P2, or else the row of `src`.  Raw
// costs are computed with lane `lane` on columns x0 + 64 j + lane (coalesced
// pixel loads) and restaged through `stage` (kPreChunk floats); `src` is read
// directly in the four-column layout.  Fixed order, bit-reproducible.
template <bool kCost, bool kDeriv>
__device__ inline void prefix_row(const uint4* pl, const uint4* pr, const float* src, int W, int d,
                                  const float* tab, float* stage, double* P, double* P2) {
    const int lane = threadIdx.x & 63;
    double carry = 0.0, carry2 = 0.0;
    if (lane == 0) {
        P[0] = 0.0;
        if (kDeriv) P2[0] = 0.0;
    }
    const bool vec = (W & 3) == 0;  // 16-byte aligned rows
    for (int x0 = 0; x0 < W; x0 += kPreChunk) {
        const int x = x0 + 4 * lane;
        float v[4], v2[4];
        if (kCost) {
            uint4 a[4], b[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int xc = min(x0 + 64 * j + lane, W - 1);
                a[j] = pl[xc];
                b[j] = pr[max(xc - d, 0)];
            }
            float c[4], c2[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                float cv, dca, dcc;
                cost_px<kDeriv>(a[j], b[j], x0 + 64 * j + lane - d >= 0, tab, cv, dca, dcc);
                c[j] = kDeriv ? dca : cv;
                c2[j] = dcc;
            }
            restage(c, stage, v);
            if (kDeriv) restage(c2, stage, v2);
        } else if (vec) {
            const float4 q = *reinterpret_cast<const float4*>(src + min(x, W - 4));
            v[0] = q.x;
            v[1] = q.y;
            v[2] = q.z;
            v[3] = q.w;
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) v[k] = src[min(x + k, W - 1)];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[k] = x + k < W ? v[k] : 0.0f;
            if (kDeriv) v2[k] = x + k < W ? v2[k] : 0.0f;
        }
        carry = chunk_prefix(v, x, W, carry, P);
        if (kDeriv) carry2 = chunk_prefix(v2, x, W, carry2, P2);
    }
    __builtin_amdgcn_wave_barrier();
}

// Bytes of dynamic LDS per wavefront: forward (one FP64 prefix, and the
// stage when it computes raw costs), gradient (two and the stage) and
// adjoint (64-bit difference array, the row, its arms).
__host__ __device__ inline size_t row_bytes(int W) { return ((size_t)W * 4 + 15) / 16 * 16; }
__host__ __device__ inline size_t prefix_bytes(int W) {
    return ((size_t)(W + 1) * 8 + 15) / 16 * 16;
}
constexpr size_t kStageBytes = kPreChunk * sizeof(float);
inline size_t row_lds_fwd(int W) { return prefix_bytes(W); }
inline size_t row_lds_cost(int W) { return prefix_bytes(W) + kStageBytes; }
inline size_t row_lds_grad(int W) { return 2 * prefix_bytes(W) + kStageBytes; }
inline size_t row_lds_adj(int W) {
    return ((size_t)(W + 1) * 8 + 15) / 16 * 16 + row_bytes(W) + ((size_t)W * 2 + 15) / 16 * 16;
}

// Lets a kernel take `bytes` of dynamic LDS (above the default limit for
// wide rows).
inline hipError_t allow_lds(const void* kernel, size_t bytes) {
    return bytes > 48 * 1024 ? hipFuncSetAttribute(kernel,
                                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                                   (int)bytes)
                             : hipSuccess;
}

// Forward row passes.  kCost: E1(x) = sum of the raw cost c over
// [x - l, x + r] (Eq. 1 computed here); else A2(x) = (sum of E2 over the
// range) / N2(x).
template <bool kCost>
__global__ __launch_bounds__(64 * kRowWaves) void k_soft_hrow(SoftGeom g, SoftImg im,
                                                              const float* __restrict__ in,
                                                              float* __restrict__ out,
                                                              size_t lds_wave) {
    extern __shared__ __align__(16) unsigned char dyn[];
    const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6), lane = threadIdx.x & 63,
              W = g.W;
    float* tab = reinterpret_cast<float*>(dyn);
    double* Pf = reinterpret_cast<double*>(dyn + (kCost ? kTabLds : 0) + w * lds_wave);
    float* stage = reinterpret_cast<float*>(reinterpret_cast<unsigned char*>(Pf) + prefix_bytes(W));
    if (kCost) load_tables(im, tab);
    const size_t P = (size_t)W * g.H;
    const int nrows = g.B * g.D * g.H;
    // raw costs: the workgroups of one image row on one XCD (its pixels are
    // the shared input); the other passes stream volumes and keep the
    // round-robin order
    const int blk = kCost ? xcd_block(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int r0 = (blk * kRowWaves + w) * kRowsPerWave;
    for (int rid = r0; rid < min(nrows, r0 + kRowsPerWave); ++rid) {
        int b, d, y;
        row_of(rid, g.D, g.H, b, d, y);
        const size_t base = ((size_t)b * g.D + d) * P + (size_t)y * W;
        const size_t pix = b * P + (size_t)y * W;
        prefix_row<kCost, false>(im.pixL + pix, im.pixR + pix, in + base, W, d, tab, stage, Pf,
                                 nullptr);
        // the row's arrays through row pointers (uniform), indexed by column
        const uint32_t* __restrict__ ar = g.arms + pix;
        const float* __restrict__ nr = g.n2 + pix;
        float* __restrict__ orow = out + base;
        over_row(W, [&](auto nb, int x0) {
            constexpr int NB = decltype(nb)::value;
            uint32_t a[NB];
            float n[NB];
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const int xc = min(x0 + 64 * j + lane, W - 1);
                a[j] = ar[xc];
                n[j] = kCost ? 1.0f : nr[xc];
            }
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const int x = x0 + 64 * j + lane;
                if (x < W) {
                    const float v = (float)(Pf[x + arm(a[j], 1) + 1] - Pf[x - arm(a[j], 0)]);
                    orow[x] = kCost ? v : v * __builtin_amdgcn_rcpf(n[j]);
                }
            }
        });
        __builtin_amdgcn_wave_barrier();
    }
}

// Gradient row pass.  With G = dLoss/dE1 and E1 = H c (H the row range-sum
// operator), dLoss/dlambda = sum_p (H^T G)(p) dc/dlambda(p)
//                          = sum_x G(x) (H dc/dlambda)(x):
// the range sums of the two cost derivatives, dotted with G, give one FP64
// pair per row (no adjoint volume is formed).
__global__ __launch_bounds__(64 * kRowWaves) void k_soft_hgrad(SoftGeom g, SoftImg im,
                                                               const float* __restrict__ G,
                                                               double* __restrict__ part,
                                                               size_t lds_wave) {
    extern __shared__ __align__(16) unsigned char dyn[];
    const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6), lane = threadIdx.x & 63,
              W = g.W;
    float* tab = reinterpret_cast<float*>(dyn);
    unsigned char* mine = dyn + kTabLds + w * lds_wave;
    double* Pa = reinterpret_cast<double*>(mine);
    double* Pc = reinterpret_cast<double*>(mine + prefix_bytes(W));
    float* stage = reinterpret_cast<float*>(mine + 2 * prefix_bytes(W));
    load_tables(im, tab);
    const size_t P = (size_t)W * g.H;
    const int nrows = g.B * g.D * g.H;
    const int r0 = (blockIdx.x * kRowWaves + w) * kRowsPerWave;
    for (int rid = r0; rid < min(nrows, r0 + kRowsPerWave); ++rid) {
        int b, d, y;
        row_of(rid, g.D, g.H, b, d, y);
        const size_t base = ((size_t)b * g.D + d) * P + (size_t)y * W;
        const size_t pix = b * P + (size_t)y * W;
        prefix_row<true, true>(im.pixL + pix, im.pixR + pix, nullptr, W, d, tab, stage, Pa, Pc);
        double sa = 0.0, sc = 0.0;
        const uint32_t* __restrict__ ar = g.arms + pix;
        const float* __restrict__ grow = G + base;
        over_row(W, [&](auto nb, int x0) {
            constexpr int NB = decltype(nb)::value;
            uint32_t a[NB];
            float gv[NB];
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const int xc = min(x0 + 64 * j + lane, W - 1);
                a[j] = ar[xc];
                gv[j] = grow[xc];
            }
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const int x = x0 + 64 * j + lane;
                if (x < W) {
                    const int hi = x + arm(a[j], 1) + 1, lo = x - arm(a[j], 0);
                    sa += (double)gv[j] * (Pa[hi] - Pa[lo]);
                    sc += (double)gv[j] * (Pc[hi] - Pc[lo]);
                }
            }
        });
        for (int off = 32; off > 0; off >>= 1) {  // fixed-order wavefront reduction
            sa += __shfl_down(sa, off, 64);
            sc += __shfl_down(sc, off, 64);
        }
        if (lane == 0) {
            part[2 * (size_t)rid] = sa;
            part[2 * (size_t)rid + 1] = sc;
        }
        __builtin_amdgcn_wave_barrier();  // Pa, Pc are rewritten for the next row
    }
}

// e^x as 2^(x log2 e) on the hardware base-2 exponential (about 1 ulp); the
// rounding of the product adds a relative error of about |x| 2^-24.
__device__ inline float exp_e(float x) { return __builtin_amdgcn_exp2f(x * 1.44269504088896341f); }

// Backward seed and adjoint row pass.  Per pixel and disparity, with
// w = softmax weight and g = dLoss/d dhat:
//   G_A2 / N2 = g w (dhat - d) / (T N2),   dLoss/dT term = g w (d - dhat) A2 / T^2;
// out = the adjoint of A2's row range sums applied to G_A2 / N2 (G_E2), and
// the temperature terms of the row summed into one FP64 value per row.
// The adjoint scatters each G(x) as +G at x - l(x) and -G after x + r(x)
// into a difference array and prefix-sums it.  The array holds 64-bit
// integers: G(x) 2^k rounded, with 2^k chosen from the row's largest |G| so
// that no sum can overflow, so the scatter's LDS atomic adds give the same
// bits in any order; the result is converted back with 2^-k.
__global__ __launch_bounds__(64 * kRowWaves) void k_soft_seed_adj(
    SoftGeom g, const float* __restrict__ A2, const float* __restrict__ theta,
    const float* __restrict__ dhat, const float* __restrict__ lse,
    const float* __restrict__ gdhat, float* __restrict__ out, double* __restrict__ partT,
    size_t lds_wave) {
    extern __shared__ __align__(16) unsigned char dyn[];
    const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6), lane = threadIdx.x & 63,
              W = g.W;
    unsigned char* mine = dyn + w * lds_wave;
    long long* Dq = reinterpret_cast<long long*>(mine);  // W + 1 entries
    float* row = reinterpret_cast<float*>(mine + ((size_t)(W + 1) * 8 + 15) / 16 * 16);
    uchar2* lr = reinterpret_cast<uchar2*>(reinterpret_cast<unsigned char*>(row) + row_bytes(W));
    const float T = theta[2], invT = 1.0f / T;
    const size_t P = (size_t)W * g.H;
    const int nrows = g.B * g.D * g.H;
    const int r0 = (blockIdx.x * kRowWaves + w) * kRowsPerWave;
    const bool vec = (W & 3) == 0;  // 16-byte aligned rows
    for (int rid = r0; rid < min(nrows, r0 + kRowsPerWave); ++rid) {
        int b, d, y;
        row_of(rid, g.D, g.H, b, d, y);
        const size_t base = ((size_t)b * g.D + d) * P + (size_t)y * W;
        const size_t pix = b * P + (size_t)y * W;
        // the row's inputs through row pointers (uniform), indexed by column
        const float* __restrict__ a2r = A2 + base;
        const float* __restrict__ gr = gdhat + pix;
        const float* __restrict__ dr = dhat + pix;
        const float* __restrict__ lr0 = lse + pix;
        const float* __restrict__ nr = g.n2 + pix;
        const uint32_t* __restrict__ ar = g.arms + pix;
        double acc = 0.0;
        float gmax = 0.0f;
        over_row<4>(W, [&](auto nb, int x0) {
            constexpr int NB = decltype(nb)::value;
            float a2[NB], gp[NB], dh[NB], l[NB], n2[NB];
            uint32_t a[NB];
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const int xc = min(x0 + 64 * j + lane, W - 1);
                a2[j] = a2r[xc];
                gp[j] = gr[xc];
                dh[j] = dr[xc];
                l[j] = lr0[xc];
                n2[j] = nr[xc];
                a[j] = ar[xc];
            }
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const int x = x0 + 64 * j + lane;
                if (x < W) {
                    const float wgt = exp_e(-a2[j] * invT - l[j]);
                    const float G =
                        gp[j] * wgt * (dh[j] - (float)d) * invT * __builtin_amdgcn_rcpf(n2[j]);
                    acc += (double)(gp[j] * wgt * ((float)d - dh[j]) * a2[j]) *
                           (double)(invT * invT);
                    row[x] = G;
                    lr[x] = make_uchar2((unsigned char)arm(a[j], 0), (unsigned char)arm(a[j], 1));
                    gmax = fmaxf(gmax, fabsf(G));
                }
            }
        });
        for (int o = 32; o > 0; o >>= 1) gmax = fmaxf(gmax, __shfl_xor(gmax, o, 64));
        for (int x = lane; x <= W; x += 64) Dq[x] = 0;
        __builtin_amdgcn_wave_barrier();
        // |G| < 2^(e+1) with e the exponent of the largest; 2^k G < 2^45, and
        // a pixel sums at most 2 kLMax + 1 of them: far below 2^63
        const int e = gmax > 0.0f ? ilogbf(gmax) : 0;
        const double up = ldexp(1.0, 44 - e), down = ldexp(1.0, e - 44);
        over_row(W, [&](auto nb, int x0) {
            constexpr int NB = decltype(nb)::value;
            float gx[NB];
            uchar2 ax[NB];
#pragma unroll
            for (int j = 0; j < NB; ++j) {  // the batch's reads first, then its adds
                const int xc = min(x0 + 64 * j + lane, W - 1);
                gx[j] = row[xc];
                ax[j] = lr[xc];
            }
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const int x = x0 + 64 * j + lane;
                if (x < W) {
                    const long long q = llrint((double)gx[j] * up);
                    atomicAdd(reinterpret_cast<unsigned long long*>(&Dq[x - ax[j].x]),
                              (unsigned long long)q);
                    atomicAdd(reinterpret_cast<unsigned long long*>(&Dq[x + ax[j].y + 1]),
                              (unsigned long long)(-q));
                }
            }
        });
        __builtin_amdgcn_wave_barrier();
        // prefix of the difference array (exact integers) in 256-column
        // chunks, a lane owning four consecutive columns: a local prefix, one
        // wavefront scan of the lane totals, and the outputs stored straight
        // from registers (16-byte stores when rows are 16-byte aligned)
        long long carry = 0;
        for (int x0 = 0; x0 < W; x0 += kPreChunk) {
            const int x = x0 + 4 * lane;
            long long sk[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) sk[k] = x + k < W ? Dq[min(x + k, W - 1)] : 0;
#pragma unroll
            for (int k = 1; k < 4; ++k) sk[k] += sk[k - 1];
            const long long inc = wave_scan_i64(sk[3]);
            const long long before = carry + (inc - sk[3]);
            float o[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) o[k] = (float)((double)(before + sk[k]) * down);
            if (vec) {
                if (x < W)
                    *reinterpret_cast<float4*>(out + base + x) =
                        make_float4(o[0], o[1], o[2], o[3]);
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (x + k < W) out[base + x + k] = o[k];
            }
            carry += readlane_i64(inc, 63);
        }
        __builtin_amdgcn_wave_barrier();
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
        if (lane == 0) partT[rid] = acc;
        __builtin_amdgcn_wave_barrier();
    }
}

// Column passes, streamed down each column: one thread per column, kSoftCols
// columns per workgroup, rows in batches of kSoftPre.  FP64 running sums in an
// LDS ring of kSoftRing rows per column keep every range sum exact to FP32
// rounding of the final value, and each thread touches only its own column,
// so the result does not depend on scheduling.  A batch makes all its ring
// writes before its ring reads: one LDS round trip per batch, not per row.
//
// The ring (20 KB per workgroup) bounds a CU to eight such workgroups, so
// the loads of one wavefront have to cover the memory latency by themselves:
// each thread keeps kSoftDepth batches of inputs in registers and loads
// kSoftDepth - 1 batches ahead of the one it processes.  The row loop is
// unrolled over one turn of the ring (kSoftTurn batches), so every ring slot
// and every buffer index is a compile-time constant: slots are immediate LDS
// offsets, and the wrap of a per-pixel range end around the ring is tested
// only in the batches where it can happen.  The loop body has no branch:
// loads read clamped rows, stores of rows outside the image get an
// out-of-range buffer offset (the hardware drops them), and the row count is
// rounded up to whole turns.
constexpr int kSoftCols = 64;
constexpr int kSoftPre = 5;                       // rows per batch
constexpr int kSoftRing = 2 * kLMax + 1 + kSoftPre;  // 40 rows
constexpr int kSoftTurn = kSoftRing / kSoftPre;   // batches per turn of the ring
constexpr int kSoftDepth = 4;                     // batches held per thread
constexpr int kSoftLead = (kSoftDepth - 1) * kSoftPre;  // rows streamed before row 0
constexpr uint32_t kSoftDrop = 0x80000000u;       // buffer offset past any plane (W H <= 2^27)
static_assert(kSoftRing % kSoftPre == 0 && kSoftTurn % kSoftDepth == 0,
              "a turn of the ring is a whole number of batches and of buffer rotations");
static_assert(kSoftLead < kSoftRing, "the lead-in rows fit in the ring");

// kSoftPre rows of a column pass's per-row inputs.
struct ColBatch {
    float v[kSoftPre];     // input of row y
    uint32_t a[kSoftPre];  // arms of row y (adjoint) or of row y - kLMax (forward)
    float s[kSoftPre];     // scale of row y - kLMax
};

// Per-column state of a column pass: buffer resources over one plane of the
// input, output, arms and scale, and the running state.
struct ColPass {
    double (*ring)[kSoftCols];  // the workgroup's LDS ring
    __amdgpu_buffer_rsrc_t src, arms, sc, dst;
    uint32_t x4, W4;  // byte offset of the (clamped) column, bytes per row
    int t, H, rows;
    bool ok;
    double acc;  // running prefix (forward) or running sum of differences (adjoint)
};

template <bool kScale, bool kAdj>
__device__ inline void col_load(const ColPass& c, int y0, ColBatch& b) {
#pragma unroll
    for (int k = 0; k < kSoftPre; ++k) {
        const int y = y0 + k, yo = y - kLMax;
        const uint32_t yq = (uint32_t)min(y, c.H - 1);  // y >= 0
        const uint32_t oq = (uint32_t)min(max(yo, 0), c.H - 1);
        b.v[k] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(c.src, c.x4,
                                                                                 yq * c.W4, 0));
        b.a[k] = __builtin_amdgcn_raw_buffer_load_b32(c.arms, c.x4, (kAdj ? yq : oq) * c.W4, 0);
        b.s[k] = kScale ? __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                                        c.sc, c.x4, oq * c.W4, 0))
                        : 1.0f;
    }
}

// Stores r as row yo of the column; dropped for rows outside the image and
// for lanes past the last column.
__device__ inline void col_store(const ColPass& c, int yo, float r) {
    const bool in = c.ok && yo >= 0 && yo < c.H;
    const uint32_t off = in ? (uint32_t)yo * c.W4 + c.x4 : kSoftDrop;
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, r), c.dst, off, 0, 0);
}

// Ring slot `base + v` and `base - v` (mod kSoftRing) for a compile-time
// base in [0, kSoftRing) and a per-pixel 0 <= v <= kLMax + 1 (arm lengths
// never exceed kLMax): the wrap test folds away where it cannot happen.
__device__ inline int ring_up(int base, int v) {
    const int r = base + v;
    return base + kLMax + 1 < kSoftRing ? r : (r >= kSoftRing ? r - kSoftRing : r);
}
__device__ inline int ring_down(int base, int v) {
    const int r = base - v;
    return base >= kLMax + 1 ? r : (r < 0 ? r + kSoftRing : r);
}
constexpr int ring_mod(int s) { return ((s % kSoftRing) + kSoftRing) % kSoftRing; }

template <bool kScale>
__device__ inline ColPass col_setup(const SoftGeom& g, const float* in, const float* scale,
                                    float* out, double (*ring)[kSoftCols]) {
    ColPass c;
    c.t = threadIdx.x;
    const int x = blockIdx.x * kSoftCols + c.t;
    const int bd = blockIdx.y, b = bd / g.D;
    c.ok = x < g.W;
    const size_t P = (size_t)g.W * g.H;
    const int bytes = (int)(P * 4);
    c.src = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(in + (size_t)bd * P), (short)0,
                                              bytes, 0x00020000);
    c.arms = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint32_t*>(g.arms + (size_t)b * P),
                                               (short)0, bytes, 0x00020000);
    c.sc = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>((kScale ? scale : in) + (size_t)b * P), (short)0, bytes, 0x00020000);
    c.dst = __builtin_amdgcn_make_buffer_rsrc(out + (size_t)bd * P, (short)0, bytes, 0x00020000);
    c.x4 = 4u * (uint32_t)(c.ok ? x : 0);
    c.W4 = 4u * (uint32_t)g.W;
    c.ring = ring;
    c.H = g.H;
    c.rows = g.H + kLMax;
    c.acc = 0.0;
    return c;
}

// Streams the column through `step(c, batch, y0, s0)`: rows y0 .. y0 +
// kSoftPre - 1, whose first row sits in ring slot s0 (a compile-time
// constant once unrolled).  The stream starts kSoftLead rows before row 0
// on zeroed buffers, so the loop needs no prologue of loads (whose registers
// the compiler would copy, and wait for, at the loop's entry); those rows
// add zero and store nothing, and row 0 sits in slot 0.
template <bool kScale, bool kAdj, typename Step>
__device__ inline void col_stream(ColPass& c, Step step) {
    ColBatch buf[kSoftDepth];
#pragma unroll
    for (int j = 0; j < kSoftDepth; ++j)
#pragma unroll
        for (int k = 0; k < kSoftPre; ++k) {
            buf[j].v[k] = 0.0f;
            buf[j].a[k] = 0u;
            buf[j].s[k] = 1.0f;
        }
    for (int y0 = -kSoftLead; y0 < c.rows; y0 += kSoftRing) {
#pragma unroll
        for (int j = 0; j < kSoftTurn; ++j) {
            const int yb = y0 + j * kSoftPre;
            col_load<kScale, kAdj>(c, yb + kSoftLead, buf[(j + kSoftDepth - 1) % kSoftDepth]);
            ColBatch& cur = buf[j % kSoftDepth];
            // The batch's values are used from here on: without this pin the
            // compiler starts converting a later batch early, which waits for
            // loads that should still be in flight.
#pragma unroll
            for (int k = 0; k < kSoftPre; ++k) {
                asm volatile("" : "+v"(cur.v[k]), "+v"(cur.a[k]));
                if (kScale) asm volatile("" : "+v"(cur.s[k]));
            }
            step(c, cur, yb, ring_mod(j * kSoftPre - kSoftLead));
        }
    }
}

// out(y) = (sum of in over the vertical range of pixel y) [/ scale(y)], with
// the running column prefix P: out(y) = P(y + dn) - P(y - u - 1).  The batch
// of rows y0 .. y0 + kSoftPre - 1 (outputs kLMax rows behind) reads prefixes
// from row y0 - 2 kLMax - 1 on; its writes land in the slots of rows
// y0 - kSoftRing ... y0 + kSoftPre - 1 - kSoftRing, which are older.  The
// lead-in rows hold P = 0, which is the prefix before row 0 (read as row -1
// by a range that starts at row 0); rows past the image only feed outputs
// that are dropped.
template <bool kScale>
__global__ __launch_bounds__(kSoftCols) void k_soft_vs(SoftGeom g, const float* __restrict__ in,
                                                       const float* __restrict__ scale,
                                                       float* __restrict__ out) {
    __shared__ double ring[kSoftRing][kSoftCols];
    ColPass c = col_setup<kScale>(g, in, scale, out, ring);
    col_stream<kScale, false>(c, [](ColPass& c, const ColBatch& cur, int y0, int s0) {
        const int t = c.t;
#pragma unroll
        for (int k = 0; k < kSoftPre; ++k) {
            c.acc += (double)cur.v[k];
            c.ring[ring_mod(s0 + k)][t] = c.acc;
        }
        double hi[kSoftPre], lo[kSoftPre];
#pragma unroll
        for (int k = 0; k < kSoftPre; ++k) {
            const int u = arm(cur.a[k], 2), dn = arm(cur.a[k], 3);
            hi[k] = c.ring[ring_up(ring_mod(s0 + k - kLMax), dn)][t];
            lo[k] = c.ring[ring_down(ring_mod(s0 + k - kLMax - 1), u)][t];
        }
#pragma unroll
        for (int k = 0; k < kSoftPre; ++k) {
            const float r = (float)(hi[k] - lo[k]);
            col_store(c, y0 + k - kLMax, kScale ? r / cur.s[k] : r);
        }
    });
}

// Adjoint of k_soft_vs: out(y') = sum over pixels y whose vertical range
// covers y' of in(y), [/ scale(y')].  Each y adds in(y) at row y - u and
// subtracts it after row y + dn in a ring of differences (LDS FP64 adds that
// return nothing, in program order per column); row y' is final kLMax rows
// later and its running sum is the output.  A batch first makes all its
// adds, into rows y0 - kLMax ... y0 + kSoftPre + kLMax, then finishes (reads
// and clears) rows y0 - kLMax ... y0 + kSoftPre - 1 - kLMax: that span is
// kSoftRing rows, so no add lands in the slot of a row still to be finished,
// and every slot it lands in was cleared when its previous row finished.
// Rows outside the image add zero.
template <bool kScale>
__global__ __launch_bounds__(kSoftCols) void k_soft_vsa(SoftGeom g, const float* __restrict__ in,
                                                        const float* __restrict__ scale,
                                                        float* __restrict__ out) {
    __shared__ double ring[kSoftRing][kSoftCols];
    ColPass c = col_setup<kScale>(g, in, scale, out, ring);
    for (int i = 0; i < kSoftRing; ++i) ring[i][c.t] = 0.0;
    col_stream<kScale, true>(c, [](ColPass& c, const ColBatch& cur, int y0, int s0) {
        const int t = c.t;
#pragma unroll
        for (int k = 0; k < kSoftPre; ++k) {
            const int u = arm(cur.a[k], 2), dn = arm(cur.a[k], 3);
            const float vf = (unsigned)(y0 + k) < (unsigned)c.H ? cur.v[k] : 0.0f;
            const double v = (double)vf;
            __hip_atomic_fetch_add(&c.ring[ring_down(ring_mod(s0 + k), u)][t], v,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            __hip_atomic_fetch_add(&c.ring[ring_up(ring_mod(s0 + k + 1), dn)][t], -v,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        double dv[kSoftPre];
#pragma unroll
        for (int k = 0; k < kSoftPre; ++k)
            dv[k] = __hip_atomic_exchange(&c.ring[ring_mod(s0 + k - kLMax)][t], 0.0,
                                          __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        // all the batch's exchanges in flight together (one LDS round trip)
#pragma unroll
        for (int k = 0; k < kSoftPre; ++k) asm volatile("" : "+v"(dv[k]));
#pragma unroll
        for (int k = 0; k < kSoftPre; ++k) {
            c.acc += dv[k];
            const float r = (float)c.acc;
            col_store(c, y0 + k - kLMax, kScale ? r / cur.s[k] : r);
        }
    });
}


// Soft-argmin over d per pixel: dhat and lse (log-sum-exp of -A2/T), in one
// pass over the slices: kArgBatch slices are loaded at a time and the running
// sums are rescaled whenever the running maximum grows.
constexpr int kArgBatch = 16;

__global__ __launch_bounds__(256) void k_soft_argmin(SoftGeom g, const float* __restrict__ A2,
                                                     const float* __restrict__ theta,
                                                     float* __restrict__ dhat,
                                                     float* __restrict__ lse) {
    const size_t P = (size_t)g.W * g.H;
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    const int b = blockIdx.y;
    if (i >= P) return;
    const float invT = 1.0f / theta[2];
    const float* a = A2 + (size_t)b * g.D * P + i;
    float m = -INFINITY, z = 0.0f, zd = 0.0f;
    for (int d0 = 0; d0 < g.D; d0 += kArgBatch) {
        float v[kArgBatch];
#pragma unroll
        for (int j = 0; j < kArgBatch; ++j) v[j] = -a[(size_t)min(d0 + j, g.D - 1) * P] * invT;
        float mb = m;
#pragma unroll
        for (int j = 0; j < kArgBatch; ++j) mb = d0 + j < g.D ? fmaxf(mb, v[j]) : mb;
        const float sc = exp_e(m - mb);  // 0 on the first batch (m = -inf)
        z *= sc;
        zd *= sc;
#pragma unroll
        for (int j = 0; j < kArgBatch; ++j) {
            if (d0 + j < g.D) {
                const float e = exp_e(v[j] - mb);
                z += e;
                zd += (float)(d0 + j) * e;
            }
        }
        m = mb;
    }
    dhat[(size_t)b * P + i] = zd / z;
    lse[(size_t)b * P + i] = m + logf(z);
}

// Two-level fixed-order reduction of the gradient partial sums: block k of
// kRedBlocks sums a contiguous chunk of the per-row lambda partials and of
// the per-block temperature partials; then one block sums the block totals.
constexpr int kRedBlocks = 256;

__device__ inline void tree3(double (*red)[256], double a, double c, double t) {
    red[0][threadIdx.x] = a;
    red[1][threadIdx.x] = c;
    red[2][threadIdx.x] = t;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_soft_reduce1(const double* __restrict__ partAC,
                                                      size_t nAC,
                                                      const double* __restrict__ partT, size_t nT,
                                                      double* __restrict__ blk) {
    __shared__ double red[3][256];
    const size_t ca = (nAC + kRedBlocks - 1) / kRedBlocks, ct = (nT + kRedBlocks - 1) / kRedBlocks;
    const size_t a0 = blockIdx.x * ca, a1 = a0 + ca < nAC ? a0 + ca : nAC;
    const size_t t0 = blockIdx.x * ct, t1 = t0 + ct < nT ? t0 + ct : nT;
    double a = 0.0, c = 0.0, t = 0.0;
    for (size_t i = a0 + threadIdx.x; i < a1; i += 256) {
        a += partAC[2 * i];
        c += partAC[2 * i + 1];
    }
    for (size_t i = t0 + threadIdx.x; i < t1; i += 256) t += partT[i];
    tree3(red, a, c, t);
    if (threadIdx.x == 0)
        for (int k = 0; k < 3; ++k) blk[3 * blockIdx.x + k] = red[k][0];
}

__global__ __launch_bounds__(256) void k_soft_reduce2(const double* __restrict__ blk,
                                                      float* __restrict__ grad) {
    __shared__ double red[3][256];
    const int t = threadIdx.x;
    tree3(red, blk[3 * t], blk[3 * t + 1], blk[3 * t + 2]);
    if (t == 0)
        for (int k = 0; k < 3; ++k) grad[k] = (float)red[k][0];
}

}  // namespace

// ---- launchers -------------------------------------------------------------

hipError_t soft_prepare(const float* theta, float* tab, const uint32_t* arms, int B, int W, int H,
                        int D, float* n1, float* n2, hipStream_t st) {
    hipLaunchKernelGGL(k_soft_tables, dim3(4), dim3(256), 0, st, theta, tab);
    SoftGeom g{arms, nullptr, nullptr, B, W, H, D};
    hipLaunchKernelGGL(k_soft_counts, dim3((W + kCntTW - 1) / kCntTW, (H + kCntTH - 1) / kCntTH, B),
                       dim3(256), 0, st, g, n1,
                       n2);
    return hipGetLastError();
}

// Forward aggregation into A2 (B x D x H x W); t1, t2 are volume-sized scratch.
hipError_t soft_aggregate(const SoftBuffers& s, int B, int W, int H, int D, float* A2, float* t1,
                          float* t2, hipStream_t st) {
    SoftGeom g{s.arms, s.n1, s.n2, B, W, H, D};
    SoftImg im{s.pixL, s.pixR, s.alpha, s.tab};
    const int nrows = B * D * H;
    const dim3 gr((nrows + kRowWaves * kRowsPerWave - 1) / (kRowWaves * kRowsPerWave));
    const size_t lf = row_lds_fwd(W), lc = row_lds_cost(W);
    hipError_t e = allow_lds(reinterpret_cast<const void*>(&k_soft_hrow<true>),
                             kTabLds + kRowWaves * lc);
    if (e == hipSuccess)
        e = allow_lds(reinterpret_cast<const void*>(&k_soft_hrow<false>), kRowWaves * lf);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_soft_hrow<true>, gr, dim3(64 * kRowWaves), kTabLds + kRowWaves * lc, st, g,
                       im, (const float*)nullptr, t1, lc);                                   // E1
    const dim3 gv((W + kSoftCols - 1) / kSoftCols, B * D);
    hipLaunchKernelGGL(k_soft_vs<true>, gv, dim3(kSoftCols), 0, st, g, t1, s.n1, t2);      // a1
    hipLaunchKernelGGL(k_soft_vs<false>, gv, dim3(kSoftCols), 0, st, g, t2,
                       (const float*)nullptr, t1);                                           // E2
    hipLaunchKernelGGL(k_soft_hrow<false>, gr, dim3(64 * kRowWaves), kRowWaves * lf, st, g, im, t1,
                       A2, lf);                                                              // A2
    return hipGetLastError();
}

hipError_t soft_argmin(const SoftBuffers& s, int B, int W, int H, int D, const float* A2,
                       const float* theta, float* dhat, float* lse, hipStream_t st) {
    SoftGeom g{s.arms, s.n1, s.n2, B, W, H, D};
    const size_t P = (size_t)W * H;
    hipLaunchKernelGGL(k_soft_argmin, dim3((unsigned)((P + 255) / 256), B), dim3(256), 0, st, g,
                       A2, theta, dhat, lse);
    return hipGetLastError();
}

// Backward: A2 recomputed by the caller into `A2`; t1, t2 volume scratch.
hipError_t soft_backward(const SoftBuffers& s, int B, int W, int H, int D, const float* A2,
                         const float* theta, const float* dhat, const float* lse,
                         const float* gdhat, float* t1, float* t2, double* partAC,
                         double* partT, float* grad, hipStream_t st) {
    SoftGeom g{s.arms, s.n1, s.n2, B, W, H, D};
    SoftImg im{s.pixL, s.pixR, s.alpha, s.tab};
    const int nrows = B * D * H;
    const dim3 gr((nrows + kRowWaves * kRowsPerWave - 1) / (kRowWaves * kRowsPerWave));
    const size_t la = row_lds_adj(W), lg = row_lds_grad(W);
    hipError_t e = allow_lds(reinterpret_cast<const void*>(&k_soft_seed_adj), kRowWaves * la);
    if (e == hipSuccess)
        e = allow_lds(reinterpret_cast<const void*>(&k_soft_hgrad), kTabLds + kRowWaves * lg);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_soft_seed_adj, gr, dim3(64 * kRowWaves), kRowWaves * la, st, g, A2, theta,
                       dhat, lse, gdhat, t2, partT, la);                 // G_E2, T-gradient terms
    const dim3 gv((W + kSoftCols - 1) / kSoftCols, B * D);
    hipLaunchKernelGGL(k_soft_vsa<true>, gv, dim3(kSoftCols), 0, st, g, t2, s.n1, t1);  // G_a1/N1
    hipLaunchKernelGGL(k_soft_vsa<false>, gv, dim3(kSoftCols), 0, st, g, t1,
                       (const float*)nullptr, t2);                                    // G_E1
    hipLaunchKernelGGL(k_soft_hgrad, gr, dim3(64 * kRowWaves), kTabLds + kRowWaves * lg, st, g,
                       im, t2, partAC, lg);                                // G_E1 . H dc/dlambda
    double* blk = partT + (size_t)nrows;  // kRedBlocks x 3 after the row partials
    hipLaunchKernelGGL(k_soft_reduce1, dim3(kRedBlocks), dim3(256), 0, st, partAC,
                       (size_t)nrows, partT, (size_t)nrows, blk);
    hipLaunchKernelGGL(k_soft_reduce2, dim3(1), dim3(256), 0, st, blk, grad);
    return hipGetLastError();
}
