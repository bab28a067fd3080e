// k_soft.hip -- differentiable soft-argmin form of the matcher (left view).
//
// Forward, per pair b, disparity d, pixel p (all float):
//   c(p,d)  = alpha_p (1 - exp(-(s/3)/lambda_AD)) + (1 - alpha_p)(1 - exp(-h/lambda_census))
//             (Eq. 1; c = 1 where the partner pixel x - d is outside the image)
//   E1 = row range sum of c       a1 = (column range sum of E1) / N1     (Eq. 2, stage 1)
//   E2 = column range sum of a1   A2 = (row range sum of E2) / N2         (Eq. 2, stage 2)
//   dhat = sum_d d softmax_d(-A2 / T),  lse = log sum_d exp(-A2 / T)
// Row range sums add at most 2 kLMax + 1 terms directly; column range sums
// are differences of FP64 running column sums (exact to the final FP32
// rounding).  Every sum runs in a fixed order, so results are bit-reproducible.
//
// Backward, given g = dLoss/d dhat:
//   G_A2  = g w (dhat - d) / T,   dLoss/dT = sum g w (d - dhat) A2 / T^2
// then the adjoint of each range sum: an output that summed a range hands its
// adjoint back to every pixel of that range.  Row adjoints are gathers over
// the (at most 2 kLMax + 1) candidate pixels whose range can cover a pixel;
// column adjoints are FP64 difference arrays streamed down each column by
// one thread.  There are no atomics and no float reductions of unspecified
// order.  Finally
//   dLoss/dlambda_AD     = sum G_c alpha   d(1 - exp(-(s/3)/lambda_AD))/dlambda_AD
//   dLoss/dlambda_census = sum G_c (1 - alpha) d(1 - exp(-h/lambda_census))/dlambda_census
// with fixed-order two-level reductions.
//
// Layout: volumes are B x D x H x W float in handle scratch; arms, census
// and packed RGB are per pair B x H x W.  Row passes run one workgroup per
// image row with the row in LDS; column passes one thread per column,
// streaming down the rows with a ring of FP64 sums in LDS.
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

// Region pixel counts of the left view (as floats) for every pair.
__global__ void k_soft_counts(SoftGeom g, float* __restrict__ n1, float* __restrict__ n2) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int b = blockIdx.z;
    if (x >= g.W || y >= g.H) return;
    const uint32_t* A = g.arms + (size_t)b * g.W * g.H;
    const uint32_t a = A[(size_t)y * g.W + x];
    int s1 = 0, s2 = 0;
    for (int yy = max(0, y - arm(a, 2)); yy <= min(g.H - 1, y + arm(a, 3)); ++yy) {
        const uint32_t q = A[(size_t)yy * g.W + x];
        s1 += arm(q, 0) + arm(q, 1) + 1;
    }
    for (int xx = max(0, x - arm(a, 0)); xx <= min(g.W - 1, x + arm(a, 1)); ++xx) {
        const uint32_t q = A[(size_t)y * g.W + xx];
        s2 += arm(q, 2) + arm(q, 3) + 1;
    }
    const size_t i = (size_t)b * g.W * g.H + (size_t)y * g.W + x;
    n1[i] = (float)s1;
    n2[i] = (float)s2;
}

// Raw costs c (and, with kDeriv, the two lambda-derivative factors packed as
// dc/dlambda_AD and dc/dlambda_c) of one image row for one (pair, d).
template <bool kDeriv>
__device__ inline void cost_row(const uint32_t* rgbL, const uint32_t* rgbR, const uint64_t* cenL,
                                const uint64_t* cenR, const uint32_t* arms, const float* alpha,
                                const float* tab, int W, int y, int d, int x, float* c,
                                float* dca, float* dcc) {
    const size_t i = (size_t)y * W + x;
    if (x - d < 0) {
        *c = 1.0f;
        if (kDeriv) *dca = 0.0f, *dcc = 0.0f;
        return;
    }
    const uint32_t s = __builtin_amdgcn_sad_u8(rgbL[i], rgbR[i - d], 0u);
    const int h = __popcll(cenL[i] ^ cenR[i - d]);
    const uint32_t a = arms[i];
    const int lmin = min(min(arm(a, 0), arm(a, 1)), min(arm(a, 2), arm(a, 3)));
    const float al = alpha[lmin];
    *c = al * tab[s] + (1.0f - al) * tab[1536 + h];
    if (kDeriv) {
        *dca = al * tab[768 + s];
        *dcc = (1.0f - al) * tab[1664 + h];
    }
}

struct SoftImg {
    const uint32_t* rgbL;  // B x H x W packed RGB
    const uint32_t* rgbR;
    const uint64_t* cenL;  // B x H x W census
    const uint64_t* cenR;
    const float* alpha;    // alpha_L, L = 0..kLMax
    const float* tab;      // k_soft_tables output
};

// Row passes: one wavefront per image row, kRowWaves wavefronts per
// workgroup, each with its own LDS slice (no workgroup barriers) and
// kRowsPerWave rows in turn.  Row ids run over (b, d, y) with y fastest.
constexpr int kRowWaves = 4;
constexpr int kRowsPerWave = 4;

__device__ inline void row_of(int rid, int D, int H, int& b, int& d, int& y) {
    y = rid % H;
    const int bd = rid / H;
    d = bd % D;
    b = bd / D;
}

// FP64 inclusive prefix of the wavefront's row (W <= 2048): P[0] = 0,
// P[x + 1] = row[0] + ... + row[x].  Lane L sums its contiguous run of
// ceil(W / 64) values, the run totals are scanned across the wavefront, and
// the runs are written with their offsets; fixed order, bit-reproducible.
__device__ inline void wave_row_prefix(const float* row, double* P, int W) {
    const int lane = threadIdx.x & 63, c = (W + 63) / 64, x0 = lane * c;
    double acc = 0.0;
    for (int k = 0; k < c; ++k)
        if (x0 + k < W) acc += (double)row[x0 + k];
    double inc = acc;
    for (int off = 1; off < 64; off <<= 1) {
        const double n = __shfl_up(inc, off, 64);
        if (lane >= off) inc += n;
    }
    double run = inc - acc;
    if (lane == 0) P[0] = 0.0;
    for (int k = 0; k < c; ++k)
        if (x0 + k < W) {
            run += (double)row[x0 + k];
            P[x0 + k + 1] = run;
        }
    __builtin_amdgcn_wave_barrier();
}

// Adjoint of a row range sum at x': the pixels x whose horizontal range
// covers x' are x' itself, x' + k with l(x' + k) >= k and x' - k with
// r(x' - k) >= k (k = 1 .. kLMax); added in a fixed order.  lr holds the
// arms of the row as bytes (l, r); row and lr are zero-padded by kLMax.
__device__ inline float row_adjoint(const float* rowp, const uchar2* lrp, int xp) {
    float s = rowp[xp];
#pragma unroll
    for (int k = 1; k <= kLMax; ++k) {
        s += lrp[xp + k].x >= k ? rowp[xp + k] : 0.0f;
        s += lrp[xp - k].y >= k ? rowp[xp - k] : 0.0f;
    }
    return s;
}

// Bytes of dynamic LDS per wavefront: forward (row + FP64 prefix) and
// adjoint (padded row + padded arms).
inline size_t row_lds_fwd(int W) { return ((size_t)W * 4 + 15) / 16 * 16 + (size_t)(W + 1) * 8; }
inline size_t row_lds_adj(int W) {
    return ((size_t)(W + 2 * kLMax) * 4 + 15) / 16 * 16 + (size_t)(W + 2 * kLMax) * 2;
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
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, W = g.W;
    unsigned char* mine = dyn + w * lds_wave;
    float* row = reinterpret_cast<float*>(mine);
    double* Pf = reinterpret_cast<double*>(mine + ((size_t)W * 4 + 15) / 16 * 16);
    const size_t P = (size_t)W * g.H;
    const int nrows = g.B * g.D * g.H;
    const int r0 = (blockIdx.x * kRowWaves + w) * kRowsPerWave;
    for (int rid = r0; rid < min(nrows, r0 + kRowsPerWave); ++rid) {
        int b, d, y;
        row_of(rid, g.D, g.H, b, d, y);
        const size_t base = ((size_t)b * g.D + d) * P + (size_t)y * W;
        const uint32_t* arms = g.arms + b * P + (size_t)y * W;
        for (int x = lane; x < W; x += 64) {
            float c;
            if (kCost)
                cost_row<false>(im.rgbL + b * P, im.rgbR + b * P, im.cenL + b * P,
                                im.cenR + b * P, g.arms + b * P, im.alpha, im.tab, W, y, d, x, &c,
                                nullptr, nullptr);
            else
                c = in[base + x];
            row[x] = c;
        }
        __builtin_amdgcn_wave_barrier();
        wave_row_prefix(row, Pf, W);
        for (int x = lane; x < W; x += 64) {
            const uint32_t a = arms[x];
            const float v = (float)(Pf[x + arm(a, 1) + 1] - Pf[x - arm(a, 0)]);
            out[base + x] = kCost ? v : v / g.n2[b * P + (size_t)y * W + x];
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// Adjoint row passes.  kGrad: the adjoint of E1's row sums (G_c), dotted
// with dc/dlambda_AD and dc/dlambda_census into one FP64 pair per row;
// else out = the adjoint of A2's row sums (G_E2).
template <bool kGrad>
__global__ __launch_bounds__(64 * kRowWaves) void k_soft_hrow_adj(SoftGeom g, SoftImg im,
                                                                  const float* __restrict__ in,
                                                                  float* __restrict__ out,
                                                                  double* __restrict__ part,
                                                                  size_t lds_wave) {
    extern __shared__ __align__(16) unsigned char dyn[];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, W = g.W;
    unsigned char* mine = dyn + w * lds_wave;
    float* row = reinterpret_cast<float*>(mine);
    uchar2* lr = reinterpret_cast<uchar2*>(mine + ((size_t)(W + 2 * kLMax) * 4 + 15) / 16 * 16);
    const size_t P = (size_t)W * g.H;
    const int nrows = g.B * g.D * g.H;
    const int r0 = (blockIdx.x * kRowWaves + w) * kRowsPerWave;
    for (int rid = r0; rid < min(nrows, r0 + kRowsPerWave); ++rid) {
        int b, d, y;
        row_of(rid, g.D, g.H, b, d, y);
        const size_t base = ((size_t)b * g.D + d) * P + (size_t)y * W;
        const uint32_t* arms = g.arms + b * P + (size_t)y * W;
        for (int x = lane - kLMax; x < W + kLMax; x += 64) {
            const bool in_row = x >= 0 && x < W;
            const uint32_t a = in_row ? arms[x] : 0u;
            row[x + kLMax] = in_row ? in[base + x] : 0.0f;
            lr[x + kLMax] = make_uchar2((unsigned char)arm(a, 0), (unsigned char)arm(a, 1));
        }
        __builtin_amdgcn_wave_barrier();
        double sa = 0.0, sc = 0.0;
        for (int xp = lane; xp < W; xp += 64) {
            const float s = row_adjoint(row + kLMax, lr + kLMax, xp);
            if (kGrad) {
                float c, dca, dcc;
                cost_row<true>(im.rgbL + b * P, im.rgbR + b * P, im.cenL + b * P,
                               im.cenR + b * P, g.arms + b * P, im.alpha, im.tab, W, y, d, xp, &c,
                               &dca, &dcc);
                sa += (double)(s * dca);
                sc += (double)(s * dcc);
            } else {
                out[base + xp] = s;
            }
        }
        if (kGrad) {  // fixed-order wavefront reduction
            for (int off = 32; off > 0; off >>= 1) {
                sa += __shfl_down(sa, off, 64);
                sc += __shfl_down(sc, off, 64);
            }
            if (lane == 0) {
                part[2 * (size_t)rid] = sa;
                part[2 * (size_t)rid + 1] = sc;
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// Column passes, streamed down each column: one thread per column, kSoftCols
// columns per workgroup, rows in order.  FP64 running sums in an LDS ring of
// kSoftRing rows per column keep every range sum exact to FP32 rounding of
// the final value, and each thread touches only its own column, so the result
// does not depend on scheduling.
constexpr int kSoftCols = 128;
constexpr int kSoftRing = 2 * kLMax + 2;
constexpr int kSoftPre = 8;  // rows loaded ahead

// out(y) = (sum of in over the vertical range of pixel y) [/ scale(y)], with
// the running column prefix P: out(y) = P(y + dn) - P(y - u - 1).
template <bool kScale>
__global__ __launch_bounds__(kSoftCols) void k_soft_vs(SoftGeom g, const float* __restrict__ in,
                                                       const float* __restrict__ scale,
                                                       float* __restrict__ out) {
    __shared__ double ring[kSoftRing][kSoftCols];
    const int t = threadIdx.x, x = blockIdx.x * kSoftCols + t;
    const int bd = blockIdx.y, b = bd / g.D;
    const bool ok = x < g.W;
    const int xc = ok ? x : 0;
    const size_t P = (size_t)g.W * g.H;
    const float* src = in + (size_t)bd * P + xc;
    const uint32_t* arms = g.arms + (size_t)b * P + xc;
    const float* sc = (kScale ? scale : in) + (size_t)b * P + xc;
    float* dst = out + (size_t)bd * P + xc;
    double acc = 0.0;
    int slot = 0;  // ring slot of row y (y mod kSoftRing)
    for (int y0 = 0; y0 < g.H + kLMax; y0 += kSoftPre) {
        float v[kSoftPre];
        uint32_t a[kSoftPre];
        float s[kSoftPre];
#pragma unroll
        for (int k = 0; k < kSoftPre; ++k) {  // clamped rows: every load is unconditional
            const int y = y0 + k, yo = y - kLMax;
            const size_t yq = (size_t)min(y, g.H - 1), oq = (size_t)min(max(yo, 0), g.H - 1);
            v[k] = src[yq * g.W];
            a[k] = arms[oq * g.W];
            s[k] = kScale ? sc[oq * g.W] : 1.0f;
            v[k] = y < g.H ? v[k] : 0.0f;
        }
#pragma unroll
        for (int k = 0; k < kSoftPre; ++k) {
            const int y = y0 + k, yo = y - kLMax;
            acc += (double)v[k];
            ring[slot][t] = acc;
            if (yo >= 0 && yo < g.H) {
                const int u = arm(a[k], 2), dn = arm(a[k], 3);
                // P(yo + dn) is kLMax - dn rows back, P(yo - u - 1) kLMax + u + 1
                int sh = slot - (kLMax - dn), sl = slot - (kLMax + u + 1);
                sh += sh < 0 ? kSoftRing : 0;
                sl += sl < 0 ? kSoftRing : 0;
                const double lo = yo - u - 1 >= 0 ? ring[sl][t] : 0.0;
                const float r = (float)(ring[sh][t] - lo);
                if (ok) dst[(size_t)yo * g.W] = kScale ? r / s[k] : r;
            }
            slot = slot + 1 == kSoftRing ? 0 : slot + 1;
        }
    }
}

// Adjoint of k_soft_vs: out(y') = sum over pixels y whose vertical range
// covers y' of in(y), [/ scale(y')].  Each y adds in(y) at row y - u and
// subtracts it after row y + dn in a ring of differences; row y' is final
// kLMax rows later and its running sum is the output.
template <bool kScale>
__global__ __launch_bounds__(kSoftCols) void k_soft_vsa(SoftGeom g, const float* __restrict__ in,
                                                        const float* __restrict__ scale,
                                                        float* __restrict__ out) {
    __shared__ double ring[kSoftRing][kSoftCols];
    const int t = threadIdx.x, x = blockIdx.x * kSoftCols + t;
    const int bd = blockIdx.y, b = bd / g.D;
    const bool ok = x < g.W;
    const int xc = ok ? x : 0;
    const size_t P = (size_t)g.W * g.H;
    const float* src = in + (size_t)bd * P + xc;
    const uint32_t* arms = g.arms + (size_t)b * P + xc;
    const float* sc = (kScale ? scale : in) + (size_t)b * P + xc;
    float* dst = out + (size_t)bd * P + xc;
    for (int i = 0; i < kSoftRing; ++i) ring[i][t] = 0.0;
    double run = 0.0;
    int slot = 0;  // ring slot of row y
    for (int y0 = 0; y0 < g.H + kLMax; y0 += kSoftPre) {
        float v[kSoftPre];
        uint32_t a[kSoftPre];
        float s[kSoftPre];
#pragma unroll
        for (int k = 0; k < kSoftPre; ++k) {  // clamped rows: every load is unconditional
            const int y = y0 + k, yo = y - kLMax;
            const size_t yq = (size_t)min(y, g.H - 1), oq = (size_t)min(max(yo, 0), g.H - 1);
            v[k] = src[yq * g.W];
            a[k] = arms[yq * g.W];
            s[k] = kScale ? sc[oq * g.W] : 1.0f;
        }
#pragma unroll
        for (int k = 0; k < kSoftPre; ++k) {
            const int y = y0 + k, yo = y - kLMax;
            if (y < g.H) {  // uniform
                const int u = arm(a[k], 2), dn = arm(a[k], 3);
                int sa = slot - u, se = slot + dn + 1;
                sa += sa < 0 ? kSoftRing : 0;
                se -= se >= kSoftRing ? kSoftRing : 0;
                ring[sa][t] += (double)v[k];
                ring[se][t] -= (double)v[k];
            }
            if (yo >= 0) {  // row yo is final: its slot is kLMax rows back
                int so = slot - kLMax;
                so += so < 0 ? kSoftRing : 0;
                run += ring[so][t];
                ring[so][t] = 0.0;  // reused for row yo + kSoftRing
                if (ok && yo < g.H) dst[(size_t)yo * g.W] = kScale ? (float)run / s[k] : (float)run;
            }
            slot = slot + 1 == kSoftRing ? 0 : slot + 1;
        }
    }
}


// Soft-argmin over d per pixel: dhat and lse (log-sum-exp of -A2/T).
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
    float m = -a[0] * invT;
    for (int d = 1; d < g.D; ++d) m = fmaxf(m, -a[(size_t)d * P] * invT);
    float z = 0.0f, zd = 0.0f;
    for (int d = 0; d < g.D; ++d) {
        const float e = expf(-a[(size_t)d * P] * invT - m);
        z += e;
        zd += (float)d * e;
    }
    dhat[(size_t)b * P + i] = zd / z;
    lse[(size_t)b * P + i] = m + logf(z);
}

// Backward seed: G(p,d) = g w (dhat - d) / (T N2), per-block partial sums of
// the T-gradient terms g w (d - dhat) A2 / T^2 (one partial per block).
__global__ __launch_bounds__(256) void k_soft_seed(SoftGeom g, const float* __restrict__ A2,
                                                   const float* __restrict__ theta,
                                                   const float* __restrict__ dhat,
                                                   const float* __restrict__ lse,
                                                   const float* __restrict__ gdhat,
                                                   float* __restrict__ G,
                                                   double* __restrict__ partT) {
    __shared__ double red[256];
    const size_t P = (size_t)g.W * g.H;
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    const int b = blockIdx.y;
    const float T = theta[2], invT = 1.0f / T;
    double acc = 0.0;
    if (i < P) {
        const size_t pi = (size_t)b * P + i;
        const float gp = gdhat[pi], dh = dhat[pi], l = lse[pi], n2 = g.n2[pi];
        for (int d = 0; d < g.D; ++d) {
            const size_t vi = ((size_t)b * g.D + d) * P + i;
            const float a2 = A2[vi];
            const float w = expf(-a2 * invT - l);
            G[vi] = gp * w * (dh - (float)d) * invT / n2;
            acc += (double)(gp * w * ((float)d - dh) * a2) * (double)(invT * invT);
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partT[(size_t)b * gridDim.x + blockIdx.x] = red[0];
}

// Adjoint of a row range sum: out(x') = sum over x with x' in [x - l(x), x + r(x)]
// of in(x).  The candidates are x in [x' - kLMax, x' + kLMax].

// Adjoint of a column range sum, then an optional per-pixel scale:
// out(x, y') = scale(x, y') * sum over y with y' in [y - u(y), y + dn(y)] of in(x, y).

// Last adjoint (row direction, onto the raw costs) fused with the lambda
// derivatives: per-block partial sums of G_c dc/dlambda_AD and G_c dc/dlambda_c.

// Final fixed-order reduction of the partial sums into grad_theta (float).
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
        if (threadIdx.x < s)
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
    hipLaunchKernelGGL(k_soft_counts, dim3((W + 63) / 64, (H + 3) / 4, B), dim3(256), 0, st, g, n1,
                       n2);
    return hipGetLastError();
}

// Forward aggregation into A2 (B x D x H x W); t1, t2 are volume-sized scratch.
hipError_t soft_aggregate(const SoftBuffers& s, int B, int W, int H, int D, float* A2, float* t1,
                          float* t2, hipStream_t st) {
    SoftGeom g{s.arms, s.n1, s.n2, B, W, H, D};
    SoftImg im{s.rgbL, s.rgbR, s.cenL, s.cenR, s.alpha, s.tab};
    const int nrows = B * D * H;
    const dim3 gr((nrows + kRowWaves * kRowsPerWave - 1) / (kRowWaves * kRowsPerWave));
    const size_t lf = row_lds_fwd(W);
    hipError_t e = allow_lds(reinterpret_cast<const void*>(&k_soft_hrow<true>), kRowWaves * lf);
    if (e == hipSuccess)
        e = allow_lds(reinterpret_cast<const void*>(&k_soft_hrow<false>), kRowWaves * lf);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_soft_hrow<true>, gr, dim3(64 * kRowWaves), kRowWaves * lf, st, g, im,
                       (const float*)nullptr, t1, lf);                                       // E1
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
    SoftImg im{s.rgbL, s.rgbR, s.cenL, s.cenR, s.alpha, s.tab};
    const size_t P = (size_t)W * H;
    const unsigned nb = (unsigned)((P + 255) / 256);
    hipLaunchKernelGGL(k_soft_seed, dim3(nb, B), dim3(256), 0, st, g, A2, theta, dhat, lse, gdhat,
                       t1, partT);                                              // G_A2 / N2
    const int nrows = B * D * H;
    const dim3 gr((nrows + kRowWaves * kRowsPerWave - 1) / (kRowWaves * kRowsPerWave));
    const size_t la = row_lds_adj(W);
    hipError_t e = allow_lds(reinterpret_cast<const void*>(&k_soft_hrow_adj<false>), kRowWaves * la);
    if (e == hipSuccess)
        e = allow_lds(reinterpret_cast<const void*>(&k_soft_hrow_adj<true>), kRowWaves * la);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_soft_hrow_adj<false>, gr, dim3(64 * kRowWaves), kRowWaves * la, st, g, im,
                       t1, t2, (double*)nullptr, la);                         // G_E2
    const dim3 gv((W + kSoftCols - 1) / kSoftCols, B * D);
    hipLaunchKernelGGL(k_soft_vsa<true>, gv, dim3(kSoftCols), 0, st, g, t2, s.n1, t1);  // G_a1/N1
    hipLaunchKernelGGL(k_soft_vsa<false>, gv, dim3(kSoftCols), 0, st, g, t1,
                       (const float*)nullptr, t2);                                    // G_E1
    hipLaunchKernelGGL(k_soft_hrow_adj<true>, gr, dim3(64 * kRowWaves), kRowWaves * la, st, g, im,
                       t2, (float*)nullptr, partAC, la);                      // G_c . dc/dlambda
    double* blk = partT + (size_t)B * nb;  // kRedBlocks x 3 after the block partials
    hipLaunchKernelGGL(k_soft_reduce1, dim3(kRedBlocks), dim3(256), 0, st, partAC,
                       (size_t)B * D * H, partT, (size_t)B * nb, blk);
    hipLaunchKernelGGL(k_soft_reduce2, dim3(1), dim3(256), 0, st, blk, grad);
    return hipGetLastError();
}
