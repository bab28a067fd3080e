// k_cost.hip -- raw AD-census cost volume of one reference view (Eq. 1) in
// fixed point: q = rint(alpha_L * TA[s] * 2^20) + rint(beta_L * TC[h] * 2^20),
// each term rounded once from the exact product of its float factors, stored
// as q * 2^-20.
//
// One workgroup = one image row, 256 consecutive reference pixels and a chunk
// of kDC disparities.  The partner row segment those pixels can reach (packed
// RGB and census codes) is staged in LDS together with the two lookup tables,
// so the inner loop is: one SAD of packed bytes (v_sad_u8), two popcounts,
// two table reads, two fused multiply-adds that round the products to
// integers, one store.
// Stores are coalesced along x for each d.
#include "dco_device.h"

namespace {

constexpr int kDC = 32;

__global__ __launch_bounds__(256) void k_cost(int ref, const uint8_t* __restrict__ rgbL,
                                              const uint8_t* __restrict__ rgbR,
                                              const uint64_t* __restrict__ cenL,
                                              const uint64_t* __restrict__ cenR,
                                              const uint32_t* __restrict__ arms, int W, int H,
                                              int D, const float* __restrict__ tabA,
                                              const float* __restrict__ tabC,
                                              const float* __restrict__ alpha,
                                              const float* __restrict__ beta,
                                              float* __restrict__ cost) {
    __shared__ float s_tabA[768];
    __shared__ float s_tabC[65];
    __shared__ uint32_t s_prgb[256 + kDC];
    __shared__ uint64_t s_pcen[256 + kDC];

    const int t = threadIdx.x;
    const int x0 = blockIdx.x * 256, y = blockIdx.y, d0 = blockIdx.z * kDC;
    const uint8_t* Iref = ref == 0 ? rgbL : rgbR;
    const uint8_t* Ipar = ref == 0 ? rgbR : rgbL;
    const uint64_t* Cref = ref == 0 ? cenL : cenR;
    const uint64_t* Cpar = ref == 0 ? cenR : cenL;

    for (int i = t; i < 766; i += 256) s_tabA[i] = tabA[i];
    if (t < 65) s_tabC[t] = tabC[t];
    // partner columns: base .. base + 256 + kDC - 2
    const int base = ref == 0 ? x0 - d0 - (kDC - 1) : x0 + d0;
    for (int i = t; i < 256 + kDC - 1; i += 256) {
        int xp = base + i;
        uint32_t c = 0;
        uint64_t cc = 0;
        if (xp >= 0 && xp < W) {
            const uint8_t* p = Ipar + 3 * ((size_t)y * W + xp);
            c = (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16);
            cc = Cpar[(size_t)y * W + xp];
        }
        s_prgb[i] = c;
        s_pcen[i] = cc;
    }
    __syncthreads();

    const int x = x0 + t;
    if (x >= W) return;
    const size_t pix = (size_t)y * W + x;
    const uint8_t* pr = Iref + 3 * pix;
    const uint32_t crgb = (uint32_t)pr[0] | ((uint32_t)pr[1] << 8) | ((uint32_t)pr[2] << 16);
    const uint64_t ccen = Cref[pix];
    const uint32_t a = arms[pix];
    const int lmin = min(min((int)(a & 0xff), (int)((a >> 8) & 0xff)),
                         min((int)((a >> 16) & 0xff), (int)(a >> 24)));
    const float al = alpha[min(lmin, kLMax)], be = beta[min(lmin, kLMax)];
    const size_t slice = (size_t)W * H;
    const int dend = min(D, d0 + kDC);
    for (int d = d0; d < dend; ++d) {
        const int xo = ref == 0 ? x - d : x + d;
        float v = 1.0f;
        if (xo >= 0 && xo < W) {
            const int i = xo - base;
            const uint32_t s = __builtin_amdgcn_sad_u8(crgb, s_prgb[i], 0u);
            const uint64_t xr = ccen ^ s_pcen[i];
            const int h = __popcll(xr);
            v = (float)(dco::q20_term(al, s_tabA[s]) + dco::q20_term(be, s_tabC[h])) * 0x1p-20f;
        }
        cost[(size_t)d * slice + pix] = v;
    }
}

}  // namespace

hipError_t launch_cost(int ref, const uint8_t* rgbL, const uint8_t* rgbR, const uint64_t* cenL,
                       const uint64_t* cenR, const uint32_t* arms_ref, int W, int H, int D,
                       const float* tabA, const float* tabC, const float* alpha,
                       const float* beta, int L1, float* cost, hipStream_t st) {
    (void)L1;
    dim3 grid((W + 255) / 256, H, (D + kDC - 1) / kDC);
    hipLaunchKernelGGL(k_cost, grid, dim3(256), 0, st, ref, rgbL, rgbR, cenL, cenR, arms_ref, W,
                       H, D, tabA, tabC, alpha, beta, cost);
    return hipGetLastError();
}
