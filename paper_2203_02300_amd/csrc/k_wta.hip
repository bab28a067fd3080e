// k_wta.hip -- winner-take-all over the aggregated volume (Eq. 3) with
// parabola sub-pixel refinement, and the left-right consistency check.
//
// One thread per pixel walks d = 0 .. D-1 (loads of one slice are coalesced
// across the block) keeping the running minimum, its predecessor value and
// its successor value, so the volume is read exactly once.  Ties keep the
// smallest d.  All float operations follow the order stated in the ABI.
#include "dco_internal.h"

namespace {

__global__ __launch_bounds__(256) void k_wta(const float* __restrict__ aggL,
                                             const float* __restrict__ aggR, int P, int D,
                                             int subpixel, int16_t* __restrict__ dL,
                                             float* __restrict__ deltaL,
                                             int16_t* __restrict__ dR) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int view = blockIdx.y;
    if (i >= P) return;
    const float* agg = view == 0 ? aggL : aggR;
    float best = agg[i], prev = best, m = 0.f, pl = 0.f;
    int bd = 0;
    constexpr int U = 8;
    int d = 1;
    for (; d + U <= D; d += U) {
        float v[U];
#pragma unroll
        for (int k = 0; k < U; ++k) v[k] = agg[(size_t)(d + k) * P + i];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            if (d + k == bd + 1) pl = v[k];
            if (v[k] < best) {
                best = v[k];
                bd = d + k;
                m = prev;
            }
            prev = v[k];
        }
    }
    for (; d < D; ++d) {
        const float v = agg[(size_t)d * P + i];
        if (d == bd + 1) pl = v;
        if (v < best) {
            best = v;
            bd = d;
            m = prev;
        }
        prev = v;
    }
    if (view == 0) {
        float del = 0.f;
        if (subpixel && bd > 0 && bd < D - 1) {
            const float num = m - pl;
            const float den = (m - best) + (pl - best);
            if (den > 0.f) {
                del = num / (2.0f * den);
                del = fminf(fmaxf(del, -0.5f), 0.5f);
            }
        }
        dL[i] = (int16_t)bd;
        deltaL[i] = del;
    } else {
        dR[i] = (int16_t)bd;
    }
}

__global__ __launch_bounds__(256) void k_lrcheck(const int16_t* __restrict__ dL,
                                                 const float* __restrict__ deltaL,
                                                 const int16_t* __restrict__ dR, int W, int H,
                                                 int maxdiff, float* __restrict__ disp,
                                                 uint8_t* __restrict__ valid) {
    const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
    if (x >= W) return;
    const size_t i = (size_t)y * W + x;
    const int dl = dL[i];
    const int xr = x - dl;
    const bool ok = xr >= 0 && abs(dl - (int)dR[(size_t)y * W + xr]) <= maxdiff;
    valid[i] = ok ? 1 : 0;
    disp[i] = ok ? (float)dl + deltaL[i] : 0.0f;
}

}  // namespace

hipError_t launch_wta2(const float* aggL, const float* aggR, int W, int H, int D, int subpixel,
                       int16_t* dL, float* deltaL, int16_t* dR, hipStream_t st) {
    const int P = W * H;
    dim3 grid((P + 255) / 256, 2);
    hipLaunchKernelGGL(k_wta, grid, dim3(256), 0, st, aggL, aggR, P, D, subpixel, dL, deltaL, dR);
    return hipGetLastError();
}

hipError_t launch_lrcheck(const int16_t* dL, const float* deltaL, const int16_t* dR, int W,
                          int H, int maxdiff, float* disp, uint8_t* valid, hipStream_t st) {
    dim3 grid((W + 255) / 256, H);
    hipLaunchKernelGGL(k_lrcheck, grid, dim3(256), 0, st, dL, deltaL, dR, W, H, maxdiff, disp,
                       valid);
    return hipGetLastError();
}
