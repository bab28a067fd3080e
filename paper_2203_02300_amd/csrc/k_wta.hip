// k_wta.hip -- winner-take-all over the aggregated volumes (Eq. 3) with
// parabola sub-pixel refinement, and the left-right consistency check.
// k_wta_pairs* take the same decision on volumes in the paired layout
// (dco::paired_at): they read only the even slices; for the sub-pixel step
// they gather the winner's pair partner and, when it is not the adjacent
// pair's minimum kept from the scan, its other neighbour.
// One thread per pixel (or per four pixels, with 16-byte loads, when W * H is
// a multiple of four) walks d = 0 .. D-1; loads of one slice are coalesced
// across the block, so each volume is read exactly once.  The stage bodies
// live in dco_device.h.
#include "dco_device.h"

namespace {

__global__ __launch_bounds__(256) void k_wta(const float* __restrict__ aggL,
                                             const float* __restrict__ aggR, int P, int D,
                                             int subpixel, int16_t* __restrict__ dL,
                                             float* __restrict__ deltaL,
                                             int16_t* __restrict__ dR) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= P) return;
    if (blockIdx.y == 0)
        dco::wta_pixel(aggL, P, D, i, subpixel, dL + i, deltaL + i);
    else
        dco::wta_pixel(aggR, P, D, i, subpixel, dR + i, nullptr);
}

__global__ __launch_bounds__(256) void k_wta4(const float* __restrict__ aggL,
                                              const float* __restrict__ aggR, int P, int D,
                                              int subpixel, int16_t* __restrict__ dL,
                                              float* __restrict__ deltaL,
                                              int16_t* __restrict__ dR) {
    const int i4 = (blockIdx.x * 256 + threadIdx.x) * 4;
    if (i4 >= P) return;
    if (blockIdx.y == 0)
        dco::wta_quad(aggL, P, D, i4, subpixel, dL, deltaL);
    else
        dco::wta_quad(aggR, P, D, i4, subpixel, dR, nullptr);
}

__global__ __launch_bounds__(256) void k_wta_pairs(const float* __restrict__ aggL,
                                                   const float* __restrict__ aggR, int P, int D,
                                                   int subpixel, int16_t* __restrict__ dL,
                                                   float* __restrict__ deltaL,
                                                   int16_t* __restrict__ dR) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= P) return;
    if (blockIdx.y == 0)
        dco::wta_pairs_pixel(aggL, P, D, i, subpixel, dL + i, deltaL + i);
    else
        dco::wta_pairs_pixel(aggR, P, D, i, subpixel, dR + i, nullptr);
}

__global__ __launch_bounds__(256) void k_wta_pairs4(const float* __restrict__ aggL,
                                                    const float* __restrict__ aggR, int P, int D,
                                                    int subpixel, int16_t* __restrict__ dL,
                                                    float* __restrict__ deltaL,
                                                    int16_t* __restrict__ dR) {
    const int i4 = (blockIdx.x * 256 + threadIdx.x) * 4;
    if (i4 >= P) return;
    if (blockIdx.y == 0)
        dco::wta_pairs_quad<true>(aggL, P, D, i4, subpixel, dL, deltaL);
    else
        dco::wta_pairs_quad<false>(aggR, P, D, i4, subpixel, dR, nullptr);
}

// Slices d0 .. d0 + n - 1 of a paired-layout volume, decoded to n x P.
__global__ __launch_bounds__(256) void k_unpair(const float* __restrict__ vol, int P, int D,
                                                int d0, int n, float* __restrict__ out) {
    const size_t k = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= (size_t)n * P) return;
    const int s = (int)(k / P), i = (int)(k - (size_t)s * P);
    out[k] = dco::paired_at(vol, P, D, d0 + s, i);
}

__global__ __launch_bounds__(256) void k_lrcheck(const int16_t* __restrict__ dL,
                                                 const float* __restrict__ deltaL,
                                                 const int16_t* __restrict__ dR, int W, int H,
                                                 int maxdiff, float* __restrict__ disp,
                                                 uint8_t* __restrict__ valid) {
    const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
    if (x < W) dco::lr_pixel(dL, deltaL, dR, W, x, y, maxdiff, disp, valid);
}

}  // namespace

hipError_t launch_wta2(const float* aggL, const float* aggR, int W, int H, int D, int subpixel,
                       int16_t* dL, float* deltaL, int16_t* dR, hipStream_t st) {
    const int P = W * H;
    const bool aligned = ((uintptr_t)aggL | (uintptr_t)aggR | (uintptr_t)deltaL) % 16 == 0 &&
                         ((uintptr_t)dL | (uintptr_t)dR) % 8 == 0;
    if (P % 4 == 0 && aligned) {
        dim3 grid((P / 4 + 255) / 256, 2);
        hipLaunchKernelGGL(k_wta4, grid, dim3(256), 0, st, aggL, aggR, P, D, subpixel, dL, deltaL,
                           dR);
    } else {
        dim3 grid((P + 255) / 256, 2);
        hipLaunchKernelGGL(k_wta, grid, dim3(256), 0, st, aggL, aggR, P, D, subpixel, dL, deltaL,
                           dR);
    }
    return hipGetLastError();
}

hipError_t launch_wta_pairs(const float* aggL, const float* aggR, int W, int H, int D,
                            int subpixel, int16_t* dL, float* deltaL, int16_t* dR,
                            hipStream_t st) {
    const int P = W * H;
    const bool aligned = ((uintptr_t)aggL | (uintptr_t)aggR | (uintptr_t)deltaL) % 16 == 0 &&
                         ((uintptr_t)dL | (uintptr_t)dR) % 8 == 0;
    if (P % 4 == 0 && aligned) {
        dim3 grid((P / 4 + 255) / 256, 2);
        hipLaunchKernelGGL(k_wta_pairs4, grid, dim3(256), 0, st, aggL, aggR, P, D, subpixel, dL,
                           deltaL, dR);
    } else {
        dim3 grid((P + 255) / 256, 2);
        hipLaunchKernelGGL(k_wta_pairs, grid, dim3(256), 0, st, aggL, aggR, P, D, subpixel, dL,
                           deltaL, dR);
    }
    return hipGetLastError();
}

hipError_t launch_unpair(const float* vol, int W, int H, int D, int d0, int n, float* out,
                         hipStream_t st) {
    const size_t total = (size_t)n * W * H;
    hipLaunchKernelGGL(k_unpair, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, vol,
                       W * H, D, d0, n, out);
    return hipGetLastError();
}

hipError_t launch_lrcheck(const int16_t* dL, const float* deltaL, const int16_t* dR, int W,
                          int H, int maxdiff, float* disp, uint8_t* valid, hipStream_t st) {
    dim3 grid((W + 255) / 256, H);
    hipLaunchKernelGGL(k_lrcheck, grid, dim3(256), 0, st, dL, deltaL, dR, W, H, maxdiff, disp,
                       valid);
    return hipGetLastError();
}
