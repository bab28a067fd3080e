// k_half.hip -- the quarter-size front end (Sec. 4.4): the pair is reduced
// to half width and half height before matching, and the disparity found
// there is doubled and turned into depth.
#include "dco_internal.h"

namespace {

// Both views in one launch (blockIdx.y = view): out pixel (x, y) channel c =
// (sum of the 2 x 2 input block + 2) >> 2.  One thread per output byte, so
// the three channels of a pixel are three consecutive threads.
__global__ __launch_bounds__(256) void k_downscale2(const uint8_t* __restrict__ rgbL,
                                                    const uint8_t* __restrict__ rgbR, int W2,
                                                    int W, int H, uint8_t* __restrict__ outL,
                                                    uint8_t* __restrict__ outR) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= 3 * W * H) return;
    const bool r = blockIdx.y != 0;
    const uint8_t* in = r ? rgbR : rgbL;
    const int px = i / 3, c = i - 3 * px;
    const int y = px / W, x = px - y * W;
    const size_t row0 = (size_t)(2 * y) * W2, row1 = row0 + W2;
    const int s = in[(row0 + 2 * x) * 3 + c] + in[(row0 + 2 * x + 1) * 3 + c] +
                  in[(row1 + 2 * x) * 3 + c] + in[(row1 + 2 * x + 1) * 3 + c];
    (r ? outR : outL)[i] = (uint8_t)((s + 2) >> 2);
}

// disp (in place) = 2 disp where valid, else 0; depth = fB / disp where that
// is > 0, else 0 (optional).
__global__ __launch_bounds__(256) void k_depth_half(float* __restrict__ disp,
                                                    const uint8_t* __restrict__ valid, int P,
                                                    float fB, float* __restrict__ depth) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= P) return;
    const float d2 = valid[i] ? 2.0f * disp[i] : 0.0f;
    disp[i] = d2;
    if (depth) depth[i] = d2 > 0.0f ? fB / d2 : 0.0f;
}

}  // namespace

hipError_t launch_downscale2(const uint8_t* rgbL, const uint8_t* rgbR, int W2, int W, int H,
                             uint8_t* outL, uint8_t* outR, hipStream_t st) {
    const int n = 3 * W * H;
    hipLaunchKernelGGL(k_downscale2, dim3((n + 255) / 256, 2), dim3(256), 0, st, rgbL, rgbR, W2, W,
                       H, outL, outR);
    return hipGetLastError();
}

hipError_t launch_depth_half(float* disp, const uint8_t* valid, int W, int H, float fB,
                             float* depth, hipStream_t st) {
    const int P = W * H;
    hipLaunchKernelGGL(k_depth_half, dim3((P + 255) / 256), dim3(256), 0, st, disp, valid, P, fB,
                       depth);
    return hipGetLastError();
}
