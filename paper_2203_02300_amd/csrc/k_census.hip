// k_census.hip -- census codes and cross-support arms of one image
// (Sec. 4.1; the C_census term of Eq. 1), and the per-pixel region counts and
// aggregation records.  The stage bodies live in dco_device.h.
#include "dco_device.h"

namespace {

// One thread per pixel of a tile (1024 threads, at most 64 VGPRs so that two
// workgroups share a CU).
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8))) void k_census_arms(
    const uint8_t* __restrict__ rgb, int W, int H, int cw, int ch, int L1, int tau1,
    uint64_t* __restrict__ census, uint32_t* __restrict__ arms, uint32_t* __restrict__ rgb_packed,
    uint4* __restrict__ pix) {
    __shared__ dco::CensusLds S;
    dco::census_tile<1024>(rgb, W, H, cw, ch, L1, tau1, census, arms, rgb_packed, pix,
                           blockIdx.x * dco::kCenTW, blockIdx.y * dco::kCenTH, S);
}

__global__ __launch_bounds__(1024) void k_geometry(const uint32_t* __restrict__ arms, int W, int H,
                                                   int iters, AggRecords rec, RecGeom g) {
    __shared__ dco::GeomLds S;
    dco::geometry_tile<1024>(arms, W, H, iters, rec, blockIdx.x * dco::kGeoTW,
                             blockIdx.y * dco::kGeoTH, S, g);
}

// Both views of the one-call path in one launch each (blockIdx.z = view);
// one thread per pixel of a tile.
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8))) void k_census_arms2(
    const uint8_t* __restrict__ rgbL, const uint8_t* __restrict__ rgbR, int W, int H, int cw,
    int ch, int L1, int tau1, uint32_t* __restrict__ armsL, uint32_t* __restrict__ armsR,
    uint4* __restrict__ pixL, uint4* __restrict__ pixR) {
    __shared__ dco::CensusLds S;
    const bool r = blockIdx.z != 0;
    dco::census_tile<1024>(r ? rgbR : rgbL, W, H, cw, ch, L1, tau1, nullptr, r ? armsR : armsL,
                           nullptr, r ? pixR : pixL, blockIdx.x * dco::kCenTW,
                           blockIdx.y * dco::kCenTH, S);
}

__global__ __launch_bounds__(1024) void k_geometry2(const uint32_t* __restrict__ armsL,
                                                   const uint32_t* __restrict__ armsR, int W,
                                                   int H, int iters, AggRecords recL,
                                                   AggRecords recR, RecGeom g) {
    __shared__ dco::GeomLds S;
    const bool r = blockIdx.z != 0;
    dco::geometry_tile<1024>(r ? armsR : armsL, W, H, iters, r ? recR : recL,
                             blockIdx.x * dco::kGeoTW, blockIdx.y * dco::kGeoTH, S, g);
}

// Every view of a batch of pairs in one launch (blockIdx.z = 2 * pair + view),
// for the soft path: arms and packed pixels; one thread per pixel of a tile.
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8))) void k_census_pairs(
    const uint8_t* __restrict__ rgbL, const uint8_t* __restrict__ rgbR, int W, int H, int cw,
    int ch, int L1, int tau1, uint32_t* __restrict__ armsL, uint32_t* __restrict__ armsR,
    uint4* __restrict__ pixL, uint4* __restrict__ pixR) {
    __shared__ dco::CensusLds S;
    const bool r = (blockIdx.z & 1) != 0;
    const size_t P = (size_t)W * H, o = P * (blockIdx.z >> 1);
    dco::census_tile<1024>((r ? rgbR : rgbL) + 3 * o, W, H, cw, ch, L1, tau1, nullptr,
                           (r ? armsR : armsL) + o, nullptr, (r ? pixR : pixL) + o,
                           blockIdx.x * dco::kCenTW, blockIdx.y * dco::kCenTH, S);
}

}  // namespace

hipError_t launch_census_pairs(const uint8_t* rgbL, const uint8_t* rgbR, int B, int W, int H,
                               int cw, int ch, int L1, int tau1, uint32_t* armsL, uint32_t* armsR,
                               uint4* pixL, uint4* pixR, hipStream_t st) {
    const size_t P = (size_t)W * H;
    constexpr int kMaxPairs = 16384;  // keeps gridDim.z = 2 * pairs within the launch limit
    for (int b0 = 0; b0 < B; b0 += kMaxPairs) {
        const int nb = B - b0 < kMaxPairs ? B - b0 : kMaxPairs;
        const size_t o = P * b0;
        dim3 g((W + dco::kCenTW - 1) / dco::kCenTW, (H + dco::kCenTH - 1) / dco::kCenTH, 2 * nb);
        hipLaunchKernelGGL(k_census_pairs, g, dim3(1024), 0, st, rgbL + 3 * o, rgbR + 3 * o, W, H,
                           cw, ch, L1, tau1, armsL + o, armsR + o, pixL + o, pixR + o);
    }
    return hipGetLastError();
}

hipError_t launch_front2(const uint8_t* rgbL, const uint8_t* rgbR, int W, int H, int cw, int ch,
                         int L1, int tau1, int iters, uint32_t* armsL, uint32_t* armsR,
                         uint4* pixL, uint4* pixR, const AggRecords& recL, const AggRecords& recR,
                         const RecGeom& g, hipStream_t st) {
    dim3 g1((W + dco::kCenTW - 1) / dco::kCenTW, (H + dco::kCenTH - 1) / dco::kCenTH, 2);
    hipLaunchKernelGGL(k_census_arms2, g1, dim3(1024), 0, st, rgbL, rgbR, W, H, cw, ch, L1, tau1,
                       armsL, armsR, pixL, pixR);
    dim3 g2((W + dco::kGeoTW - 1) / dco::kGeoTW, (H + dco::kGeoTH - 1) / dco::kGeoTH, 2);
    hipLaunchKernelGGL(k_geometry2, g2, dim3(1024), 0, st, armsL, armsR, W, H, iters, recL, recR,
                       g);
    return hipGetLastError();
}

hipError_t launch_census_arms(const uint8_t* rgb, int W, int H, int cw, int ch, int L1, int tau1,
                              uint64_t* census, uint32_t* arms, uint32_t* rgb_packed, uint4* pix,
                              hipStream_t st) {
    dim3 grid((W + dco::kCenTW - 1) / dco::kCenTW, (H + dco::kCenTH - 1) / dco::kCenTH);
    hipLaunchKernelGGL(k_census_arms, grid, dim3(1024), 0, st, rgb, W, H, cw, ch, L1, tau1, census,
                       arms, rgb_packed, pix);
    return hipGetLastError();
}

hipError_t launch_geometry(const uint32_t* arms, int W, int H, int iters, const AggRecords& rec,
                           const RecGeom& g, hipStream_t st) {
    dim3 grid((W + dco::kGeoTW - 1) / dco::kGeoTW, (H + dco::kGeoTH - 1) / dco::kGeoTH);
    hipLaunchKernelGGL(k_geometry, grid, dim3(1024), 0, st, arms, W, H, iters, rec, g);
    return hipGetLastError();
}
