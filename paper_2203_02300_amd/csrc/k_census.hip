// k_census.hip -- census codes and cross-support arms of one image
// (Sec. 4.1; the C_census term of Eq. 1), and the per-pixel region counts and
// aggregation records.  The stage bodies live in dco_device.h.
#include "dco_device.h"

namespace {

__global__ __launch_bounds__(256) void k_census_arms(const uint8_t* __restrict__ rgb, int W,
                                                     int H, int cw, int ch, int L1, int tau1,
                                                     uint64_t* __restrict__ census,
                                                     uint32_t* __restrict__ arms,
                                                     uint32_t* __restrict__ rgb_packed,
                                                     uint4* __restrict__ pix) {
    __shared__ dco::CensusLds S;
    dco::census_tile(rgb, W, H, cw, ch, L1, tau1, census, arms, rgb_packed, pix,
                     blockIdx.x * dco::kCenTW, blockIdx.y * dco::kCenTH, S);
}

__global__ __launch_bounds__(256) void k_geometry(const uint32_t* __restrict__ arms, int W, int H,
                                                  int iters, AggRecords rec) {
    __shared__ dco::GeomLds S;
    dco::geometry_tile(arms, W, H, iters, rec, blockIdx.x * dco::kGeoTW, blockIdx.y * dco::kGeoTH,
                       S);
}

}  // namespace

hipError_t launch_census_arms(const uint8_t* rgb, int W, int H, int cw, int ch, int L1, int tau1,
                              uint64_t* census, uint32_t* arms, uint32_t* rgb_packed, uint4* pix,
                              hipStream_t st) {
    dim3 grid((W + dco::kCenTW - 1) / dco::kCenTW, (H + dco::kCenTH - 1) / dco::kCenTH);
    hipLaunchKernelGGL(k_census_arms, grid, dim3(256), 0, st, rgb, W, H, cw, ch, L1, tau1, census,
                       arms, rgb_packed, pix);
    return hipGetLastError();
}

hipError_t launch_geometry(const uint32_t* arms, int W, int H, int iters, const AggRecords& rec,
                           hipStream_t st) {
    dim3 grid((W + dco::kGeoTW - 1) / dco::kGeoTW, (H + dco::kGeoTH - 1) / dco::kGeoTH);
    hipLaunchKernelGGL(k_geometry, grid, dim3(256), 0, st, arms, W, H, iters, rec);
    return hipGetLastError();
}
