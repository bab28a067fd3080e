// k_batch.hip -- the batched matcher's kernels: one persistent work-list
// kernel per stage, all five captured in one HIP graph.
//
// The host builds a work list ordered by stage (0 census + arms of a 64 x 64
// block, 1 region counts and records of a 64 x 64 block, 2 cost +
// aggregation of d-chunk x column strip x row band, cut into one contiguous
// part per XCD and ordered longest first within it, 3 WTA of a pixel block,
// 4 LR check of a row block) over every pair of the batch.  The kernels of
// stages 0, 1, 3 and 4 run a grid sized to the GPU's resident capacity;
// workgroup w takes the stage's items w, w + G, w + 2G, ...  Stage 2 runs one
// workgroup per item.  The kernel boundary is the barrier between stages, so
// workgroups never wait on each other and need no atomics.
//
// Each stage runs the same device function as the one-call matcher
// (dco_device.h), so per-pair results are bit-identical to dco_stereo_match.
#include <type_traits>

#include "dco_batch.h"
#include "dco_device.h"

namespace {

struct NoLds {
    int unused;
};

// Stage 2 with two aggregation stages: slices a .. a + dchunk - 1 of strip b,
// row band c, two adjacent disparities per pass of dco::agg_stream_ws (512
// threads, one workgroup per CU).  The workgroups of XCD x take that XCD's
// contiguous part of the list, one item each.
__global__ __launch_bounds__(dco::kWsThreads, 1) void k_batch_agg_ws(BatchArgs B, int first) {
    __shared__ dco::AggLdsWs S;
    const int x = blockIdx.x % kXcds;
    const int k = B.xsplit[x] - first + blockIdx.x / kXcds;
    if (k >= B.xsplit[x + 1] - first) return;  // uniform
    const BatchItem I = B.items[first + k];
    const BatchPair& pr = B.pairs[I.pair];
    dco::AggArgs A{};
    A.pixL = pr.pix[0];
    A.pixR = pr.pix[1];
    A.tabA = B.tabA;
    A.tabC = B.tabC;
    A.alpha = B.alpha;
    A.beta = B.beta;
    A.rec = pr.rec[I.view];
    A.out = pr.agg[I.view];
    A.W = pr.W;
    A.H = pr.H;
    A.D = pr.D;
    A.nstrips = pr.nstrips;
    A.ref = I.view;
    A.L1 = B.L1;
    // with an even chunk every pass starts at an even slice, so the passes'
    // slice pairs are the layout's pairs; stage 3 reads the even slices
    A.paired = pr.dchunk % 2 == 0;
    const int y0 = I.c * pr.band, y1 = min(pr.H, y0 + pr.band);
    const int dend = min(pr.D, I.a + pr.dchunk);
    for (int d = I.a; d < dend; d += dco::kWsSlices) {
        dco::agg_stream_ws(A, d, dend, I.b, y0, y1, S);
        __syncthreads();
    }
}

// Stages 0 and 1 with one thread per pixel of a tile (1024 threads), the
// same tiles as the one-call front end: census + arms + packed pixels, then
// region counts and records, of 64 x 64 blocks; persistent over the items.
template <int ITERS, int STAGE>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8))) void k_batch_front(
    BatchArgs B, int first, int count) {
    __shared__ typename std::conditional<STAGE == 0, dco::CensusLds, dco::GeomLds>::type S;
    for (int k = blockIdx.x; k < count; k += gridDim.x) {
        const BatchItem I = B.items[first + k];
        const BatchPair& pr = B.pairs[I.pair];
        const int W = pr.W, H = pr.H;
        if constexpr (STAGE == 0) {
            const uint8_t* img = I.view == 0 ? B.io[I.pair].L : B.io[I.pair].R;
            for (int r = 0; r < 64 / dco::kCenTH; ++r) {
                const int y0 = I.b * 64 + r * dco::kCenTH;
                if (y0 >= H) break;
                dco::census_tile<1024>(img, W, H, B.cw, B.ch, B.L1, B.tau1, nullptr,
                                       pr.arms[I.view], nullptr, pr.pix[I.view],
                                       I.a * dco::kCenTW, y0, S);
                __syncthreads();
            }
        } else {
            for (int r = 0; r < 64 / dco::kGeoTH; ++r) {
                const int y0 = I.b * 64 + r * dco::kGeoTH;
                if (y0 >= H) break;
                dco::geometry_tile<1024>(pr.arms[I.view], W, H, ITERS, pr.rec[I.view],
                                         I.a * dco::kGeoTW, y0, S,
                                         ITERS == 2 ? dco::kRecWs : dco::kRecPlain);
                __syncthreads();
            }
        }
    }
}

// LDS of stages 2 (one aggregation stage), 3 and 4: aggregation rings or none.
template <int ITERS, int STAGE>
using StageLds =
    typename std::conditional<STAGE == 2, dco::AggLds<ITERS, true>, NoLds>::type;

template <int ITERS, int STAGE>
__global__ __launch_bounds__(256, 2) void k_batch_stage(BatchArgs B, int first, int count) {
    __shared__ StageLds<ITERS, STAGE> S;
    const int t = threadIdx.x;
    // stage 2: one item per workgroup, the workgroups of XCD x (blockIdx %
    // kXcds, dispatched in order) taking that XCD's contiguous part of the
    // list, so the hardware dispatcher balances the items; the other stages
    // are persistent and stride over the whole list
    int k0 = blockIdx.x, kend = count, kstep = gridDim.x;
    if (STAGE == 2) {
        const int x = blockIdx.x % kXcds;
        k0 = B.xsplit[x] - first + blockIdx.x / kXcds;
        kend = min(B.xsplit[x + 1] - first, k0 + 1);
        kstep = 1;
    }
    for (int k = k0; k < kend; k += kstep) {
        const BatchItem I = B.items[first + k];
        const BatchPair& pr = B.pairs[I.pair];
        const BatchIO& io = B.io[I.pair];
        const int W = pr.W, H = pr.H;
        if constexpr (STAGE == 2) {  // slices a .. a+dchunk-1, strip b, row band c
            dco::AggArgs A{};
            A.pixL = pr.pix[0];
            A.pixR = pr.pix[1];
            A.tabA = B.tabA;
            A.tabC = B.tabC;
            A.alpha = B.alpha;
            A.beta = B.beta;
            A.rec = pr.rec[I.view];
            A.out = pr.agg[I.view];
            A.W = W;
            A.H = H;
            A.D = pr.D;
            A.nstrips = pr.nstrips;
            A.ref = I.view;
            A.L1 = B.L1;
            const int y0 = I.c * pr.band, y1 = min(H, y0 + pr.band);
            const int dend = min(pr.D, I.a + pr.dchunk);
            for (int d = I.a; d < dend; ++d) {
                dco::agg_stream<ITERS, true>(A, d, I.b, y0, y1, S);
                __syncthreads();
            }
        } else if constexpr (STAGE == 3) {  // WTA of both views for pixels [a, a + kWtaPx)
            // two stages with an even chunk write the volumes in the paired
            // layout (even slices hold each pair's minimum), else plain
            const int P = W * H;
            const bool paired = ITERS == 2 && pr.dchunk % 2 == 0;
            if (P % 4 == 0) {  // 16-byte loads (the pair's buffers are 256-byte aligned)
                for (int r = 0; r < kWtaPx / 1024; ++r) {
                    const int i4 = I.a + (r * 256 + t) * 4;
                    if (i4 >= P) break;
                    if (paired) {
                        dco::wta_pairs_quad<true>(pr.agg[0], P, pr.D, i4, B.subpixel,
                                                  pr.dint[0], pr.delta);
                        dco::wta_pairs_quad<false>(pr.agg[1], P, pr.D, i4, B.subpixel,
                                                   pr.dint[1], nullptr);
                    } else {
                        dco::wta_quad(pr.agg[0], P, pr.D, i4, B.subpixel, pr.dint[0], pr.delta);
                        dco::wta_quad(pr.agg[1], P, pr.D, i4, B.subpixel, pr.dint[1], nullptr);
                    }
                }
            } else {
                for (int r = 0; r < kWtaPx / 256; ++r) {
                    const int i = I.a + r * 256 + t;
                    if (i >= P) break;
                    if (paired) {
                        dco::wta_pairs_pixel(pr.agg[0], P, pr.D, i, B.subpixel, pr.dint[0] + i,
                                             pr.delta + i);
                        dco::wta_pairs_pixel(pr.agg[1], P, pr.D, i, B.subpixel, pr.dint[1] + i,
                                             nullptr);
                    } else {
                        dco::wta_pixel(pr.agg[0], P, pr.D, i, B.subpixel, pr.dint[0] + i,
                                       pr.delta + i);
                        dco::wta_pixel(pr.agg[1], P, pr.D, i, B.subpixel, pr.dint[1] + i,
                                       nullptr);
                    }
                }
            }
        } else {  // LR check of rows [a, a + kLrRows)
            for (int y = I.a; y < min(H, I.a + kLrRows); ++y)
                for (int x = t; x < W; x += 256)
                    dco::lr_pixel(pr.dint[0], pr.delta, pr.dint[1], W, x, y, B.maxdiff,
                                  io.disp, io.valid);
        }
        __syncthreads();
    }
}

template <int ITERS, int STAGE>
int stage_blocks_per_cu() {
    int nb = 0;
    hipError_t e =
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_stage<ITERS, STAGE>, 256, 0);
    return e == hipSuccess && nb > 0 ? nb : 1;
}

template <int ITERS>
hipError_t launch_all(const BatchArgs& a, const int* first, const int* grid, hipStream_t st) {
    hipLaunchKernelGGL((k_batch_front<ITERS, 0>), dim3(grid[0]), dim3(1024), 0, st, a, first[0],
                       first[1] - first[0]);
    hipLaunchKernelGGL((k_batch_front<ITERS, 1>), dim3(grid[1]), dim3(1024), 0, st, a, first[1],
                       first[2] - first[1]);
    if constexpr (ITERS == 2)
        hipLaunchKernelGGL(k_batch_agg_ws, dim3(grid[2]), dim3(dco::kWsThreads), 0, st, a,
                           first[2]);
    else
        hipLaunchKernelGGL((k_batch_stage<ITERS, 2>), dim3(grid[2]), dim3(256), 0, st, a,
                           first[2], first[3] - first[2]);
    hipLaunchKernelGGL((k_batch_stage<ITERS, 3>), dim3(grid[3]), dim3(256), 0, st, a, first[3],
                       first[4] - first[3]);
    hipLaunchKernelGGL((k_batch_stage<ITERS, 4>), dim3(grid[4]), dim3(256), 0, st, a, first[4],
                       first[5] - first[4]);
    return hipGetLastError();
}

template <int ITERS>
void blocks_per_cu(int* per_stage) {
    for (int k = 0; k < 2; ++k) {
        int nb = 0;
        const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, k ? k_batch_front<ITERS, 1> : k_batch_front<ITERS, 0>, 1024, 0);
        per_stage[k] = e == hipSuccess && nb > 0 ? nb : 1;
    }
    if constexpr (ITERS == 2) {
        int nb = 0;
        const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, k_batch_agg_ws, dco::kWsThreads, 0);
        per_stage[2] = e == hipSuccess && nb > 0 ? nb : 1;
    } else {
        per_stage[2] = stage_blocks_per_cu<ITERS, 2>();
    }
    per_stage[3] = stage_blocks_per_cu<ITERS, 3>();
    per_stage[4] = stage_blocks_per_cu<ITERS, 4>();
}

}  // namespace

hipError_t launch_batch(const BatchArgs& a, int iters, const int* first, const int* grid,
                        hipStream_t st) {
    return iters == 1 ? launch_all<1>(a, first, grid, st) : launch_all<2>(a, first, grid, st);
}

void batch_blocks_per_cu(int iters, int* per_stage) {
    if (iters == 1)
        blocks_per_cu<1>(per_stage);
    else
        blocks_per_cu<2>(per_stage);
}
