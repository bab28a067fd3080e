// k_aggregate.hip -- aggregation over the adaptive cross region (Eq. 2),
// applied as two stages, in exact integer arithmetic: one workgroup per
// (disparity slice, column strip) streaming down the rows.  With kFused the
// raw cost of Eq. 1 is computed on the fly from the images and census codes
// (the one-call matcher) instead of being read from a cost volume (the
// staged dco_aggregate).  The stage body (dco::agg_stream) lives in
// dco_device.h.
#include "dco_device.h"

namespace {

template <int ITERS, bool kFused>
__global__ __launch_bounds__(kStripThreads, 2) void k_agg_stream(dco::AggArgs A) {
    __shared__ dco::AggLds<ITERS, kFused> S;
    // strip-major items, consecutive per XCD: the workgroups one XCD runs at
    // a time share a strip (its records and reference pixels) and read
    // overlapping partner columns, so most loads hit that XCD's L2
    const int work = dco::xcd_work_item(blockIdx.x, A.nstrips * A.D);
    const int strip = work / A.D, d = work - strip * A.D;
    dco::agg_stream<ITERS, kFused>(A, d, strip, 0, A.H, S);
}

template <int ITERS, bool kFused>
hipError_t launch_stream(const dco::AggArgs& a, hipStream_t st) {
    const int nblk = a.nstrips * a.D;
    hipLaunchKernelGGL((k_agg_stream<ITERS, kFused>), dim3(nblk), dim3(kStripThreads), 0, st, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_aggregate(const float* cost, const AggRecords& rec, int W, int H, int D,
                            int iters, float* out, hipStream_t st) {
    dco::AggArgs a{};
    a.cost = cost;
    a.rec = rec;
    a.out = out;
    a.W = W;
    a.H = H;
    a.D = D;
    a.nstrips = (W + kStripOut - 1) / kStripOut;
    return iters == 1 ? launch_stream<1, false>(a, st) : launch_stream<2, false>(a, st);
}

hipError_t launch_cost_aggregate(int ref, const uint4* pixL, const uint4* pixR,
                                 const AggRecords& rec, int W, int H, int D, int iters,
                                 const float* tabA, const float* tabC, const float* alpha,
                                 const float* beta, int L1, float* out, hipStream_t st) {
    dco::AggArgs a{};
    a.pixL = pixL;
    a.pixR = pixR;
    a.tabA = tabA;
    a.tabC = tabC;
    a.alpha = alpha;
    a.beta = beta;
    a.rec = rec;
    a.out = out;
    a.W = W;
    a.H = H;
    a.D = D;
    a.ref = ref;
    a.L1 = L1;
    a.nstrips = (W + kStripOut - 1) / kStripOut;
    return iters == 1 ? launch_stream<1, true>(a, st) : launch_stream<2, true>(a, st);
}
