// k_aggregate.hip -- aggregation over the adaptive cross region (Eq. 2), in
// exact integer arithmetic, each workgroup streaming a column strip down the
// rows.  Two stages (the path's reading of Eq. 2): k_agg_pair_ws, two
// adjacent disparity slices per workgroup (dco::agg_stream_ws), with the raw
// cost of Eq. 1 computed on the fly for both views in one launch (the
// one-call matcher) or read from one view's cost volume (the staged
// dco_aggregate).  One stage: one slice per workgroup (dco::agg_stream,
// k_agg_stream for the staged call, k_agg_pair for the one-call matcher).
// The stage bodies live in dco_device.h.
#include <atomic>

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

// Blocks of XCD x in the two-view launch: its nx items (a contiguous,
// strip-major run), the last m = nx mod s8 of them split into a top and a
// bottom half, so that the final round of workgroups is one round of half
// items instead of a part-empty round of whole ones.  The top halves of the
// m items run before their bottom halves: workgroups resident together then
// walk the same rows of one strip, which the XCD's L2 serves once.
// s8 = resident workgroups per XCD.
__host__ __device__ inline void pair_part(int N, int x, int s8, int H, int& start, int& nx,
                                          int& m) {
    const int per = N / 8, rem = N % 8;
    nx = per + (x < rem ? 1 : 0);
    start = x * per + (x < rem ? x : rem);
    m = 0;
    if (H < 8 || s8 < 1) return;
    if (nx <= s8) {
        m = 2 * nx <= s8 ? nx : 0;
    } else {
        m = nx % s8;
    }
}

// Cost + two-stage aggregation of both views in one launch (one-call path).
// Items: view, then strip, then disparity (strip-major); each XCD runs a
// contiguous part of them.
template <int ITERS>
__global__ __launch_bounds__(kStripThreads, 2) void k_agg_pair(dco::AggArgs A0, AggRecords rec1,
                                                              float* out1, int s8) {
    __shared__ dco::AggLds<ITERS, true> S;
    const int per_view = A0.nstrips * A0.D, N = 2 * per_view;
    const int x = blockIdx.x % 8, i = blockIdx.x / 8;
    int start, nx, m;
    pair_part(N, x, s8, A0.H, start, nx, m);
    int item, y0 = 0, y1 = A0.H;
    if (i < nx - m) {
        item = start + i;
    } else {
        const int j = i - (nx - m);
        if (j >= 2 * m) return;  // uniform: the whole workgroup leaves
        item = start + nx - m + (j < m ? j : j - m);  // all top halves, then bottoms
        if (j >= m)
            y0 = A0.H / 2;
        else
            y1 = A0.H / 2;
    }
    const int view = item / per_view, rest = item - view * per_view;
    const int strip = rest / A0.D, d = rest - strip * A0.D;
    dco::AggArgs A = A0;  // left view; the right view differs in three fields
    if (view) {
        A.ref = 1;
        A.rec = rec1;
        A.out = out1;
    }
    dco::agg_stream<ITERS, true>(A, d, strip, y0, y1, S);
}

// Two stages: the same items with two adjacent disparities per item, one
// 512-thread workgroup per CU (dco::agg_stream_ws).  kFused: both views, the
// raw cost computed on the fly; else one view (nviews = 1) from its cost
// volume A0.cost (the staged dco_aggregate).
template <bool kFused>
__global__ __launch_bounds__(dco::kWsThreads, 1) void k_agg_pair_ws(dco::AggArgs A0,
                                                                    AggRecords rec1, float* out1,
                                                                    int s8, int nviews) {
    __shared__ dco::AggLdsWs S;
    const int groups = (A0.D + dco::kWsSlices - 1) / dco::kWsSlices;
    const int per_view = A0.nstrips * groups, N = nviews * per_view;
    const int x = blockIdx.x % 8, i = blockIdx.x / 8;
    int start, nx, m;
    pair_part(N, x, s8, A0.H, start, nx, m);
    int item, y0 = 0, y1 = A0.H;
    if (i < nx - m) {
        item = start + i;
    } else {
        const int j = i - (nx - m);
        if (j >= 2 * m) return;  // uniform: the whole workgroup leaves
        item = start + nx - m + (j < m ? j : j - m);  // all top halves, then bottoms
        if (j >= m)
            y0 = A0.H / 2;
        else
            y1 = A0.H / 2;
    }
    const int view = item / per_view, rest = item - view * per_view;
    const int strip = rest / groups, g = rest - strip * groups;
    dco::AggArgs A = A0;  // left view; the right view differs in three fields
    if (view) {
        A.ref = 1;
        A.rec = rec1;
        A.out = out1;
    }
    dco::agg_stream_ws<kFused>(A, g * dco::kWsSlices, A.D, strip, y0, y1, S);
}

// Resident workgroups per XCD of a kernel (queried once per device and
// kernel; concurrent first calls store the same value).
template <typename K>
hipError_t xcd_slots(K kernel, int threads, std::atomic<int>* slots, int* s8) {
    constexpr int kMaxDev = 64;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    int total = dev < kMaxDev ? slots[dev].load(std::memory_order_relaxed) : 0;
    if (!total) {
        int cus = 0, nb = 0;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, 0);
        if (e != hipSuccess) return e;
        total = (nb > 0 ? nb : 1) * (cus > 0 ? cus : 1);
        if (dev < kMaxDev) slots[dev].store(total, std::memory_order_relaxed);
    }
    *s8 = total / 8;
    return hipSuccess;
}

template <bool kFused>
hipError_t launch_pair_ws(const dco::AggArgs& a0, const AggRecords& rec1, float* out1, int nviews,
                          hipStream_t st) {
    static std::atomic<int> slots[64];
    int s8 = 0;
    hipError_t e = xcd_slots(k_agg_pair_ws<kFused>, dco::kWsThreads, slots, &s8);
    if (e != hipSuccess) return e;
    const int N = nviews * a0.nstrips * ((a0.D + dco::kWsSlices - 1) / dco::kWsSlices);
    int most = 1;
    for (int x = 0; x < 8; ++x) {
        int start, nx, m;
        pair_part(N, x, s8, a0.H, start, nx, m);
        most = nx + m > most ? nx + m : most;
    }
    hipLaunchKernelGGL(k_agg_pair_ws<kFused>, dim3(8 * most), dim3(dco::kWsThreads), 0, st, a0,
                       rec1, out1, s8, nviews);
    return hipGetLastError();
}

template <int ITERS>
hipError_t launch_pair(const dco::AggArgs& a0, const AggRecords& rec1, float* out1,
                       hipStream_t st) {
    // resident workgroups of the whole device, per device (queried once each;
    // concurrent first calls store the same value)
    constexpr int kMaxDev = 64;
    static std::atomic<int> slots[kMaxDev];
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    int total = dev < kMaxDev ? slots[dev].load(std::memory_order_relaxed) : 0;
    if (!total) {
        int cus = 0, nb = 0;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_agg_pair<ITERS>,
                                                             kStripThreads, 0);
        if (e != hipSuccess) return e;
        total = (nb > 0 ? nb : 1) * (cus > 0 ? cus : 1);
        if (dev < kMaxDev) slots[dev].store(total, std::memory_order_relaxed);
    }
    const int s8 = total / 8;
    const int N = 2 * a0.nstrips * a0.D;
    int most = 1;
    for (int x = 0; x < 8; ++x) {
        int start, nx, m;
        pair_part(N, x, s8, a0.H, start, nx, m);
        most = nx + m > most ? nx + m : most;
    }
    hipLaunchKernelGGL((k_agg_pair<ITERS>), dim3(8 * most), dim3(kStripThreads), 0, st, a0, rec1,
                       out1, s8);
    return hipGetLastError();
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
    // two stages: the two-slice kernel on the volume (records written with
    // kRecWs, plain slice order)
    return iters == 1 ? launch_stream<1, false>(a, st)
                      : launch_pair_ws<false>(a, rec, out, 1, st);
}

hipError_t launch_cost_aggregate2(const uint4* pixL, const uint4* pixR, const AggRecords& recL,
                                  const AggRecords& recR, int W, int H, int D, int iters,
                                  const float* tabA, const float* tabC, const float* alpha,
                                  const float* beta, int L1, float* outL, float* outR,
                                  bool paired, hipStream_t st) {
    dco::AggArgs a{};
    a.pixL = pixL;
    a.pixR = pixR;
    a.tabA = tabA;
    a.tabC = tabC;
    a.alpha = alpha;
    a.beta = beta;
    a.W = W;
    a.H = H;
    a.D = D;
    a.L1 = L1;
    a.nstrips = (W + kStripOut - 1) / kStripOut;
    a.ref = 0;
    a.rec = recL;
    a.out = outL;
    a.paired = paired && iters == 2;
    return iters == 1 ? launch_pair<1>(a, recR, outR, st)
                      : launch_pair_ws<true>(a, recR, outR, 2, st);
}

RecGeom pair_rec_geom(int iters) { return iters == 2 ? dco::kRecWs : dco::kRecPlain; }

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
