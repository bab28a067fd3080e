// k_noalloc.hip -- the one-call match with every intermediate buffer in a
// static device array: dco_stereo_match_noalloc allocates no device or host
// memory, so callers that may not allocate (stream capture into a HIP graph,
// serving loops, harnesses that forbid it) can run the whole matcher.
//
// The array `scratch` is file-scope device memory of kStaticScratchBytes.
// Each GPU the library runs this entry point on holds its own copy until the
// process ends.  Host code never uses the array's name as an address: the
// first call on a device (with that device current) asks the runtime for the
// device address of that GPU's copy with hipGetSymbolAddress and keeps it;
// every kernel argument below is derived from that address.
//
// Every call on one GPU shares the array and leaves its contents behind:
// calls that overlap on one GPU (two streams, or two threads) race and must
// be serialised by the caller.  What must start at zero (the aprons of the
// aggregation records) is cleared by a fill kernel at the start of each call.
#include <mutex>

#include "dco_device.h"

namespace {

// 160 MiB: the paper's operating point, a 640 x 360 pair with D = 64 and two
// vote passes, needs about 152 MB (both 59 MB aggregated volumes, the
// records, the packed pixels and the disparity maps).
constexpr size_t kStaticScratchBytes = size_t(160) << 20;

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices];  // device address of `scratch` on each device, once known

// Eq. 1 tables passed by value: the host builds them in double precision
// exactly as dco_stereo_create does, and a kernel stores them in the
// scratch, so no host-to-device copy (and no pinned buffer) is needed.
struct TabA {
    float v[768];
};
struct TabRest {
    float c[65];
    float alpha[kLMax + 1];
    float beta[kLMax + 1];
};

__global__ __launch_bounds__(256) void k_put_tab_a(TabA t, float* __restrict__ dst) {
    for (int i = threadIdx.x; i < 768; i += 256) dst[i] = t.v[i];
}

__global__ __launch_bounds__(128) void k_put_tab_rest(TabRest t, float* __restrict__ tabC,
                                                      float* __restrict__ alpha,
                                                      float* __restrict__ beta) {
    const int i = threadIdx.x;
    if (i < 65) tabC[i] = t.c[i];
    if (i <= kLMax) {
        alpha[i] = t.alpha[i];
        beta[i] = t.beta[i];
    }
}

// Zero n 16-byte words (a fill kernel rather than a memset, so the call can
// be captured into a graph).
__global__ __launch_bounds__(256) void k_zero16(uint4* __restrict__ p, size_t n) {
    const uint4 z = make_uint4(0u, 0u, 0u, 0u);
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
        p[i] = z;
}

// Carves the scratch into the one-call path's buffers (256-byte aligned).
struct Carve {
    unsigned char* base;
    size_t used;
    template <typename T>
    T* take(size_t n) {
        used = (used + 255) & ~size_t(255);
        T* p = base ? reinterpret_cast<T*>(base + used) : nullptr;
        used += n * sizeof(T);
        return p;
    }
};

struct StaticBufs {
    float *tabA, *tabC, *alpha, *beta;
    uint4* pix[2];
    uint32_t* arms[2];
    AggRecords rec[2];
    size_t rec_words[2][2];  // 4-word entries of b and c
    float* agg[2];
    int16_t* dint[2];
    float* delta;
    int16_t* vote[2];
};

// Layout of the buffers for a W x H pair with D disparities; with base ==
// nullptr only the size is computed.
size_t layout(unsigned char* base, int W, int H, int D, StaticBufs& b) {
    const size_t P = (size_t)W * H, V = P * D;
    Carve c{base, 0};
    b.tabA = c.take<float>(768);
    b.tabC = c.take<float>(68);
    b.alpha = c.take<float>(kLMax + 1);
    b.beta = c.take<float>(kLMax + 1);
    for (int v = 0; v < 2; ++v) {
        b.pix[v] = c.take<uint4>(P);
        b.arms[v] = c.take<uint32_t>(P);
        AggRecords& r = b.rec[v];
        r.apron = kRecApronL;
        r.Wp = W + kRecApronL + kRecApronR;
        b.rec_words[v][0] = (size_t)r.Wp * (H + kLMax + 1);
        b.rec_words[v][1] = (size_t)r.Wp * (H + 1);
        r.b = c.take<uint32_t>(4 * b.rec_words[v][0]);
        r.c = c.take<uint32_t>(4 * b.rec_words[v][1]);
        b.agg[v] = c.take<float>(V);
        b.dint[v] = c.take<int16_t>(P);
        b.vote[v] = c.take<int16_t>(P);
    }
    b.delta = c.take<float>(P);
    return (c.used + 255) & ~size_t(255);
}

// Device address of this device's `scratch`, asked once per device.
dco_status scratch_ptr(unsigned char** out) {
    int dev = 0;
    DCO_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        dco_set_error("device %d is beyond the %d devices the static scratch tracks", dev,
                      kMaxDevices);
        return DCO_ERR_ARG;
    }
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            dco_set_error("hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                          hipGetErrorString(e));
            return DCO_ERR_HIP;
        }
        g_ptr[dev] = p;
    }
    *out = static_cast<unsigned char*>(g_ptr[dev]);
    return DCO_OK;
}

}  // namespace

extern "C" dco_status dco_stereo_match_noalloc(int W, int H, int D, const dco_params* params,
                                               void* stream, const uint8_t* rgbL,
                                               const uint8_t* rgbR, float* disp,
                                               uint8_t* valid) {
    dco_params p;
    if (params)
        p = *params;
    else
        dco_default_params(&p);
    DCO_TRY(check_params(p));
    DCO_TRY(check_shape(W, H, D, p));
    DCO_TRY(need(rgbL, "rgbL"));
    DCO_TRY(need(rgbR, "rgbR"));
    DCO_TRY(need(disp, "disp"));
    DCO_TRY(need(valid, "valid"));
    StaticBufs b{};
    const size_t need_bytes = layout(nullptr, W, H, D, b);
    if (need_bytes > kStaticScratchBytes) {
        dco_set_error("dco_stereo_match_noalloc: W=%d H=%d D=%d needs %zu bytes of static "
                      "scratch, %zu available (up to 640 x 360 with D = 64)",
                      W, H, D, need_bytes, kStaticScratchBytes);
        return DCO_ERR_SHAPE;
    }
    unsigned char* base = nullptr;
    DCO_TRY(scratch_ptr(&base));
    layout(base, W, H, D, b);
    const hipStream_t st = (hipStream_t)stream;

    // Eq. 1 tables, built on the host the same way as for a handle (into
    // the kernel arguments: no host allocation either)
    TabA ta;
    TabRest tr;
    build_tables_into(p, ta.v, tr.c, tr.alpha, tr.beta);
    hipLaunchKernelGGL(k_put_tab_a, dim3(1), dim3(256), 0, st, ta, b.tabA);
    hipLaunchKernelGGL(k_put_tab_rest, dim3(1), dim3(128), 0, st, tr, b.tabC, b.alpha, b.beta);
    DCO_HIP_CHECK(hipGetLastError());
    // the records' aprons and their first and last rows must read as zero
    for (int v = 0; v < 2; ++v)
        for (int k = 0; k < 2; ++k) {
            uint4* r = reinterpret_cast<uint4*>(k ? b.rec[v].c : b.rec[v].b);
            hipLaunchKernelGGL(k_zero16, dim3(1024), dim3(256), 0, st, r, b.rec_words[v][k]);
        }
    DCO_HIP_CHECK(hipGetLastError());

    // the same kernel sequence as dco_stereo_match
    DCO_HIP_CHECK(launch_front2(rgbL, rgbR, W, H, p.census_w, p.census_h, p.arm_L1, p.arm_tau1,
                                p.agg_iters, b.arms[0], b.arms[1], b.pix[0], b.pix[1], b.rec[0],
                                b.rec[1], pair_rec_geom(p.agg_iters), st));
    DCO_HIP_CHECK(launch_cost_aggregate2(b.pix[0], b.pix[1], b.rec[0], b.rec[1], W, H, D,
                                         p.agg_iters, b.tabA, b.tabC, b.alpha, b.beta, p.arm_L1,
                                         b.agg[0], b.agg[1], true, st));
    const bool paired = p.agg_iters == 2;
    if (paired)
        DCO_HIP_CHECK(launch_wta_pairs(b.agg[0], b.agg[1], W, H, D, p.subpixel, b.dint[0],
                                       b.delta, b.dint[1], st));
    else
        DCO_HIP_CHECK(launch_wta2(b.agg[0], b.agg[1], W, H, D, p.subpixel, b.dint[0], b.delta,
                                  b.dint[1], st));
    DCO_HIP_CHECK(launch_lrcheck(b.dint[0], b.delta, b.dint[1], W, H, p.lr_max_diff, disp, valid,
                                 st));
    if (p.vote_iters > 0) {
        const int16_t* dv = nullptr;
        DCO_HIP_CHECK(launch_vote(b.dint[0], valid, b.arms[0], W, H, D, p.vote_iters, b.vote[0],
                                  b.vote[1], &dv, st));
        DCO_HIP_CHECK(launch_vote_finish(dv, nullptr, b.agg[0], paired, W, H, D, p.subpixel, disp,
                                         valid, nullptr, st));
    }
    return DCO_OK;
}
