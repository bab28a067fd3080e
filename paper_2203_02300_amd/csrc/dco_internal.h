// dco_internal.h -- shared declarations of the gfx950 stereo library (not
// part of the ABI).  Host code and kernels include it; the CPU oracle never
// does.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/dco_stereo.h"

// Largest arm length the kernels are built for.  The aggregation halo is
// 2 * kLMax columns/rows on each side of an output pixel.
constexpr int kLMax = 17;
// Rows of column-prefix history one streaming column keeps: a vertical range
// [y - u - 1, y + dn] spans at most 2 * kLMax + 2 prefix rows.
constexpr int kRing = 2 * kLMax + 2;
// Threads of a streaming-aggregation workgroup = input columns of a strip.
constexpr int kStripThreads = 256;
// Output columns of one strip.
constexpr int kStripOut = kStripThreads - 4 * kLMax;
// Rows processed per block-scan round in the streaming kernels.
constexpr int kRowChunk = 8;

// Per-pixel division data for the aggregation (computed once per view).
//   div1: stage-1 rounding a1 = ((S1 + half) * m) >> sh, exact for
//         0 <= S1 + half < 2^31 and 1 <= N1 <= 2^11.
//   div2: (N as float, RN(1/N)) of the final float division.
struct DivInt {
    uint32_t m;
    uint32_t half_sh;  // half | (sh << 16)
};

struct dco_geometry {
    uint32_t* arms;   // packed arms: l | r << 8 | u << 16 | dn << 24  (H x W)
    DivInt* div1;     // stage-1 integer division data                (H x W)
    float2* div2;     // final float division data                    (H x W)
};

// Scratch owned by a matcher handle for the one-call path.
struct dco_scratch {
    uint64_t* cen[2];
    uint32_t* arms[2];
    DivInt* div1[2];
    float2* div2[2];
    uint32_t* rgbp[2];  // packed RGB of both views
    float* agg[2];      // aggregated volumes of both views (D x H x W)
    int16_t* dint[2];
    float* delta;
};

struct dco_stereo {
    int W, H, D;
    dco_params p;
    hipStream_t stream;
    int device;
    // Eq. 1 tables in device memory:
    //   tabA[s] = TA[s] * 2^20 (s = 0..765), tabC[h] = TC[h] * 2^20 (h = 0..64)
    //   alpha[L], beta[L] (L = 0..L1)
    float* tabA;
    float* tabC;
    float* alpha;
    float* beta;
    // float (unscaled) copies for the soft path
    float* alpha_soft;
    dco_scratch s;
    bool scratch_ready;
    // stage timing of dco_stereo_match (events[k] = start/stop pairs per stage)
    bool profiling;
    std::vector<hipEvent_t> prof_events;  // 2 * DCO_NUM_STAGES per recorded call
    size_t prof_used;
    // soft-path scratch (allocated on first use)
    float* soft_vol;
    size_t soft_vol_elems;
    double* soft_partials;
    size_t soft_partials_n;
};

// ---- error helpers (api.cpp) ----
void dco_set_error(const char* fmt, ...);
#define DCO_HIP_CHECK(expr)                                                        \
    do {                                                                           \
        hipError_t _e = (expr);                                                    \
        if (_e != hipSuccess) {                                                    \
            dco_set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e), \
                          __FILE__, __LINE__);                                     \
            return DCO_ERR_HIP;                                                    \
        }                                                                          \
    } while (0)

// ---- kernel launchers (one per .hip file) ----
hipError_t launch_census_arms(const uint8_t* rgb, int W, int H, int cw, int ch, int L1, int tau1,
                              uint64_t* census, uint32_t* arms, uint32_t* rgb_packed,
                              hipStream_t st);
hipError_t launch_geometry(const uint32_t* arms, int W, int H, int iters, DivInt* div1,
                           float2* div2, hipStream_t st);
hipError_t launch_cost(int ref, const uint8_t* rgbL, const uint8_t* rgbR, const uint64_t* cenL,
                       const uint64_t* cenR, const uint32_t* arms_ref, int W, int H, int D,
                       const float* tabA, const float* tabC, const float* alpha,
                       const float* beta, int L1, float* cost, hipStream_t st);
hipError_t launch_aggregate(const float* cost, const uint32_t* arms, const DivInt* div1,
                            const float2* div2, int W, int H, int D, int iters, float* out,
                            hipStream_t st);
hipError_t launch_cost_aggregate(int ref, const uint32_t* rgbL, const uint32_t* rgbR,
                                 const uint64_t* cenL, const uint64_t* cenR,
                                 const uint32_t* arms, const DivInt* div1, const float2* div2,
                                 int W, int H, int D, int iters, const float* tabA,
                                 const float* tabC, const float* alpha, const float* beta,
                                 int L1, float* out, hipStream_t st);
hipError_t launch_wta2(const float* aggL, const float* aggR, int W, int H, int D, int subpixel,
                       int16_t* dL, float* deltaL, int16_t* dR, hipStream_t st);
hipError_t launch_lrcheck(const int16_t* dL, const float* deltaL, const int16_t* dR, int W,
                          int H, int maxdiff, float* disp, uint8_t* valid, hipStream_t st);
