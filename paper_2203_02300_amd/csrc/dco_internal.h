// dco_internal.h -- shared declarations of the gfx950 stereo library (not
// part of the ABI).  Host code and kernels include it; the CPU oracle never
// does.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>

#include <vector>

#include "../../include/dco_stereo.h"

#include "dco_layout.h"

constexpr int kVoteMaxIters = 64;  // passes of one Eq. 4 vote call

// Scratch owned by a matcher handle for the one-call path.
struct dco_scratch {
    uint32_t* arms[2];
    AggRecords rec[2];
    uint4* pix[2];      // packed pixels of both views: census lo, census hi, RGB, 8 L_min
    float* agg[2];      // aggregated volumes of both views (D x H x W)
    bool agg_paired;    // ... written in the paired layout (two-stage aggregation)
    int16_t* dint[2];
    float* delta;
    int16_t* vote[2];   // ping-pong maps of the Eq. 4 vote passes
    uint8_t* half[2];   // the reduced pair of dco_stereo_match_half (H x W x 3)
};

// Soft-path scratch of a handle: per-pair maps of B pairs and three
// B x D x H x W float volumes (grown on demand).
struct SoftScratch {
    int cap;               // pairs the buffers hold
    uint4* pix[2];         // packed pixels of left / right views (census lo, census
                           // hi, RGB, 8 L_min)
    uint32_t* arms;        // arms of the left views
    uint32_t* arms_r;      // arms of the right views (computed, unused)
    float* n1;             // region counts
    float* n2;
    float* tab;            // Eq. 1 tables and derivatives for the current theta
    float* vol[3];
    double* partAC;        // per-row partial sums of the lambda gradients
    double* partT;         // per-row partial sums of the temperature gradient, then
                           // 3 x 256 block totals of the final reduction
    // The inputs whose costs and aggregation the buffers above hold (set by
    // the last complete aggregation, cleared when the buffers change): B, the
    // device pointers L, R, theta and the stream it ran on.
    bool held;
    int held_B;
    const void* held_L;
    const void* held_R;
    const void* held_theta;
    hipStream_t held_stream;
};

// Read-only view of the soft-path inputs handed to the kernels.
struct SoftBuffers {
    const uint32_t* arms;
    const float* n1;
    const float* n2;
    const uint4* pixL;
    const uint4* pixR;
    const float* alpha;
    const float* tab;
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
    SoftScratch soft;
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

#define DCO_TRY(expr)                \
    do {                             \
        dco_status _s = (expr);      \
        if (_s != DCO_OK) return _s; \
    } while (0)

// Allocation-failure injection and accounting (testing hooks of the ABI):
// dco_debug_fail_alloc(k), or DCO_FAIL_ALLOC=k in the environment when the
// library loads, makes the k-th device or pinned allocation from then on
// fail as if memory were exhausted; every allocation and free made through
// the helpers below is counted, so a test can check that an error path
// frees exactly what it allocated.
bool alloc_fault_injected();
void alloc_count(int delta);

// hipMalloc of n elements with the library's error reporting.
template <class T>
inline dco_status dev_alloc(T** p, size_t n) {
    *p = nullptr;
    if (n == 0) return DCO_OK;
    if (alloc_fault_injected()) {
        dco_set_error("allocation of %zu bytes refused (injected failure)", n * sizeof(T));
        return DCO_ERR_OOM;
    }
    hipError_t e = hipMalloc((void**)p, n * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        dco_set_error("hipMalloc(%zu) failed: %s", n * sizeof(T), hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? DCO_ERR_OOM : DCO_ERR_HIP;
    }
    alloc_count(1);
    return DCO_OK;
}

// hipFree of a dev_alloc pointer (nullptr is ignored).
inline void dev_free(void* p) {
    if (!p) return;
    (void)hipFree(p);
    alloc_count(-1);
}

// Pinned host memory of `bytes` bytes, counted like device memory.
inline dco_status pinned_alloc(void** p, size_t bytes) {
    *p = nullptr;
    if (alloc_fault_injected() || hipHostMalloc(p, bytes, hipHostMallocDefault) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        dco_set_error("pinned allocation of %zu bytes failed", bytes);
        return DCO_ERR_OOM;
    }
    alloc_count(1);
    return DCO_OK;
}

inline void pinned_free(void* p) {
    if (!p) return;
    (void)hipHostFree(p);
    alloc_count(-1);
}

// ---- host helpers shared by api.cpp and batch.cpp ----
dco_status need(const void* ptr, const char* what);
dco_status need_align(const void* ptr, size_t a, const char* what);
dco_status check_params(const dco_params& p);
dco_status check_shape(int W, int H, int D, const dco_params& p);
void build_tables_into(const dco_params& p, float* tabA, float* tabC, float* alpha, float* beta);
void build_tables(const dco_params& p, std::vector<float>& tabA, std::vector<float>& tabC,
                  std::vector<float>& alpha, std::vector<float>& beta);
dco_status alloc_records(AggRecords* r, int W, int H);

// ---- kernel launchers (one per .hip file) ----
// census, rgb_packed (R | G << 8 | B << 16) and pix (census lo, census hi,
// packed RGB, 8 L_min) are optional outputs
hipError_t launch_census_arms(const uint8_t* rgb, int W, int H, int cw, int ch, int L1, int tau1,
                              uint64_t* census, uint32_t* arms, uint32_t* rgb_packed, uint4* pix,
                              hipStream_t st);
// Eq. 4 vote: `iters` passes (>= 1) over the left integer map dL (pixels
// with valid = 0 or a value outside [0, D) do not vote), ping-ponging between
// buf0 and buf1 (H x W int16 each); *result points at the final map (-1 where
// invalid).  Then the output step: disp / valid from a voted map (valid_in
// null) or from dL and its mask (no pass).
hipError_t launch_vote(const int16_t* dL, const uint8_t* valid, const uint32_t* arms, int W, int H,
                       int D, int iters, int16_t* buf0, int16_t* buf1, const int16_t** result,
                       hipStream_t st);
hipError_t launch_vote_finish(const int16_t* dv, const uint8_t* valid_in, const float* agg,
                              bool paired, int W, int H, int D, int subpixel, float* disp,
                              uint8_t* valid, int16_t* dv_out, hipStream_t st);
// Quarter-size front end: 2 x 2 block means of both full images (row length
// W2 pixels) into W x H x 3 outputs; then disp = 2 disp where valid (else 0)
// in place, and depth = fB / disp where > 0 (depth optional).
hipError_t launch_downscale2(const uint8_t* rgbL, const uint8_t* rgbR, int W2, int W, int H,
                             uint8_t* outL, uint8_t* outR, hipStream_t st);
hipError_t launch_depth_half(float* disp, const uint8_t* valid, int W, int H, float fB,
                             float* depth, hipStream_t st);
// Depth densification (Eq. 13-20): device buffers of one grid (FP64 state,
// nblk = densify_blocks(W, H) block partials per sum) and its launches.
struct DensifyBufs {
    double *cr, *cd, *diag, *invdiag;  // edge coefficients (p, p + x), (p, p + y); diagonal
    double *x, *r, *q, *p[2];          // solution, residual, A p, search directions
    double *rz[2], *rr[2], *pq, *bb;   // block partial sums
    int* flags;                        // [0] converged, [1] iterations done
};
int densify_blocks(int W, int H);
hipError_t launch_densify_setup(const DensifyBufs& b, const float* Ds, const float* Dpre,
                                const uint8_t* Bdp, const float* Mfuse, const float* MI, int W,
                                int H, double lam_d, double lam_s, double lam_s2, hipStream_t st);
hipError_t launch_densify_iters(const DensifyBufs& b, int W, int H, double tol, int n,
                                hipStream_t st);
hipError_t launch_densify_out(const DensifyBufs& b, int W, int H, float* D, hipStream_t st);

// Depth contour extraction given the flows (Sec. 5): scratch of one frame
// (full size W x H, flow grid w x h) and its launches.
constexpr int kContourMaxSlots = 64;  // slots of the contour kernels' block maxima
struct ContourBufs {
    float* fused;        // w x h: Eq. 12 before the box filter
    unsigned* box_max;   // largest box mean (float bits), kContourMaxSlots partial maxima
    int* g2_max;         // largest G2, kContourMaxSlots partial maxima
    short2* g;           // W x H Sobel gradients
    int* G2;             // W x H squared magnitudes
    uint8_t* state[2];   // W x H: 0 none, 1 weak, 2 strong (hysteresis ping-pong)
    int* changed;        // kHystGroup flags: set by a hysteresis launch that changed a pixel
};
hipError_t launch_contour_maps(const float* past, const float* future, int w, int h, int R,
                               const uint8_t* rgb, int W, int H, float Thigh, float Tlow,
                               float Tdepth, const ContourBufs& b, float* Mn, float* MI,
                               hipStream_t st);
// Hysteresis launches go in groups of kHystGroup with one host check per
// group: launch k of a group does nothing once launch k - 1 changed nothing.
constexpr int kHystGroup = 4;
hipError_t launch_contour_hyst_group(const ContourBufs& b, int W, int H, int parity,
                                     hipStream_t st);
hipError_t launch_contour_edges(const ContourBufs& b, int W, int H, int parity, uint8_t* B,
                                hipStream_t st);
// Arms and packed pixels of both views of B pairs (HWC images of 3 W H
// bytes each, outputs of W H entries each, pair-major) in one launch.
hipError_t launch_census_pairs(const uint8_t* rgbL, const uint8_t* rgbR, int B, int W, int H,
                               int cw, int ch, int L1, int tau1, uint32_t* armsL, uint32_t* armsR,
                               uint4* pixL, uint4* pixR, hipStream_t st);
// Census + arms + packed pixels, then region counts + records, of both views
// (the one-call path): two launches.  The records address the LDS of the
// aggregation kernel that launch_cost_aggregate2 runs (pair_rec_geom).
hipError_t launch_front2(const uint8_t* rgbL, const uint8_t* rgbR, int W, int H, int cw, int ch,
                         int L1, int tau1, int iters, uint32_t* armsL, uint32_t* armsR,
                         uint4* pixL, uint4* pixR, const AggRecords& recL, const AggRecords& recR,
                         const RecGeom& g, hipStream_t st);
RecGeom pair_rec_geom(int iters);
// Records for the aggregation kernels; g = pair_rec_geom(iters) for the
// kernels of dco_aggregate and dco_stereo_match.
hipError_t launch_geometry(const uint32_t* arms, int W, int H, int iters, const AggRecords& rec,
                           const RecGeom& g, hipStream_t st);
hipError_t launch_cost(int ref, const uint8_t* rgbL, const uint8_t* rgbR, const uint64_t* cenL,
                       const uint64_t* cenR, const uint32_t* arms_ref, int W, int H, int D,
                       const float* tabA, const float* tabC, const float* alpha,
                       const float* beta, int L1, float* cost, hipStream_t st);
hipError_t launch_aggregate(const float* cost, const AggRecords& rec, int W, int H, int D,
                            int iters, float* out, hipStream_t st);
// Both views in one launch (the one-call path).  With two stages and
// `paired`, the volumes are written in the paired layout (dco::paired_at);
// with one stage they are always plain.
hipError_t launch_cost_aggregate2(const uint4* pixL, const uint4* pixR, const AggRecords& recL,
                                  const AggRecords& recR, int W, int H, int D, int iters,
                                  const float* tabA, const float* tabC, const float* alpha,
                                  const float* beta, int L1, float* outL, float* outR,
                                  bool paired, hipStream_t st);
hipError_t launch_cost_aggregate(int ref, const uint4* pixL, const uint4* pixR,
                                 const AggRecords& rec, int W, int H, int D, int iters,
                                 const float* tabA, const float* tabC, const float* alpha,
                                 const float* beta, int L1, float* out, hipStream_t st);
hipError_t launch_wta2(const float* aggL, const float* aggR, int W, int H, int D, int subpixel,
                       int16_t* dL, float* deltaL, int16_t* dR, hipStream_t st);
// The same outputs from volumes in the paired layout (even slices only).
hipError_t launch_wta_pairs(const float* aggL, const float* aggR, int W, int H, int D,
                            int subpixel, int16_t* dL, float* deltaL, int16_t* dR,
                            hipStream_t st);
// Slices d0 .. d0 + n - 1 of a paired-layout volume, decoded into out (n x H x W).
hipError_t launch_unpair(const float* vol, int W, int H, int D, int d0, int n, float* out,
                         hipStream_t st);
hipError_t launch_lrcheck(const int16_t* dL, const float* deltaL, const int16_t* dR, int W,
                          int H, int maxdiff, float* disp, uint8_t* valid, hipStream_t st);

// k_soft.hip
hipError_t soft_prepare(const float* theta, float* tab, const uint32_t* arms, int B, int W, int H,
                        int D, float* n1, float* n2, hipStream_t st);
hipError_t soft_aggregate(const SoftBuffers& s, int B, int W, int H, int D, float* A2, float* t1,
                          float* t2, hipStream_t st);
hipError_t soft_argmin(const SoftBuffers& s, int B, int W, int H, int D, const float* A2,
                       const float* theta, float* dhat, float* lse, hipStream_t st);
hipError_t soft_backward(const SoftBuffers& s, int B, int W, int H, int D, const float* A2,
                         const float* theta, const float* dhat, const float* lse,
                         const float* gdhat, float* t1, float* t2, double* partAC,
                         double* partT, float* grad, hipStream_t st);
