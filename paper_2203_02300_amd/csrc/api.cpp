// api.cpp -- host side of the C ABI declared in include/dco_stereo.h:
// argument validation, the matcher handle, the Eq. 1 lookup tables, scratch
// memory and the kernel sequence of each entry point.
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "dco_internal.h"

static thread_local char g_err[512] = "";

// Allocation-failure injection: allocations left before the one that fails
// (0 = none armed), and the count of live allocations.
static std::atomic<long> g_fail_countdown{[] {
    const char* v = getenv("DCO_FAIL_ALLOC");
    return v ? atol(v) : 0L;
}()};
static std::atomic<long> g_live_allocs{0};

bool alloc_fault_injected() {
    long v = g_fail_countdown.load(std::memory_order_relaxed);
    while (v > 0)
        if (g_fail_countdown.compare_exchange_weak(v, v - 1)) return v == 1;
    return false;
}

void alloc_count(int delta) { g_live_allocs.fetch_add(delta); }

extern "C" void dco_debug_fail_alloc(int k) { g_fail_countdown.store(k > 0 ? k : 0); }

extern "C" long dco_debug_live_allocations(void) { return g_live_allocs.load(); }

void dco_set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

extern "C" const char* dco_last_error(void) { return g_err; }

extern "C" const char* dco_status_string(dco_status s) {
    switch (s) {
        case DCO_OK: return "ok";
        case DCO_ERR_ARG: return "invalid argument";
        case DCO_ERR_SHAPE: return "invalid shape";
        case DCO_ERR_HIP: return "HIP runtime error";
        case DCO_ERR_OOM: return "out of device memory";
        case DCO_ERR_STATE: return "invalid handle state";
    }
    return "unknown status";
}

extern "C" dco_status dco_default_params(dco_params* out) {
    if (!out) {
        dco_set_error("dco_default_params: out is NULL");
        return DCO_ERR_ARG;
    }
    out->census_w = 9;
    out->census_h = 7;
    out->arm_L1 = 17;
    out->arm_tau1 = 20;
    out->lambda_ad = 10.0f;
    out->lambda_census = 40.0f;
    out->gamma_L = 1.0f;
    out->eps = 0.8f;
    out->agg_iters = 2;
    out->lr_max_diff = 0;
    out->subpixel = 1;
    out->vote_iters = 0;
    return DCO_OK;
}


static bool pos_finite(float v) { return std::isfinite(v) && v > 0.0f; }

dco_status check_params(const dco_params& p) {
    if (p.census_w < 1 || p.census_h < 1 || !(p.census_w & 1) || !(p.census_h & 1) ||
        p.census_w > 9 || p.census_h > 9 || p.census_w * p.census_h - 1 > 64) {
        dco_set_error("census window %d x %d: need odd sizes <= 9 with w*h-1 <= 64", p.census_w,
                      p.census_h);
        return DCO_ERR_ARG;
    }
    if (p.arm_L1 < 0 || p.arm_L1 > kLMax || p.arm_tau1 < 1 || p.arm_tau1 > 256) {
        dco_set_error("arms: need 0 <= L1 <= %d and 1 <= tau1 <= 256 (got %d, %d)", kLMax,
                      p.arm_L1, p.arm_tau1);
        return DCO_ERR_ARG;
    }
    if (!pos_finite(p.lambda_ad) || !pos_finite(p.lambda_census) || !pos_finite(p.gamma_L) ||
        !pos_finite(p.eps)) {
        dco_set_error("lambda_ad, lambda_census, gamma_L and eps must be finite and > 0");
        return DCO_ERR_ARG;
    }
    if (p.agg_iters != 1 && p.agg_iters != 2) {
        dco_set_error("agg_iters must be 1 or 2 (got %d)", p.agg_iters);
        return DCO_ERR_ARG;
    }
    if (p.lr_max_diff < 0 || (p.subpixel != 0 && p.subpixel != 1)) {
        dco_set_error("lr_max_diff must be >= 0 and subpixel 0 or 1");
        return DCO_ERR_ARG;
    }
    if (p.vote_iters < 0 || p.vote_iters > kVoteMaxIters) {
        dco_set_error("vote_iters must be in [0, %d] (got %d)", kVoteMaxIters, p.vote_iters);
        return DCO_ERR_ARG;
    }
    return DCO_OK;
}

// W * H <= 2^27 keeps every byte offset of the aggregation kernels' 32-bit
// buffer addressing in range (16-byte packed pixels, and 16-byte records
// over the padded width and H + kLMax + 1 rows).
dco_status check_shape(int W, int H, int D, const dco_params& p) {
    if (W < p.census_w || H < p.census_h || W > 16384 || H > 16384 || D < 1 || D >= W ||
        D > 32767 || (long long)W * H > (1LL << 27) || (long long)W * H * D >= (1LL << 31)) {
        dco_set_error("shape W=%d H=%d D=%d: need 1 <= D < W, W >= census_w, H >= census_h, "
                      "W, H <= 16384, W*H <= 2^27 and W*H*D < 2^31",
                      W, H, D);
        return DCO_ERR_SHAPE;
    }
    return DCO_OK;
}

// Eq. 1 tables, evaluated in double and rounded once to float.  The AD and
// census tables are stored scaled by 2^20 (an exact power-of-two scaling), so
// a kernel's alpha_L * tabA[s] equals RN(alpha_L * TA[s]) * 2^20.  Writes
// tabA[0..767] (765 used), tabC[0..64] and alpha, beta[0..kLMax].
void build_tables_into(const dco_params& p, float* tabA, float* tabC, float* alpha, float* beta) {
    for (int s = 0; s < 768; ++s) tabA[s] = 0.0f;
    const double g = p.gamma_L, e = p.eps, la = p.lambda_ad, lc = p.lambda_census;
    for (int L = 0; L <= kLMax; ++L) {
        const double w = std::exp(-g / ((double)L + e));
        alpha[L] = (float)(1.0 - w);
        beta[L] = (float)w;
    }
    for (int s = 0; s <= 765; ++s)
        tabA[s] = std::ldexp((float)(-std::expm1(-(double)s / (3.0 * la))), 20);
    for (int h = 0; h <= 64; ++h) tabC[h] = std::ldexp((float)(-std::expm1(-(double)h / lc)), 20);
}

void build_tables(const dco_params& p, std::vector<float>& tabA, std::vector<float>& tabC,
                  std::vector<float>& alpha, std::vector<float>& beta) {
    tabA.assign(768, 0.0f);
    tabC.assign(65, 0.0f);
    alpha.assign(kLMax + 1, 0.0f);
    beta.assign(kLMax + 1, 0.0f);
    build_tables_into(p, tabA.data(), tabC.data(), alpha.data(), beta.data());
}

static void free_handle_memory(dco_stereo* h) {
    void* ptrs[] = {h->tabA,         h->tabC,         h->alpha,        h->beta,
                    h->alpha_soft,   h->s.pix[0],     h->s.pix[1],     h->s.arms[0],
                    h->s.arms[1],    h->s.rec[0].b,   h->s.rec[0].c,
                    h->s.rec[1].b,   h->s.rec[1].c,
                    h->s.agg[0],     h->s.agg[1],     h->s.dint[0],
                    h->s.dint[1],    h->s.delta,      h->s.vote[0],    h->s.vote[1],
                    h->s.half[0],    h->s.half[1],
                    h->soft.pix[0],  h->soft.pix[1],
                    h->soft.arms,    h->soft.arms_r,  h->soft.n1,      h->soft.n2,
                    h->soft.tab,     h->soft.vol[0],  h->soft.vol[1],  h->soft.vol[2],
                    h->soft.partAC,  h->soft.partT};
    for (void* p : ptrs) dev_free(p);
}

// Aggregation records with a zero apron and a zero extra row (zeroed once:
// the geometry kernel writes only the interior).
dco_status alloc_records(AggRecords* r, int W, int H) {
    r->apron = kRecApronL;
    r->Wp = W + kRecApronL + kRecApronR;
    const size_t n = (size_t)r->Wp * (H + 1);
    const size_t nb = (size_t)r->Wp * (H + kLMax + 1);
    DCO_TRY(dev_alloc(&r->b, 4 * nb));
    DCO_TRY(dev_alloc(&r->c, 4 * n));
    DCO_HIP_CHECK(hipMemset(r->b, 0, 4 * nb * sizeof(uint32_t)));
    DCO_HIP_CHECK(hipMemset(r->c, 0, 4 * n * sizeof(uint32_t)));
    return DCO_OK;
}

static dco_status alloc_scratch(dco_stereo* h) {
    const size_t P = (size_t)h->W * h->H, V = P * h->D;
    dco_scratch& s = h->s;
    for (int v = 0; v < 2; ++v) {
        DCO_TRY(dev_alloc(&s.arms[v], P));
        DCO_TRY(alloc_records(&s.rec[v], h->W, h->H));
        DCO_TRY(dev_alloc(&s.pix[v], P));
        DCO_TRY(dev_alloc(&s.agg[v], V));
        DCO_TRY(dev_alloc(&s.dint[v], P));
    }
    DCO_TRY(dev_alloc(&s.delta, P));
    DCO_TRY(dev_alloc(&s.vote[0], P));
    DCO_TRY(dev_alloc(&s.vote[1], P));
    DCO_TRY(dev_alloc(&s.half[0], 3 * P));
    DCO_TRY(dev_alloc(&s.half[1], 3 * P));
    h->scratch_ready = true;
    return DCO_OK;
}

extern "C" dco_status dco_stereo_create(dco_stereo** out, int W, int H, int D,
                                        const dco_params* p, void* stream) {
    if (!out) {
        dco_set_error("dco_stereo_create: out is NULL");
        return DCO_ERR_ARG;
    }
    *out = nullptr;
    dco_params prm;
    if (p)
        prm = *p;
    else
        dco_default_params(&prm);
    DCO_TRY(check_params(prm));
    DCO_TRY(check_shape(W, H, D, prm));
    dco_stereo* h = new (std::nothrow) dco_stereo();
    if (!h) {
        dco_set_error("host allocation failed");
        return DCO_ERR_OOM;
    }
    h->W = W;
    h->H = H;
    h->D = D;
    h->p = prm;
    h->stream = (hipStream_t)stream;
    if (hipGetDevice(&h->device) != hipSuccess) {
        (void)hipGetLastError();
        delete h;
        dco_set_error("hipGetDevice failed: no usable GPU");
        return DCO_ERR_HIP;
    }
    std::vector<float> tabA, tabC, alpha, beta;
    build_tables(prm, tabA, tabC, alpha, beta);
    dco_status st = DCO_OK;
    auto fail = [&](dco_status s) {
        free_handle_memory(h);
        delete h;
        return s;
    };
    if ((st = dev_alloc(&h->tabA, tabA.size())) != DCO_OK) return fail(st);
    if ((st = dev_alloc(&h->tabC, tabC.size())) != DCO_OK) return fail(st);
    if ((st = dev_alloc(&h->alpha, alpha.size())) != DCO_OK) return fail(st);
    if ((st = dev_alloc(&h->beta, beta.size())) != DCO_OK) return fail(st);
    struct {
        float* dst;
        const std::vector<float>* src;
    } ups[] = {{h->tabA, &tabA}, {h->tabC, &tabC}, {h->alpha, &alpha}, {h->beta, &beta}};
    for (auto& u : ups) {
        hipError_t e = hipMemcpy(u.dst, u.src->data(), u.src->size() * sizeof(float),
                                 hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            dco_set_error("hipMemcpy of tables failed: %s", hipGetErrorString(e));
            return fail(DCO_ERR_HIP);
        }
    }
    if ((st = alloc_scratch(h)) != DCO_OK) return fail(st);
    *out = h;
    return DCO_OK;
}

extern "C" void dco_stereo_destroy(dco_stereo* h) {
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    for (hipEvent_t e : h->prof_events) (void)hipEventDestroy(e);
    free_handle_memory(h);
    delete h;
}

// Next free event of the profiling pool (created on demand).
static dco_status prof_event(dco_stereo* h, hipEvent_t* out) {
    if (h->prof_used == h->prof_events.size()) {
        hipEvent_t e;
        DCO_HIP_CHECK(hipEventCreate(&e));
        h->prof_events.push_back(e);
    }
    *out = h->prof_events[h->prof_used++];
    return DCO_OK;
}

static dco_status prof_mark(dco_stereo* h) {
    if (!h->profiling) return DCO_OK;
    hipEvent_t e;
    DCO_TRY(prof_event(h, &e));
    DCO_HIP_CHECK(hipEventRecord(e, h->stream));
    return DCO_OK;
}

extern "C" dco_status dco_stereo_profile(dco_stereo* h, int enable) {
    DCO_TRY(need(h, "handle"));
    h->profiling = enable != 0;
    if (enable) h->prof_used = 0;
    return DCO_OK;
}

extern "C" dco_status dco_stereo_stage_times(dco_stereo* h, float* ms, int n, int* calls) {
    DCO_TRY(need(h, "handle"));
    DCO_TRY(need(ms, "ms"));
    const size_t per = 2 * DCO_NUM_STAGES;
    const size_t ncalls = h->prof_used / per;
    for (int s = 0; s < n; ++s) ms[s] = 0.0f;
    for (size_t c = 0; c < ncalls; ++c)
        for (int s = 0; s < n && s < DCO_NUM_STAGES; ++s) {
            hipEvent_t a = h->prof_events[c * per + 2 * s], b = h->prof_events[c * per + 2 * s + 1];
            DCO_HIP_CHECK(hipEventSynchronize(b));
            float t = 0.0f;
            DCO_HIP_CHECK(hipEventElapsedTime(&t, a, b));
            ms[s] += t;
        }
    if (calls) *calls = (int)ncalls;
    return DCO_OK;
}

extern "C" dco_status dco_stereo_set_stream(dco_stereo* h, void* stream) {
    if (!h) {
        dco_set_error("dco_stereo_set_stream: handle is NULL");
        return DCO_ERR_ARG;
    }
    h->stream = (hipStream_t)stream;
    return DCO_OK;
}

dco_status need(const void* ptr, const char* what) {
    if (!ptr) {
        dco_set_error("%s is NULL", what);
        return DCO_ERR_ARG;
    }
    return DCO_OK;
}

dco_status need_align(const void* ptr, size_t a, const char* what) {
    if (((uintptr_t)ptr) % a) {
        dco_set_error("%s must be %zu-byte aligned", what, a);
        return DCO_ERR_ARG;
    }
    return DCO_OK;
}

extern "C" dco_status dco_census(dco_stereo* h, const uint8_t* rgb, uint64_t* census,
                                 uint8_t* arms) {
    DCO_TRY(need(h, "handle"));
    DCO_TRY(need(rgb, "rgb"));
    DCO_TRY(need(census, "census"));
    DCO_TRY(need(arms, "arms"));
    DCO_TRY(need_align(census, 8, "census"));
    DCO_TRY(need_align(arms, 4, "arms"));
    DCO_HIP_CHECK(launch_census_arms(rgb, h->W, h->H, h->p.census_w, h->p.census_h, h->p.arm_L1,
                                     h->p.arm_tau1, census, (uint32_t*)arms, nullptr, nullptr,
                                     h->stream));
    return DCO_OK;
}

extern "C" dco_status dco_cost_volume(dco_stereo* h, int ref, const uint8_t* rgbL,
                                      const uint8_t* rgbR, const uint64_t* cenL,
                                      const uint64_t* cenR, const uint8_t* arms_ref,
                                      float* cost) {
    DCO_TRY(need(h, "handle"));
    if (ref != 0 && ref != 1) {
        dco_set_error("ref must be 0 (left) or 1 (right), got %d", ref);
        return DCO_ERR_ARG;
    }
    DCO_TRY(need(rgbL, "rgbL"));
    DCO_TRY(need(rgbR, "rgbR"));
    DCO_TRY(need(cenL, "cenL"));
    DCO_TRY(need(cenR, "cenR"));
    DCO_TRY(need(arms_ref, "arms_ref"));
    DCO_TRY(need(cost, "cost"));
    DCO_TRY(need_align(cenL, 8, "cenL"));
    DCO_TRY(need_align(cenR, 8, "cenR"));
    DCO_TRY(need_align(arms_ref, 4, "arms_ref"));
    DCO_TRY(need_align(cost, 4, "cost"));
    DCO_HIP_CHECK(launch_cost(ref, rgbL, rgbR, cenL, cenR, (const uint32_t*)arms_ref, h->W, h->H,
                              h->D, h->tabA, h->tabC, h->alpha, h->beta, h->p.arm_L1, cost,
                              h->stream));
    return DCO_OK;
}

extern "C" dco_status dco_aggregate(dco_stereo* h, const float* cost, const uint8_t* arms_ref,
                                    float* agg) {
    DCO_TRY(need(h, "handle"));
    DCO_TRY(need(cost, "cost"));
    DCO_TRY(need(arms_ref, "arms_ref"));
    DCO_TRY(need(agg, "agg"));
    DCO_TRY(need_align(arms_ref, 4, "arms_ref"));
    DCO_TRY(need_align(cost, 4, "cost"));
    DCO_TRY(need_align(agg, 4, "agg"));
    if ((const void*)cost == (const void*)agg) {
        dco_set_error("dco_aggregate: agg must not alias cost");
        return DCO_ERR_ARG;
    }
    const uint32_t* arms = (const uint32_t*)arms_ref;
    DCO_HIP_CHECK(launch_geometry(arms, h->W, h->H, h->p.agg_iters, h->s.rec[0],
                                  pair_rec_geom(h->p.agg_iters), h->stream));
    DCO_HIP_CHECK(launch_aggregate(cost, h->s.rec[0], h->W, h->H, h->D, h->p.agg_iters, agg,
                                   h->stream));
    return DCO_OK;
}

extern "C" dco_status dco_wta_lrcheck(dco_stereo* h, const float* aggL, const float* aggR,
                                      float* disp, uint8_t* valid, int16_t* dL, int16_t* dR) {
    DCO_TRY(need(h, "handle"));
    DCO_TRY(need(aggL, "aggL"));
    DCO_TRY(need(aggR, "aggR"));
    DCO_TRY(need(disp, "disp"));
    DCO_TRY(need(valid, "valid"));
    int16_t* oL = dL ? dL : h->s.dint[0];
    int16_t* oR = dR ? dR : h->s.dint[1];
    DCO_HIP_CHECK(launch_wta2(aggL, aggR, h->W, h->H, h->D, h->p.subpixel, oL, h->s.delta, oR,
                              h->stream));
    DCO_HIP_CHECK(launch_lrcheck(oL, h->s.delta, oR, h->W, h->H, h->p.lr_max_diff, disp, valid,
                                 h->stream));
    return DCO_OK;
}

extern "C" dco_status dco_stereo_match(dco_stereo* h, const uint8_t* rgbL, const uint8_t* rgbR,
                                       float* disp, uint8_t* valid) {
    DCO_TRY(need(h, "handle"));
    DCO_TRY(need(rgbL, "rgbL"));
    DCO_TRY(need(rgbR, "rgbR"));
    DCO_TRY(need(disp, "disp"));
    DCO_TRY(need(valid, "valid"));
    if (!h->scratch_ready) {
        dco_set_error("handle has no scratch");
        return DCO_ERR_STATE;
    }
    dco_scratch& s = h->s;
    const dco_params& p = h->p;
    const uint8_t* img[2] = {rgbL, rgbR};
    DCO_TRY(prof_mark(h));
    DCO_HIP_CHECK(launch_front2(img[0], img[1], h->W, h->H, p.census_w, p.census_h, p.arm_L1,
                                p.arm_tau1, p.agg_iters, s.arms[0], s.arms[1], s.pix[0], s.pix[1],
                                s.rec[0], s.rec[1], pair_rec_geom(p.agg_iters), h->stream));
    DCO_TRY(prof_mark(h));
    DCO_TRY(prof_mark(h));
    DCO_HIP_CHECK(launch_cost_aggregate2(s.pix[0], s.pix[1], s.rec[0], s.rec[1], h->W, h->H, h->D,
                                         p.agg_iters, h->tabA, h->tabC, h->alpha, h->beta,
                                         p.arm_L1, s.agg[0], s.agg[1], true, h->stream));
    s.agg_paired = p.agg_iters == 2;
    DCO_TRY(prof_mark(h));
    DCO_TRY(prof_mark(h));
    if (s.agg_paired)  // WTA from the even slices (each pair's minimum)
        DCO_HIP_CHECK(launch_wta_pairs(s.agg[0], s.agg[1], h->W, h->H, h->D, p.subpixel,
                                       s.dint[0], s.delta, s.dint[1], h->stream));
    else
        DCO_HIP_CHECK(launch_wta2(s.agg[0], s.agg[1], h->W, h->H, h->D, p.subpixel, s.dint[0],
                                  s.delta, s.dint[1], h->stream));
    DCO_TRY(prof_mark(h));
    DCO_TRY(prof_mark(h));
    DCO_HIP_CHECK(launch_lrcheck(s.dint[0], s.delta, s.dint[1], h->W, h->H, p.lr_max_diff, disp,
                                 valid, h->stream));
    DCO_TRY(prof_mark(h));
    DCO_TRY(prof_mark(h));
    if (p.vote_iters > 0) {
        const int16_t* dv = nullptr;
        DCO_HIP_CHECK(launch_vote(s.dint[0], valid, s.arms[0], h->W, h->H, h->D, p.vote_iters,
                                  s.vote[0], s.vote[1], &dv, h->stream));
        DCO_HIP_CHECK(launch_vote_finish(dv, nullptr, s.agg[0], s.agg_paired, h->W, h->H, h->D,
                                         p.subpixel, disp, valid, nullptr, h->stream));
    }
    DCO_TRY(prof_mark(h));
    return DCO_OK;
}

extern "C" dco_status dco_stereo_match_half(dco_stereo* h, const uint8_t* rgbL2,
                                            const uint8_t* rgbR2, int W2, int H2, float fB,
                                            float* disp2, uint8_t* valid, float* depth) {
    DCO_TRY(need(h, "handle"));
    DCO_TRY(need(rgbL2, "rgbL2"));
    DCO_TRY(need(rgbR2, "rgbR2"));
    DCO_TRY(need(disp2, "disp2"));
    DCO_TRY(need(valid, "valid"));
    if (W2 / 2 != h->W || H2 / 2 != h->H || W2 < 0 || H2 < 0) {
        dco_set_error("full images of %d x %d do not reduce to the handle's %d x %d", W2, H2, h->W,
                      h->H);
        return DCO_ERR_SHAPE;
    }
    if (depth && !pos_finite(fB)) {
        dco_set_error("fB must be finite and > 0 when depth is requested");
        return DCO_ERR_ARG;
    }
    if (!h->scratch_ready) {
        dco_set_error("handle has no scratch");
        return DCO_ERR_STATE;
    }
    DCO_HIP_CHECK(launch_downscale2(rgbL2, rgbR2, W2, h->W, h->H, h->s.half[0], h->s.half[1],
                                    h->stream));
    DCO_TRY(dco_stereo_match(h, h->s.half[0], h->s.half[1], disp2, valid));
    DCO_HIP_CHECK(launch_depth_half(disp2, valid, h->W, h->H, fB, depth, h->stream));
    return DCO_OK;
}

extern "C" dco_status dco_vote_refine(dco_stereo* h, const uint8_t* armsL, const float* aggL,
                                      const int16_t* dL, const uint8_t* valid, int iters,
                                      float* disp, uint8_t* valid_out, int16_t* dvote) {
    DCO_TRY(need(h, "handle"));
    DCO_TRY(need(armsL, "armsL"));
    DCO_TRY(need(aggL, "aggL"));
    DCO_TRY(need(dL, "dL"));
    DCO_TRY(need(valid, "valid"));
    DCO_TRY(need(disp, "disp"));
    DCO_TRY(need(valid_out, "valid_out"));
    DCO_TRY(need_align(armsL, 4, "armsL"));
    if (iters < 0 || iters > kVoteMaxIters) {
        dco_set_error("iters must be in [0, %d] (got %d)", kVoteMaxIters, iters);
        return DCO_ERR_ARG;
    }
    if (!h->scratch_ready) {
        dco_set_error("handle has no scratch");
        return DCO_ERR_STATE;
    }
    const int16_t* dv = dL;
    const uint8_t* mask = valid;
    if (iters > 0) {
        DCO_HIP_CHECK(launch_vote(dL, valid, reinterpret_cast<const uint32_t*>(armsL), h->W, h->H,
                                  h->D, iters, h->s.vote[0], h->s.vote[1], &dv, h->stream));
        mask = nullptr;
    }
    DCO_HIP_CHECK(launch_vote_finish(dv, mask, aggL, false, h->W, h->H, h->D, h->p.subpixel, disp,
                                     valid_out, dvote, h->stream));
    return DCO_OK;
}

extern "C" dco_status dco_stereo_agg_slices(dco_stereo* h, int view, int d0, int n, float* out) {
    DCO_TRY(need(h, "handle"));
    DCO_TRY(need(out, "out"));
    if (view != 0 && view != 1) {
        dco_set_error("view must be 0 (left) or 1 (right), got %d", view);
        return DCO_ERR_ARG;
    }
    if (d0 < 0 || n < 1 || d0 > h->D - n) {
        dco_set_error("slices %d .. %d outside 0 .. %d", d0, d0 + n - 1, h->D - 1);
        return DCO_ERR_ARG;
    }
    if (!h->scratch_ready) {
        dco_set_error("handle has no scratch");
        return DCO_ERR_STATE;
    }
    const size_t P = (size_t)h->W * h->H;
    if (h->s.agg_paired)
        DCO_HIP_CHECK(launch_unpair(h->s.agg[view], h->W, h->H, h->D, d0, n, out, h->stream));
    else
        DCO_HIP_CHECK(hipMemcpyAsync(out, h->s.agg[view] + (size_t)d0 * P,
                                     (size_t)n * P * sizeof(float), hipMemcpyDeviceToDevice,
                                     h->stream));
    return DCO_OK;
}

extern "C" dco_status dco_stereo_last_disparities(dco_stereo* h, int16_t* dL, int16_t* dR) {
    DCO_TRY(need(h, "handle"));
    const size_t bytes = (size_t)h->W * h->H * sizeof(int16_t);
    if (dL)
        DCO_HIP_CHECK(hipMemcpyAsync(dL, h->s.dint[0], bytes, hipMemcpyDeviceToDevice, h->stream));
    if (dR)
        DCO_HIP_CHECK(hipMemcpyAsync(dR, h->s.dint[1], bytes, hipMemcpyDeviceToDevice, h->stream));
    return DCO_OK;
}

// ---- differentiable soft-argmin form ----

static void free_soft(SoftScratch& f) {
    void* ptrs[] = {f.pix[0], f.pix[1], f.arms,   f.arms_r, f.n1,     f.n2,
                    f.tab,    f.vol[0], f.vol[1], f.vol[2], f.partAC, f.partT};
    for (void* p : ptrs) dev_free(p);
    f = SoftScratch{};
}

static dco_status soft_reserve(dco_stereo* h, int B) {
    SoftScratch& f = h->soft;
    if (f.cap >= B) return DCO_OK;
    (void)hipStreamSynchronize(h->stream);
    free_soft(f);
    const size_t P = (size_t)h->W * h->H, V = P * h->D * B;
    DCO_TRY(dev_alloc(&f.pix[0], P * B));
    DCO_TRY(dev_alloc(&f.pix[1], P * B));
    DCO_TRY(dev_alloc(&f.arms, P * B));
    DCO_TRY(dev_alloc(&f.arms_r, P * B));
    DCO_TRY(dev_alloc(&f.n1, P * B));
    DCO_TRY(dev_alloc(&f.n2, P * B));
    DCO_TRY(dev_alloc(&f.tab, 1792));
    for (int k = 0; k < 3; ++k) DCO_TRY(dev_alloc(&f.vol[k], V));
    DCO_TRY(dev_alloc(&f.partAC, 2 * (size_t)B * h->D * h->H));
    DCO_TRY(dev_alloc(&f.partT, (size_t)B * h->D * h->H + 3 * 256));  // + the block totals
    f.cap = B;
    return DCO_OK;
}

// Arms and packed pixels of every pair, the Eq. 1 tables for theta,
// region counts, and the aggregated volume A2 (vol[0]).
static dco_status soft_front(dco_stereo* h, int B, const uint8_t* L, const uint8_t* R,
                             const float* theta, SoftBuffers* sb) {
    SoftScratch& f = h->soft;
    const dco_params& p = h->p;
    f.held = false;
    DCO_HIP_CHECK(launch_census_pairs(L, R, B, h->W, h->H, p.census_w, p.census_h, p.arm_L1,
                                      p.arm_tau1, f.arms, f.arms_r, f.pix[0], f.pix[1],
                                      h->stream));
    DCO_HIP_CHECK(soft_prepare(theta, f.tab, f.arms, B, h->W, h->H, h->D, f.n1, f.n2, h->stream));
    *sb = SoftBuffers{f.arms, f.n1, f.n2, f.pix[0], f.pix[1], h->alpha, f.tab};
    DCO_HIP_CHECK(
        soft_aggregate(*sb, B, h->W, h->H, h->D, f.vol[0], f.vol[1], f.vol[2], h->stream));
    f.held = true;
    f.held_B = B;
    f.held_L = L;
    f.held_R = R;
    f.held_theta = theta;
    f.held_stream = h->stream;
    return DCO_OK;
}

static dco_status soft_check(dco_stereo* h, int B) {
    DCO_TRY(need(h, "handle"));
    if (B < 1) {
        dco_set_error("B must be >= 1 (got %d)", B);
        return DCO_ERR_ARG;
    }
    if (h->W > 2048 || h->p.agg_iters != 2) {
        dco_set_error("the soft path needs W <= 2048 and two-stage aggregation");
        return DCO_ERR_SHAPE;
    }
    if ((long long)B * h->D > 65535 || (long long)B * h->D * h->H >= (1LL << 31)) {
        dco_set_error("the soft path needs B*D <= 65535 and B*D*H < 2^31 (B=%d, D=%d, H=%d)", B,
                      h->D, h->H);
        return DCO_ERR_SHAPE;
    }
    return DCO_OK;
}

extern "C" dco_status dco_soft_forward(dco_stereo* h, int B, const uint8_t* L, const uint8_t* R,
                                       const float* theta, float* dhat, float* lse) {
    DCO_TRY(soft_check(h, B));
    DCO_TRY(need(L, "L"));
    DCO_TRY(need(R, "R"));
    DCO_TRY(need(theta, "theta"));
    DCO_TRY(need(dhat, "dhat"));
    DCO_TRY(need(lse, "lse"));
    DCO_TRY(soft_reserve(h, B));
    SoftBuffers sb;
    DCO_TRY(soft_front(h, B, L, R, theta, &sb));
    DCO_HIP_CHECK(soft_argmin(sb, B, h->W, h->H, h->D, h->soft.vol[0], theta, dhat, lse,
                              h->stream));
    return DCO_OK;
}

extern "C" dco_status dco_soft_backward(dco_stereo* h, int B, const uint8_t* L, const uint8_t* R,
                                        const float* theta, const float* dhat, const float* lse,
                                        const float* grad_dhat, float* grad_theta) {
    DCO_TRY(soft_check(h, B));
    DCO_TRY(need(L, "L"));
    DCO_TRY(need(R, "R"));
    DCO_TRY(need(theta, "theta"));
    DCO_TRY(need(dhat, "dhat"));
    DCO_TRY(need(lse, "lse"));
    DCO_TRY(need(grad_dhat, "grad_dhat"));
    DCO_TRY(need(grad_theta, "grad_theta"));
    DCO_TRY(soft_reserve(h, B));
    SoftBuffers sb;
    DCO_TRY(soft_front(h, B, L, R, theta, &sb));  // recompute the aggregation
    SoftScratch& f = h->soft;
    DCO_HIP_CHECK(soft_backward(sb, B, h->W, h->H, h->D, f.vol[0], theta, dhat, lse, grad_dhat,
                                f.vol[1], f.vol[2], f.partAC, f.partT, grad_theta, h->stream));
    return DCO_OK;
}

extern "C" dco_status dco_soft_backward_reuse(dco_stereo* h, int B, const uint8_t* L,
                                              const uint8_t* R, const float* theta,
                                              const float* dhat, const float* lse,
                                              const float* grad_dhat, float* grad_theta) {
    DCO_TRY(soft_check(h, B));
    DCO_TRY(need(L, "L"));
    DCO_TRY(need(R, "R"));
    DCO_TRY(need(theta, "theta"));
    DCO_TRY(need(dhat, "dhat"));
    DCO_TRY(need(lse, "lse"));
    DCO_TRY(need(grad_dhat, "grad_dhat"));
    DCO_TRY(need(grad_theta, "grad_theta"));
    DCO_TRY(soft_reserve(h, B));
    SoftScratch& f = h->soft;
    SoftBuffers sb;
    // the backward kernels leave the held aggregation, tables, counts, arms
    // and pixels as they are, so any number of backward calls can reuse them
    if (f.held && f.held_B == B && f.held_L == L && f.held_R == R && f.held_theta == theta &&
        f.held_stream == h->stream)
        sb = SoftBuffers{f.arms, f.n1, f.n2, f.pix[0], f.pix[1], h->alpha, f.tab};
    else
        DCO_TRY(soft_front(h, B, L, R, theta, &sb));
    DCO_HIP_CHECK(soft_backward(sb, B, h->W, h->H, h->D, f.vol[0], theta, dhat, lse, grad_dhat,
                                f.vol[1], f.vol[2], f.partAC, f.partT, grad_theta, h->stream));
    return DCO_OK;
}
