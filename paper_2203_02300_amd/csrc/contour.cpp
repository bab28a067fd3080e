// contour.cpp -- host side of the depth contour extraction (Sec. 5):
// scratch, the map launches and the hysteresis loop.
#include <cmath>
#include <new>

#include "dco_internal.h"

struct dco_contour {
    int W = 0, H = 0, w = 0, h = 0;
    dco_contour_params p{};
    hipStream_t stream = nullptr;
    ContourBufs b{};
    float* Mn = nullptr;        // the normalised fused amplitude when the caller wants none
    int* changed_host = nullptr;
    int launches = 0;
};

extern "C" dco_status dco_contour_default_params(dco_contour_params* out) {
    if (!out) {
        dco_set_error("dco_contour_default_params: out is NULL");
        return DCO_ERR_ARG;
    }
    out->T_high = 0.06f;   // Sec. 7.2
    out->T_low = 0.03f;
    out->T_depth = 0.03f;
    out->box_radius = 2;
    return DCO_OK;
}

static void free_contour(dco_contour* h) {
    ContourBufs& b = h->b;
    void* ptrs[] = {b.fused, b.box_max, b.g2_max, b.g, b.G2, b.state[0], b.state[1], b.changed,
                    h->Mn};
    for (void* q : ptrs) dev_free(q);
    pinned_free(h->changed_host);
}

extern "C" void dco_contour_destroy(dco_contour* h) {
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    free_contour(h);
    delete h;
}

extern "C" dco_status dco_contour_create(dco_contour** out, int W, int H,
                                         const dco_contour_params* p, void* stream) {
    if (!out) {
        dco_set_error("dco_contour_create: out is NULL");
        return DCO_ERR_ARG;
    }
    *out = nullptr;
    dco_contour_params prm;
    if (p)
        prm = *p;
    else
        dco_contour_default_params(&prm);
    if (W < 2 || H < 2 || (long long)W * H > (1LL << 28)) {
        dco_set_error("contour frame %d x %d: need W, H >= 2 and W*H <= 2^28", W, H);
        return DCO_ERR_SHAPE;
    }
    auto ok = [](float v) { return std::isfinite(v) && v >= 0.0f; };
    if (!ok(prm.T_high) || !ok(prm.T_low) || !ok(prm.T_depth) || prm.box_radius < 0 ||
        prm.box_radius > 16) {
        dco_set_error("contour parameters: need finite thresholds >= 0 and 0 <= box_radius <= 16");
        return DCO_ERR_ARG;
    }
    dco_contour* h = new (std::nothrow) dco_contour();
    if (!h) {
        dco_set_error("host allocation failed");
        return DCO_ERR_OOM;
    }
    h->W = W;
    h->H = H;
    h->w = W / 2;
    h->h = H / 2;
    h->p = prm;
    h->stream = (hipStream_t)stream;
    const size_t P = (size_t)W * H, q = (size_t)h->w * h->h;
    ContourBufs& b = h->b;
    auto fail = [&](dco_status s) {
        free_contour(h);
        delete h;
        return s;
    };
    dco_status st;
    if ((st = dev_alloc(&b.fused, q)) != DCO_OK) return fail(st);
    if ((st = dev_alloc(&h->Mn, q)) != DCO_OK) return fail(st);
    if ((st = dev_alloc(&b.box_max, kContourMaxSlots)) != DCO_OK) return fail(st);
    if ((st = dev_alloc(&b.g2_max, kContourMaxSlots)) != DCO_OK) return fail(st);
    if ((st = dev_alloc(&b.g, P)) != DCO_OK) return fail(st);
    if ((st = dev_alloc(&b.G2, P)) != DCO_OK) return fail(st);
    if ((st = dev_alloc(&b.state[0], P)) != DCO_OK) return fail(st);
    if ((st = dev_alloc(&b.state[1], P)) != DCO_OK) return fail(st);
    if ((st = dev_alloc(&b.changed, kHystGroup)) != DCO_OK) return fail(st);
    if ((st = pinned_alloc((void**)&h->changed_host, kHystGroup * sizeof(int))) != DCO_OK)
        return fail(st);
    *out = h;
    return DCO_OK;
}

extern "C" dco_status dco_contour_run(dco_contour* h, const uint8_t* rgb, const float* past,
                                      const float* future, uint8_t* B, float* MI, float* Mn) {
    DCO_TRY(need(h, "handle"));
    DCO_TRY(need(rgb, "rgb"));
    DCO_TRY(need(past, "past"));
    DCO_TRY(need(future, "future"));
    DCO_TRY(need(B, "B"));
    DCO_TRY(need_align(past, 8, "past"));
    DCO_TRY(need_align(future, 8, "future"));
    float* mn = Mn ? Mn : h->Mn;
    const dco_contour_params& p = h->p;
    DCO_HIP_CHECK(launch_contour_maps(past, future, h->w, h->h, p.box_radius, rgb, h->W, h->H,
                                      p.T_high, p.T_low, p.T_depth, h->b, mn, MI, h->stream));
    // Groups of kHystGroup launches, one host check per group; each launch
    // that changes a pixel turns a weak pixel strong, so at most W H launches
    // change anything.  The first launch that changed nothing read the final
    // state; it and the launches before it are counted.
    int parity = 0;
    h->launches = 0;
    for (;;) {
        DCO_HIP_CHECK(launch_contour_hyst_group(h->b, h->W, h->H, parity, h->stream));
        DCO_HIP_CHECK(hipMemcpyAsync(h->changed_host, h->b.changed, kHystGroup * sizeof(int),
                                     hipMemcpyDeviceToHost, h->stream));
        DCO_HIP_CHECK(hipStreamSynchronize(h->stream));
        int k = 0;
        while (k < kHystGroup && h->changed_host[k]) ++k;
        if (k < kHystGroup) {
            h->launches += k + 1;
            parity ^= k & 1;  // the input of launch k
            break;
        }
        h->launches += kHystGroup;  // the group's last output is state[parity] again
    }
    DCO_HIP_CHECK(launch_contour_edges(h->b, h->W, h->H, parity, B, h->stream));
    return DCO_OK;
}

extern "C" dco_status dco_contour_launches(dco_contour* h, int* launches) {
    DCO_TRY(need(h, "handle"));
    DCO_TRY(need(launches, "launches"));
    *launches = h->launches;
    return DCO_OK;
}
