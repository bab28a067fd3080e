// densify.cpp -- host side of the depth densification (Sec. 6, Eq. 13-20):
// buffers, the captured iteration graph and the convergence loop.
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "dco_internal.h"

struct dco_densify {
    int W = 0, H = 0, nblk = 0;
    dco_densify_params p{};
    hipStream_t stream = nullptr;
    DensifyBufs b{};
    hipGraphExec_t exec = nullptr;
    int* flags_host = nullptr;  // pinned copy of b.flags
    int launches = 0;           // graph launches of the last run
};

extern "C" dco_status dco_densify_default_params(dco_densify_params* out) {
    if (!out) {
        dco_set_error("dco_densify_default_params: out is NULL");
        return DCO_ERR_ARG;
    }
    out->lambda_d = 0.8f;   // Sec. 7.2
    out->lambda_s = 1.2f;
    out->lambda_s2 = 0.02f;
    out->tol = 1e-9;
    out->max_iters = 4000;
    out->iters_per_launch = 16;
    return DCO_OK;
}

static void free_densify(dco_densify* h) {
    DensifyBufs& b = h->b;
    void* ptrs[] = {b.cr, b.cd, b.diag, b.invdiag, b.x,  b.r,     b.q,  b.p[0],
                    b.p[1], b.rz[0], b.rz[1], b.rr[0], b.rr[1], b.pq, b.bb, b.flags};
    for (void* q : ptrs) dev_free(q);
    if (h->exec) (void)hipGraphExecDestroy(h->exec);
    pinned_free(h->flags_host);
}

extern "C" void dco_densify_destroy(dco_densify* h) {
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    free_densify(h);
    delete h;
}

extern "C" dco_status dco_densify_create(dco_densify** out, int W, int H,
                                         const dco_densify_params* p, void* stream) {
    if (!out) {
        dco_set_error("dco_densify_create: out is NULL");
        return DCO_ERR_ARG;
    }
    *out = nullptr;
    dco_densify_params prm;
    if (p)
        prm = *p;
    else
        dco_densify_default_params(&prm);
    // every block sums all blocks' partials in a fixed order, a cost that grows
    // with the square of the grid: 2^23 pixels (a 3840 x 2160 frame) at most
    if (W < 1 || H < 1 || (long long)W * H > (1LL << 23)) {
        dco_set_error("densify grid %d x %d: need 1 <= W, H and W*H <= 2^23", W, H);
        return DCO_ERR_SHAPE;
    }
    if (!(std::isfinite(prm.lambda_d) && prm.lambda_d >= 0.0f) ||
        !(std::isfinite(prm.lambda_s) && prm.lambda_s >= 0.0f) ||
        !(std::isfinite(prm.lambda_s2) && prm.lambda_s2 >= 0.0f) ||
        !(std::isfinite(prm.tol) && prm.tol >= 0.0) || prm.max_iters < 0 ||
        prm.iters_per_launch < 2 || prm.iters_per_launch > 1024 || (prm.iters_per_launch & 1)) {
        dco_set_error("densify parameters: need finite lambdas and tol >= 0, max_iters >= 0 and "
                      "an even iters_per_launch in [2, 1024]");
        return DCO_ERR_ARG;
    }
    dco_densify* h = new (std::nothrow) dco_densify();
    if (!h) {
        dco_set_error("host allocation failed");
        return DCO_ERR_OOM;
    }
    h->W = W;
    h->H = H;
    h->p = prm;
    h->stream = (hipStream_t)stream;
    h->nblk = densify_blocks(W, H);
    const size_t P = (size_t)W * H, nb = (size_t)h->nblk;
    DensifyBufs& b = h->b;
    auto fail = [&](dco_status s) {
        free_densify(h);
        delete h;
        return s;
    };
    dco_status st;
    double** vecs[] = {&b.cr, &b.cd, &b.diag, &b.invdiag, &b.x, &b.r, &b.q, &b.p[0], &b.p[1]};
    for (double** v : vecs)
        if ((st = dev_alloc(v, P)) != DCO_OK) return fail(st);
    double** parts[] = {&b.rz[0], &b.rz[1], &b.rr[0], &b.rr[1], &b.pq, &b.bb};
    for (double** v : parts)
        if ((st = dev_alloc(v, nb)) != DCO_OK) return fail(st);
    if ((st = dev_alloc(&b.flags, 2)) != DCO_OK) return fail(st);
    if ((st = pinned_alloc((void**)&h->flags_host, 2 * sizeof(int))) != DCO_OK) return fail(st);
    // one launch = iters_per_launch iterations (two kernels each), captured
    // once on a private stream of default priority; no memset nodes
    hipStream_t cap;
    if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        dco_set_error("hipStreamCreate failed");
        return fail(DCO_ERR_HIP);
    }
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        const hipError_t e1 = launch_densify_iters(b, W, H, prm.tol, prm.iters_per_launch, cap);
        e = hipStreamEndCapture(cap, &g);
        if (e == hipSuccess) e = e1;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&h->exec, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(cap);
    if (e != hipSuccess) {
        dco_set_error("densify graph capture failed: %s", hipGetErrorString(e));
        (void)hipGetLastError();
        return fail(DCO_ERR_HIP);
    }
    *out = h;
    return DCO_OK;
}

extern "C" dco_status dco_densify_run(dco_densify* h, const float* Ds, const float* Dpre,
                                      const uint8_t* Bdp, const float* Mfuse, const float* MI,
                                      float* D) {
    DCO_TRY(need(h, "handle"));
    DCO_TRY(need(Ds, "Ds"));
    DCO_TRY(need(Bdp, "Bdp"));
    DCO_TRY(need(Mfuse, "Mfuse"));
    DCO_TRY(need(MI, "MI"));
    DCO_TRY(need(D, "D"));
    const dco_densify_params& p = h->p;
    DCO_HIP_CHECK(launch_densify_setup(h->b, Ds, Dpre, Bdp, Mfuse, MI, h->W, h->H, p.lambda_d,
                                       p.lambda_s, p.lambda_s2, h->stream));
    h->launches = 0;
    for (int done = 0; done < p.max_iters; done += p.iters_per_launch) {
        DCO_HIP_CHECK(hipGraphLaunch(h->exec, h->stream));
        ++h->launches;
        DCO_HIP_CHECK(hipMemcpyAsync(h->flags_host, h->b.flags, 2 * sizeof(int),
                                     hipMemcpyDeviceToHost, h->stream));
        DCO_HIP_CHECK(hipStreamSynchronize(h->stream));
        if (h->flags_host[0]) break;
    }
    DCO_HIP_CHECK(launch_densify_out(h->b, h->W, h->H, D, h->stream));
    return DCO_OK;
}

extern "C" dco_status dco_densify_stats(dco_densify* h, int* iters, double* rel_residual) {
    DCO_TRY(need(h, "handle"));
    DCO_HIP_CHECK(hipStreamSynchronize(h->stream));
    int f[2];
    DCO_HIP_CHECK(hipMemcpy(f, h->b.flags, sizeof(f), hipMemcpyDeviceToHost));
    if (iters) *iters = f[1];
    if (rel_residual) {
        // the newest r.r block sums: iteration k writes parity k & 1; setup parity 1
        const double* rr = f[1] > 0 ? h->b.rr[(f[1] - 1) & 1] : h->b.rr[1];
        std::vector<double> a((size_t)h->nblk), c((size_t)h->nblk);
        DCO_HIP_CHECK(hipMemcpy(a.data(), rr, a.size() * sizeof(double), hipMemcpyDeviceToHost));
        DCO_HIP_CHECK(
            hipMemcpy(c.data(), h->b.bb, c.size() * sizeof(double), hipMemcpyDeviceToHost));
        double sr = 0.0, sb = 0.0;
        for (size_t i = 0; i < a.size(); ++i) {
            sr += a[i];
            sb += c[i];
        }
        *rel_residual = sb > 0.0 ? std::sqrt(sr / sb) : 0.0;
    }
    return DCO_OK;
}
