/*
 * dco_stereo.h -- C ABI of the MI355X (gfx950) two-stage adaptive AD-census
 * stereo matcher: the sparse-disparity front end of the depth contour
 * occlusion method (paper Sec. 4).
 *
 * Problem statement (Sec. 3, Sec. 4): a rectified stereo pair (epipolar lines
 * are image rows) goes in, with the left view as the reference; a sparse
 * disparity map comes out, 0 marking a missing value (the convention of
 * Eq. 14).  The steps are the census transform and cross-support arms
 * (Sec. 4.1), the adaptive AD-census cost (Eq. 1), aggregation over the
 * adaptive region (Eq. 2, applied as two stages), winner-take-all (Eq. 3)
 * with parabola sub-pixel refinement, and a left-right consistency check.
 *
 * Conventions shared by every entry point
 *  - Memory: every buffer argument is a DEVICE pointer owned by the caller,
 *    contiguous, naturally aligned (uint64 to 8 bytes, float to 4).  Images
 *    are H x W x 3 uint8, row-major, RGB interleaved.  Per-pixel maps are
 *    H x W row-major.  Arms are H x W x 4 uint8 in the order (left, right,
 *    up, down).  Volumes are D x H x W float (one H x W slice per disparity,
 *    d = 0 .. D-1).  The library owns only its handle, its lookup tables and
 *    internal scratch.
 *  - Streams: every call after create is asynchronous on the handle's
 *    stream (a hipStream_t passed as void*; NULL = the default stream).
 *    Nothing synchronises except create, destroy and the batch autotuner.
 *  - Errors: every call returns a dco_status.  Argument errors (null
 *    pointers, sizes out of range) are detected before anything is launched
 *    and return DCO_ERR_ARG or DCO_ERR_SHAPE; HIP failures return
 *    DCO_ERR_HIP; allocation failures DCO_ERR_OOM.  dco_last_error() gives a
 *    thread-local message for the last failure.  Nothing throws across the ABI.
 *  - Determinism: equal inputs give bit-identical outputs, whatever the
 *    launch configuration (all sums are integer; see dco_aggregate).
 */
#ifndef DCO_STEREO_H
#define DCO_STEREO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dco_stereo dco_stereo; /* opaque matcher handle */
typedef struct dco_batch dco_batch;   /* opaque batched-matcher handle */

typedef enum {
    DCO_OK = 0,
    DCO_ERR_ARG = -1,   /* null pointer or parameter out of range */
    DCO_ERR_SHAPE = -2, /* W, H or D out of range */
    DCO_ERR_HIP = -3,   /* a HIP runtime call failed */
    DCO_ERR_OOM = -4,   /* device allocation failed */
    DCO_ERR_STATE = -5  /* handle not usable for this call */
} dco_status;

/* Matcher parameters.  Defaults (dco_default_params): the stereo constants
 * of Sec. 7.2 (lambda_AD = 10, lambda_census = 40, gamma_L = 1, eps = 0.8)
 * and, where the paper gives none, census 9 x 7, L1 = 17, tau1 = 20,
 * two-stage aggregation, LR tolerance 0, sub-pixel on. */
typedef struct {
    int census_w, census_h;   /* odd, census_w * census_h - 1 <= 64 (default 9, 7) */
    int arm_L1, arm_tau1;     /* 0 <= L1 <= 17; 1 <= tau1 <= 256 (default 17, 20).
                                 The paper gives no L1; the kernels are built for
                                 arms of at most 17 (aggregation halos of 34
                                 columns and LDS rings of 36 rows), so a larger
                                 L1 is refused with DCO_ERR_ARG. */
    float lambda_ad;          /* > 0 (Eq. 1) */
    float lambda_census;      /* > 0 (Eq. 1) */
    float gamma_L, eps;       /* > 0 (Eq. 1, weight alpha) */
    int agg_iters;            /* 2 = two-stage aggregation; 1 = Eq. 2 once */
    int lr_max_diff;          /* >= 0: LR tolerance in whole disparities */
    int subpixel;             /* 1 = parabola refinement, 0 = integer output */
    int vote_iters;           /* 0 <= n <= 64: passes of the Eq. 4 region vote that
                                 dco_stereo_match applies after the LR check
                                 (default 0 = none) */
} dco_params;

/* Fill *out with the defaults above.  DCO_ERR_ARG if out is NULL. */
dco_status dco_default_params(dco_params* out);

/* Create a matcher for W x H images and disparities d = 0 .. D-1.
 * Requires 1 <= D < W, W >= census_w, H >= census_h, W, H <= 16384,
 * W * H <= 2^27 and W * H * D < 2^31 (else DCO_ERR_SHAPE).  Copies *p
 * (NULL = defaults), builds the Eq. 1 tables on the host in double precision
 * and uploads them, and allocates the scratch that dco_stereo_match needs.
 * Synchronous.  On failure *out is NULL. */
dco_status dco_stereo_create(dco_stereo** out, int W, int H, int D, const dco_params* p,
                             void* stream);

/* Free the handle and its scratch (synchronises its stream).  NULL is a no-op. */
void dco_stereo_destroy(dco_stereo* h);

/* Make later calls enqueue on `stream` (a hipStream_t). */
dco_status dco_stereo_set_stream(dco_stereo* h, void* stream);

/* Census codes and cross arms of one image (Sec. 4.1; C_census of Eq. 1).
 *   grey:   Y = (77 R + 150 G + 29 B + 128) >> 8
 *   census: bit k of census[p] is Y(q_k) < Y(p) for the k-th neighbour q_k
 *           of the census_w x census_h window, enumerated row-major (top row
 *           first) without the centre, coordinates clamped to the image
 *   arms:   for each direction, the largest k <= L1 such that every step
 *           j = 1..k stays inside the image and the largest per-channel
 *           absolute difference to p is below tau1
 * rgb: H x W x 3 uint8; census: H x W uint64 (out); arms: H x W x 4 uint8 (out). */
dco_status dco_census(dco_stereo* h, const uint8_t* rgb, uint64_t* census, uint8_t* arms);

/* Raw AD-census cost volume of one reference view (Eq. 1), fixed point.
 * ref = 0: reference = left view, partner pixel (x - d, y) in the right view;
 * ref = 1: reference = right view, partner pixel (x + d, y) in the left view.
 *   s = sum over RGB of |I_ref - I_partner|     (C_AD = s / 3)
 *   h = popcount(census_ref ^ census_partner)
 *   L = min of the four arms of the reference pixel (arms_ref)
 *   q = rint(alpha_L * TA[s] * 2^20) + rint(beta_L * TC[h] * 2^20)
 * with float tables alpha_L = 1 - exp(-gamma_L / (L + eps)), beta_L =
 * exp(-gamma_L / (L + eps)), TA[s] = 1 - exp(-s / (3 lambda_AD)), TC[h] =
 * 1 - exp(-h / lambda_census), each rounded once from double; each term is
 * rounded once (half to even) from the exact product of its float factors.
 * A partner outside the image gives q = 2^20.
 * cost[d][y][x] = q * 2^-20 (D x H x W float, out). */
dco_status dco_cost_volume(dco_stereo* h, int ref, const uint8_t* rgbL, const uint8_t* rgbR,
                           const uint64_t* cenL, const uint64_t* cenR, const uint8_t* arms_ref,
                           float* cost);

/* Aggregation over the reference view's adaptive cross region (Eq. 2).
 * cost must hold values q * 2^-20 with integer 0 <= q <= 2^20 (as written by
 * dco_cost_volume); other values give unspecified results.  With agg_iters = 2:
 *   stage 1: S1 = sum over the horizontal-then-vertical cross region of q,
 *            N1 = its pixel count, a1 = floor((S1 + floor(N1/2)) / N1)
 *   stage 2: S2 = sum over the vertical-then-horizontal cross region of a1,
 *            N2 = its pixel count, agg = ((float)S2 / (float)N2) * 2^-20
 * With agg_iters = 1: agg = ((float)S1 / (float)N1) * 2^-20.
 * cost, agg: D x H x W float (agg out, must not alias cost); arms_ref: the
 * reference view's arms. */
dco_status dco_aggregate(dco_stereo* h, const float* cost, const uint8_t* arms_ref, float* agg);

/* Winner-take-all (Eq. 3) of both views, sub-pixel refinement of the left
 * view and the left-right check.
 *   d* = smallest d minimising agg(p, d)
 *   delta = (m - p) / (2 ((m - c) + (p - c))) with m, c, p the aggregated
 *           costs at d*-1, d*, d*+1, clamped to [-0.5, 0.5]; 0 when d* is 0
 *           or D-1 (or subpixel = 0)
 *   valid(x, y) = x - dL >= 0 and |dL(x, y) - dR(x - dL, y)| <= lr_max_diff
 *   disp = dL + delta where valid, else 0
 * aggL, aggR: D x H x W float; disp: H x W float (out); valid: H x W uint8
 * (out); dL, dR: H x W int16 (out, optional: NULL to skip). */
dco_status dco_wta_lrcheck(dco_stereo* h, const float* aggL, const float* aggR, float* disp,
                           uint8_t* valid, int16_t* dL, int16_t* dR);

/* The whole plain matcher in one call (Sec. 4, Eq. 1-3, LR check):
 *  1. census, arms and the region counts of both views (one launch);
 *  2. the raw cost of Eq. 1 computed on the fly inside the two-stage
 *     aggregation of both views (one launch): no raw cost volume exists,
 *     but the two aggregated volumes (D x H x W float each, 2 x 472 MB at
 *     1280 x 720, D = 128) are written to the handle's scratch; with two
 *     stages each pair of slices (2g, 2g + 1) is stored with its smaller
 *     cost and that cost's slice in slice 2g and the other cost in 2g + 1;
 *  3. WTA with sub-pixel refinement of both views, reading those volumes
 *     (a separate pass; with two stages only the even slices, plus the
 *     costs at d - 1 and d + 1 for the parabola), then the LR check;
 *  4. when vote_iters > 0, the Eq. 4 vote of dco_vote_refine.
 * With vote_iters = 0 the results are bit-identical to dco_census ->
 * dco_cost_volume -> dco_aggregate -> dco_wta_lrcheck; with vote_iters = n
 * they equal that chain followed by dco_vote_refine with iters = n.
 * rgbL, rgbR: H x W x 3 uint8; disp: H x W float (out); valid: H x W uint8 (out). */
dco_status dco_stereo_match(dco_stereo* h, const uint8_t* rgbL, const uint8_t* rgbR, float* disp,
                            uint8_t* valid);

/* The quarter-size front end (Sec. 4.4): the disparity is computed on the
 * pair reduced to half width and half height, then doubled and converted to
 * depth.  The handle is created for the reduced size W x H (and the
 * disparity range D of the reduced pair); the full images are W2 x H2 with
 * W2 / 2 = W and H2 / 2 = H (an odd last column or row is dropped).
 *   reduction: each reduced pixel and channel = (sum of its 2 x 2 block + 2) >> 2
 *   then dco_stereo_match on the reduced pair (vote_iters applies)
 *   disp2 = 2 x the reduced disparity where valid, else 0
 *   depth = fB / disp2 where disp2 > 0, else 0 (0 = no depth, as in Eq. 14)
 * fB = focal length (pixels of the full image) x baseline, in the unit wanted
 * for depth; not used when depth is NULL.
 * rgbL2, rgbR2: H2 x W2 x 3 uint8; disp2, depth: H x W float (out; depth
 * optional); valid: H x W uint8 (out). */
dco_status dco_stereo_match_half(dco_stereo* h, const uint8_t* rgbL2, const uint8_t* rgbR2,
                                 int W2, int H2, float fB, float* disp2, uint8_t* valid,
                                 float* depth);

/* Disparity refinement by region vote (Eq. 4, Sec. 4.3), `iters` passes.
 * In each pass every valid pixel p takes the disparity with the most votes
 * in its stage-1 cross region N_p: for each y' in [y - u(p), y + dn(p)] the
 * pixels x' in [x - l(x, y'), x + r(x, y')].  Only valid pixels vote, with
 * their integer disparity; equal counts go to the smallest disparity; a
 * pass reads only the previous pass's map.  Then, where the voted map dv is
 * valid: disp = dv + the parabola offset of dco_wta_lrcheck taken at dv on
 * aggL (0 if subpixel = 0), valid_out = 1; elsewhere disp = 0, valid_out = 0.
 * A pixel with valid = 0 or dL outside [0, D) is invalid and stays so.
 * dco_stereo_match with vote_iters = n gives the same result as
 * dco_wta_lrcheck followed by this call with iters = n.
 * armsL: H x W x 4 uint8 left arms as from dco_census (4-byte aligned; arms
 * are clipped to 17); aggL: D x H x W float; dL: H x W int16; valid: H x W
 * uint8; disp: H x W float (out); valid_out: H x W uint8 (out, may alias
 * valid); dvote: H x W int16 (out, optional: the voted map, -1 where
 * invalid).  Needs 0 <= iters <= 64. */
dco_status dco_vote_refine(dco_stereo* h, const uint8_t* armsL, const float* aggL,
                           const int16_t* dL, const uint8_t* valid, int iters, float* disp,
                           uint8_t* valid_out, int16_t* dvote);

/* Integer disparities of both views from the last dco_stereo_match on this
 * handle (H x W int16 each, device, out; either may be NULL). */
dco_status dco_stereo_last_disparities(dco_stereo* h, int16_t* dL, int16_t* dR);

/* Per-stage GPU timing of dco_stereo_match (diagnostics).  While enabled,
 * every kernel stage of dco_stereo_match is bracketed by HIP events recorded
 * on the handle's stream (no synchronisation is added).
 * dco_stereo_profile(h, 1) starts (and clears) the record, (h, 0) stops it.
 * dco_stereo_stage_times waits for the recorded events and writes, for each
 * stage s < n, ms[s] = total milliseconds over the recorded calls, and
 * *calls = the number of recorded calls.  Stages: 0 census + arms + region
 * counts of both views, 1 cost + aggregation of both views (one launch),
 * 2 WTA of both views, 3 LR check, 4 Eq. 4 vote and its sub-pixel output
 * (0 ms when vote_iters = 0).  ms: host array of n floats. */
#define DCO_NUM_STAGES 5
dco_status dco_stereo_profile(dco_stereo* h, int enable);
dco_status dco_stereo_stage_times(dco_stereo* h, float* ms, int n, int* calls);

/* ---- Depth densification (Sec. 6, Eq. 13-20) ---- */

/* The dense depth D of an H x W grid minimises Eq. 20:
 *   lambda_d  sum_p w_sparse(p) (D(p) - D_sparse(p))^2             (Eq. 13-14)
 * + lambda_s  sum_p sum_{q in N4(p)} w_pq (D(p) - D(q))^2           (Eq. 15-17)
 * + lambda_s2 sum_p w_stable(p) (D(p) - D_pre(p))^2                 (Eq. 18-19)
 * with w_sparse = [D_sparse > 0], w_stable = [D_pre > 0], and w_pq = 0 when
 * exactly one of p, q is on the depth contour B_dp, else
 * max(1 - min(s_p, s_q), 0) with s = M_fuse M_I.  The normal equations are
 * solved by Jacobi-preconditioned conjugate gradients in FP64 until
 * |r| <= tol |b| or max_iters iterations; pixels whose region (joined by
 * w_pq > 0 edges) holds no data or stability term get D = 0. */
typedef struct {
    float lambda_d, lambda_s, lambda_s2;  /* >= 0 (Sec. 7.2: 0.8, 1.2, 0.02) */
    double tol;                           /* relative residual to stop at (default 1e-9) */
    int max_iters;                        /* >= 0 (default 4000) */
    int iters_per_launch;                 /* even, 2..1024: iterations per graph launch,
                                             convergence is checked between launches
                                             (default 16) */
} dco_densify_params;
typedef struct dco_densify dco_densify; /* opaque densification handle */

dco_status dco_densify_default_params(dco_densify_params* out);

/* Buffers for an H x W grid and the captured iteration graph (p may be
 * NULL for the defaults; stream: the HIP stream the solves run on).
 * Requires 1 <= W, H and W * H <= 2^23 (else DCO_ERR_SHAPE). */
dco_status dco_densify_create(dco_densify** out, int W, int H, const dco_densify_params* p,
                              void* stream);
void dco_densify_destroy(dco_densify* h);

/* One solve.  Ds (D_sparse, 0 = no data), Dpre (D_pre, 0 = none; NULL for
 * none), Mfuse, MI: H x W float; Bdp: H x W uint8 (nonzero = on the depth
 * contour); D: H x W float (out).  All device pointers.  Returns when the
 * solve has converged or used max_iters iterations (the host reads the
 * convergence flag after every launch of iters_per_launch iterations). */
dco_status dco_densify_run(dco_densify* h, const float* Ds, const float* Dpre, const uint8_t* Bdp,
                           const float* Mfuse, const float* MI, float* D);

/* Iterations used by the last solve and its final |r| / |b| (host outputs,
 * either may be NULL).  Synchronises the stream. */
dco_status dco_densify_stats(dco_densify* h, int* iters, double* rel_residual);

/* ---- Depth contour extraction given the optical flows (Sec. 5) ---- */

/* From the past and future flow fields of the middle frame (computed
 * elsewhere, on the quarter-size grid w = W / 2, h = H / 2 as (U, V) float
 * pairs) and the full-size colour frame:
 *   r = |I| (correctly rounded); M = max(|r(p_right) - r(p)|, |r(p_bottom) - r(p)|)
 *       (a missing neighbour gives 0)                                    (Eq. 6-8)
 *   score = I(p1).e - I(p0).e with e = I(p) / |I(p)|, p1, p0 = p +- rint(e)
 *       clamped (0 where I(p) = 0)                                       (Eq. 9-11)
 *   Mfuse = M_past where score_past > score_future, M_future where lower,
 *       the larger of the two where equal                               (Eq. 12)
 *   Mn = the (2 box_radius + 1)^2 mean of Mfuse clipped to the grid, divided
 *       by its maximum (0 when that is 0)                                (Sec. 5.2)
 *   Canny on the census grey: 3x3 Sobel (replicated borders), G2 = gx^2 + gy^2;
 *       suppression along the gradient's sector (horizontal when 128|gy| <
 *       53|gx|, vertical when 128|gx| < 53|gy|, else the diagonal of sign(gx gy)),
 *       keeping p when G2(p) > G2 before it and >= G2 after it; p dropped when
 *       Mn(x / 2, y / 2) < T_depth; strong when G2 > T_high^2 max G2, weak when
 *       G2 > T_low^2 max G2; weak pixels 8-connected to strong ones kept (Sec. 5.3)
 *   B = the kept pixels (the depth contour B_dp of Eq. 16), MI = sqrt(G2 / max G2)
 *       (the M_I of Eq. 17). */
typedef struct {
    float T_high, T_low, T_depth;  /* >= 0 (Sec. 7.2: 0.06, 0.03, 0.03) */
    int box_radius;                /* 0..16 (default 2: a 5 x 5 box) */
} dco_contour_params;
typedef struct dco_contour dco_contour; /* opaque contour-extraction handle */

dco_status dco_contour_default_params(dco_contour_params* out);
/* Scratch for W x H frames (W, H >= 2); p may be NULL for the defaults. */
dco_status dco_contour_create(dco_contour** out, int W, int H, const dco_contour_params* p,
                              void* stream);
void dco_contour_destroy(dco_contour* h);
/* rgb: H x W x 3 uint8; past, future: h x w x 2 float (8-byte aligned);
 * B: H x W uint8 (out, 0/1); MI: H x W float (out, optional); Mn: h x w
 * float (out, optional).  Device pointers.  Synchronous: the host repeats
 * hysteresis launches until one changes nothing. */
dco_status dco_contour_run(dco_contour* h, const uint8_t* rgb, const float* past,
                           const float* future, uint8_t* B, float* MI, float* Mn);
/* Hysteresis launches of the last run (diagnostics). */
dco_status dco_contour_launches(dco_contour* h, int* launches);

/* ---- Batched matcher: many pairs of uneven size and disparity range ---- */

/* Create a batched matcher for n pairs of sizes W[i] x H[i], disparity
 * ranges D[i] (host arrays, each pair within the limits of
 * dco_stereo_create).  For every distinct (W, H, D) the tile
 * autotuner times the candidate aggregation tiles (rows per work item,
 * disparities per work item) on a synthetic pair of that size, or reads the
 * choice from its cache file (the environment variable DCO_AUTOTUNE_CACHE,
 * default $HOME/.cache/dco_stereo_autotune.txt; DCO_AUTOTUNE=0 skips tuning
 * and takes full-height bands of one disparity).  It then allocates each
 * pair's scratch, builds the device work list (stages in order; the
 * aggregation items in pair, view, strip, band, disparity order, cut into
 * one contiguous part of about equal cost per XCD, so that the workgroups
 * an XCD runs together share a strip's inputs in its L2) and captures its
 * five stage launches (each a persistent work-list kernel over all pairs)
 * in one HIP graph.  Synchronous. */
dco_status dco_batch_create(dco_batch** out, int n, const int* W, const int* H, const int* D,
                            const dco_params* p, void* stream);
void dco_batch_destroy(dco_batch* b);

/* Match every pair with one graph launch on the stream given at create.
 * L, R, disp, valid: host arrays of n device pointers (images H x W x 3
 * uint8; disp H x W float; valid H x W uint8).  The pointers are copied to
 * the device before the launch; the arrays may be reused on return.
 * Per-pair results are bit-identical to dco_stereo_match. */
dco_status dco_batch_match(dco_batch* b, const uint8_t* const* L, const uint8_t* const* R,
                           float* const* disp, uint8_t* const* valid);

/* Tiles the autotuner picked for pair i (host pointers, out): output columns
 * of an aggregation strip, rows of an aggregation band, disparities per
 * aggregation work item. */
dco_status dco_batch_tile(const dco_batch* b, int i, int* strip_w, int* band_h, int* d_chunk);

/* ---- Differentiable soft-argmin form (left view) ---- */

/* Forward for B pairs of the handle's size, stacked (L, R: B x H x W x 3).
 * theta: 3 device floats (lambda_AD, lambda_census, T).  Float costs
 *   c = alpha_L (1 - exp(-(s/3)/lambda_AD)) + (1 - alpha_L)(1 - exp(-h/lambda_census))
 * (c = 1 where the partner is outside the image), two normalised region
 * means as in dco_aggregate but in float with no rounding step, and
 *   dhat = sum_d d softmax_d(-agg(p, d) / T).
 * dhat: B x H x W float (out); lse: B x H x W float (out), the log-sum-exp
 * of -agg/T per pixel, kept for the backward pass.  DCO_ERR_SHAPE unless the
 * handle has W <= 2048 and two-stage aggregation, B * D <= 65535 and
 * B * D * H < 2^31. */
dco_status dco_soft_forward(dco_stereo* h, int B, const uint8_t* L, const uint8_t* R,
                            const float* theta, float* dhat, float* lse);

/* Backward: given grad_dhat = dLoss/d dhat (B x H x W float), writes
 * grad_theta[0..2] = dLoss/d(lambda_AD, lambda_census, T) (3 device floats,
 * overwritten).  Recomputes costs and aggregation; needs the dhat and lse of
 * the matching forward.  Deterministic. */
dco_status dco_soft_backward(dco_stereo* h, int B, const uint8_t* L, const uint8_t* R,
                             const float* theta, const float* dhat, const float* lse,
                             const float* grad_dhat, float* grad_theta);

/* The same backward, without the recomputation when it can be skipped: the
 * handle keeps the costs, region counts and aggregated volume of its last
 * soft aggregation (that of dco_soft_forward, or of a recomputing backward),
 * and the backward kernels do not overwrite them.  If that aggregation was
 * made with this B and these same L, R and theta pointers on the handle's
 * current stream, they are used as they are; otherwise the aggregation is
 * recomputed first, as in dco_soft_backward.  The caller guarantees that the
 * contents of L, R and theta have not changed since that aggregation (an
 * autograd engine's saved tensors do); under that guarantee the result is
 * bit-identical to dco_soft_backward's.  Same arguments and errors. */
dco_status dco_soft_backward_reuse(dco_stereo* h, int B, const uint8_t* L, const uint8_t* R,
                                   const float* theta, const float* dhat, const float* lse,
                                   const float* grad_dhat, float* grad_theta);

/* ---- Diagnostics ---- */
const char* dco_status_string(dco_status s);
const char* dco_last_error(void); /* thread-local; "" when none */

/* Aggregated costs A2 (Eq. 2 applied as two stages) of disparities
 * d0 .. d0 + n - 1 of one view (0 = left reference, 1 = right), as left in
 * the handle's scratch by the last dco_stereo_match: copied (and, when that
 * volume is in the paired slice order of two-stage aggregation, put back in
 * slice order) on the handle's stream into out (device, n x H x W float).
 * Lets a test compare the fused path's volume element by element.
 * DCO_ERR_ARG for a bad view or range. */
dco_status dco_stereo_agg_slices(dco_stereo* h, int view, int d0, int n, float* out);

/* The one-call match without a handle and without any allocation, for
 * callers that cannot allocate device or host memory: code under HIP stream
 * capture, tight serving loops, harnesses that forbid allocation.  Same
 * kernels and same result, bit for bit, as dco_stereo_create(W, H, D, params)
 * followed by dco_stereo_match on stream (params NULL = defaults; every
 * parameter, vote_iters included, applies).  Inputs rgbL, rgbR (device, H x W
 * x 3 uint8) and outputs disp (device, H x W float), valid (device, H x W
 * uint8) are the caller's; every intermediate buffer (packed pixels, arms,
 * records, both aggregated volumes, disparity maps, the Eq. 1 tables) lives
 * in a static device array of 160 MiB that the library holds on each GPU it
 * has run this call on until the process ends.  Shapes whose buffers do not
 * fit (beyond about 640 x 360 with D = 64) return DCO_ERR_SHAPE with the
 * bytes needed in dco_last_error(); argument and shape errors are the same
 * as dco_stereo_create's and are reported before any launch.  Asynchronous
 * on stream.  Every call on one GPU uses the same array: calls that overlap
 * on one GPU (two streams, two threads) race and must be serialised by the
 * caller; a later call overwrites what an earlier one left there. */
dco_status dco_stereo_match_noalloc(int W, int H, int D, const dco_params* params, void* stream,
                                    const uint8_t* rgbL, const uint8_t* rgbR, float* disp,
                                    uint8_t* valid);

/* Testing hooks for the error paths.  dco_debug_fail_alloc(k) makes the
 * k-th device or pinned allocation made by the library from now on fail
 * with DCO_ERR_OOM (k <= 0 disarms; DCO_FAIL_ALLOC=k in the environment arms
 * it when the library loads).  dco_debug_live_allocations() is the number
 * of the library's device and pinned allocations not yet freed, so a test
 * can check that a failed create frees exactly what it allocated.
 * Process-wide; not meant for concurrent use with other calls. */
void dco_debug_fail_alloc(int k);
long dco_debug_live_allocations(void);

#ifdef __cplusplus
}
#endif

#endif /* DCO_STEREO_H */
