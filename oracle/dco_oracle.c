/*
 * dco_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, single-threaded CPU reference of the two-stage adaptive
 * AD-census stereo matcher (paper Sec. 4).  It exists to check the GPU
 * library; nothing in the product path may call it.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg load it.
 *
 * It shares no code, header, table or constant generator with the GPU
 * library.  Every loop follows the definition directly: no blocking, no
 * prefix sums, no reordering.  Build: gcc -O2 -ffp-contract=off -shared -fPIC.
 *
 * Readings of passages the paper leaves open are marked READING below; the
 * same list is kept with the design notes.
 *
 * Layouts: images H x W x 3 uint8 (row-major, RGB interleaved); per-pixel maps
 * H x W; arms H x W x 4 uint8 in the order (left, right, up, down); volumes
 * D x H x W (one H x W slice per disparity).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q_ONE 1048576 /* 2^20: fixed-point unit of a raw cost */

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }
static int absi(int v) { return v < 0 ? -v : v; }

/* READING (census input): census compares integer grey levels
 * Y = (77 R + 150 G + 29 B + 128) >> 8; the weights sum to 256. */
void orc_grey(const uint8_t* rgb, int W, int H, uint8_t* Y) {
    for (int i = 0; i < W * H; ++i) {
        int r = rgb[3 * i], g = rgb[3 * i + 1], b = rgb[3 * i + 2];
        Y[i] = (uint8_t)((77 * r + 150 * g + 29 * b + 128) >> 8);
    }
}

/* Census transform (Sec. 4.2.1, the C_census term of Eq. 1).
 * READING: window cw columns x ch rows (9 x 7), neighbours enumerated
 * row-major (top row first, left to right) skipping the centre; bit k (LSB
 * first) is set when the neighbour's grey level is strictly below the
 * centre's; coordinates outside the image are clamped to the edge. */
void orc_census(const uint8_t* Y, int W, int H, int cw, int ch, uint64_t* out) {
    int hw = cw / 2, hh = ch / 2;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            int c = Y[y * W + x];
            uint64_t code = 0;
            int k = 0;
            for (int dy = -hh; dy <= hh; ++dy)
                for (int dx = -hw; dx <= hw; ++dx) {
                    if (dy == 0 && dx == 0) continue;
                    int yy = clampi(y + dy, 0, H - 1), xx = clampi(x + dx, 0, W - 1);
                    if (Y[yy * W + xx] < c) code |= (uint64_t)1 << k;
                    ++k;
                }
            out[y * W + x] = code;
        }
}

/* Cross-support arms (Sec. 4.1: colour and distance double threshold).
 * READING: an arm in direction e extends over step j = 1, 2, ... while the
 * step stays inside the image, j <= L1, and the largest per-channel absolute
 * difference between the pixel at p + j e and p itself is below tau1. */
void orc_arms(const uint8_t* rgb, int W, int H, int L1, int tau1, uint8_t* arms) {
    static const int ex[4] = {-1, 1, 0, 0};
    static const int ey[4] = {0, 0, -1, 1};
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            const uint8_t* p = rgb + 3 * (y * W + x);
            for (int dir = 0; dir < 4; ++dir) {
                int k = 0;
                while (k < L1) {
                    int nx = x + (k + 1) * ex[dir], ny = y + (k + 1) * ey[dir];
                    if (nx < 0 || nx >= W || ny < 0 || ny >= H) break;
                    const uint8_t* q = rgb + 3 * (ny * W + nx);
                    int m = absi(q[0] - p[0]);
                    if (absi(q[1] - p[1]) > m) m = absi(q[1] - p[1]);
                    if (absi(q[2] - p[2]) > m) m = absi(q[2] - p[2]);
                    if (m >= tau1) break;
                    ++k;
                }
                arms[4 * (y * W + x) + dir] = (uint8_t)k;
            }
        }
}

/* Eq. 1 tables, computed in double and rounded once to float.
 *   alpha[L] = 1 - exp(-gamma / (L + eps)),  beta[L] = exp(-gamma / (L + eps))
 *   TA[s]    = 1 - exp(-(s/3) / lambda_ad)   for the RGB sum s in 0..765
 *   TC[h]    = 1 - exp(-h / lambda_census)   for the Hamming distance h in 0..64
 * READING: C_AD is the mean absolute RGB difference s/3; alpha uses the
 * reference pixel's shortest arm L_min.  Parameters arrive as float. */
void orc_tables(int L1, float gamma, float eps, float lam_ad, float lam_c,
                float* alpha, float* beta, float* TA, float* TC) {
    for (int L = 0; L <= L1; ++L) {
        double e = exp(-(double)gamma / ((double)L + (double)eps));
        alpha[L] = (float)(1.0 - e);
        beta[L] = (float)e;
    }
    for (int s = 0; s <= 765; ++s) TA[s] = (float)(-expm1(-(double)s / (3.0 * (double)lam_ad)));
    for (int h = 0; h <= 64; ++h) TC[h] = (float)(-expm1(-(double)h / (double)lam_c));
}

static int lmin_of(const uint8_t* a) {
    int m = a[0];
    for (int i = 1; i < 4; ++i)
        if (a[i] < m) m = a[i];
    return m;
}

/* Raw matching cost, Eq. 1, in fixed point.
 * READING: each term is the exact product of its two FP32 factors, scaled by
 * 2^20 and rounded once to the nearest integer (ties to even):
 *   q = rint(alpha[Lmin] * TA[s] * 2^20) + rint(beta[Lmin] * TC[h] * 2^20).
 * The product of two floats is exact in double, and so is the scaling.
 * The stored cost is q * 2^-20.  ref = 0: reference = left view, partner at
 * x - d in the right view; ref = 1: reference = right view, partner at x + d
 * in the left view.  A partner outside the image costs q = 2^20 (cost 1, the
 * supremum of Eq. 1).  Output: D x H x W int32. */
void orc_cost(int ref, const uint8_t* rgbL, const uint8_t* rgbR, const uint64_t* cenL,
              const uint64_t* cenR, const uint8_t* arms_ref, int W, int H, int D, int L1,
              float gamma, float eps, float lam_ad, float lam_c, int32_t* q) {
    float alpha[256], beta[256], TA[766], TC[65];
    orc_tables(L1, gamma, eps, lam_ad, lam_c, alpha, beta, TA, TC);
    const uint8_t* I0 = ref == 0 ? rgbL : rgbR;
    const uint8_t* I1 = ref == 0 ? rgbR : rgbL;
    const uint64_t* C0 = ref == 0 ? cenL : cenR;
    const uint64_t* C1 = ref == 0 ? cenR : cenL;
    for (int d = 0; d < D; ++d)
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                int xo = ref == 0 ? x - d : x + d;
                int32_t v;
                if (xo < 0 || xo >= W) {
                    v = Q_ONE;
                } else {
                    const uint8_t* a = I0 + 3 * (y * W + x);
                    const uint8_t* b = I1 + 3 * (y * W + xo);
                    int s = absi(a[0] - b[0]) + absi(a[1] - b[1]) + absi(a[2] - b[2]);
                    uint64_t xr = C0[y * W + x] ^ C1[y * W + xo];
                    int h = 0;
                    for (int k = 0; k < 64; ++k) h += (int)((xr >> k) & 1u);
                    int L = lmin_of(arms_ref + 4 * (y * W + x));
                    double qa = rint((double)alpha[L] * (double)TA[s] * 1048576.0);
                    double qc = rint((double)beta[L] * (double)TC[h] * 1048576.0);
                    v = (int32_t)qa + (int32_t)qc;
                }
                q[((size_t)d * H + y) * W + x] = v;
            }
}

/* Cost aggregation over the adaptive support region, Eq. 2.
 * READING ("two-stage"): iters = 2 applies Eq. 2 twice, first over the
 * horizontal-then-vertical cross region, then over the vertical-then-
 * horizontal one, each a normalised mean:
 *   stage 1: E1(x,y) = sum of q over x' in [x - l, x + r] on row y
 *            S1(x,y) = sum of E1(x, y') over y' in [y - u, y + dn]
 *            N1 = number of pixels in that region
 *            a1 = floor((S1 + floor(N1 / 2)) / N1)          (integer)
 *   stage 2: E2(x,y) = sum of a1(x, y') over y' in [y - u, y + dn]
 *            S2(x,y) = sum of E2(x', y) over x' in [x - l, x + r]
 *            N2 = number of pixels in that region
 *            A2 = ((float)S2 / (float)N2) * 2^-20            (IEEE float)
 * where (l, r, u, dn) are the arms of the pixel each sum is centred on.
 * iters = 1 applies stage 1 once and returns ((float)S1 / (float)N1) * 2^-20.
 * The region is the reference view's cross region, the same for every d. */
void orc_aggregate(const int32_t* q, const uint8_t* arms, int W, int H, int D, int iters,
                   float* out) {
    int64_t* E1 = (int64_t*)malloc(sizeof(int64_t) * (size_t)W * H);
    int64_t* A1 = (int64_t*)malloc(sizeof(int64_t) * (size_t)W * H);
    int64_t* E2 = (int64_t*)malloc(sizeof(int64_t) * (size_t)W * H);
#define ARM(x, y, k) ((int)arms[4 * ((y) * W + (x)) + (k)])
    for (int d = 0; d < D; ++d) {
        const int32_t* qd = q + (size_t)d * W * H;
        float* od = out + (size_t)d * W * H;
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                int64_t s = 0;
                for (int xx = x - ARM(x, y, 0); xx <= x + ARM(x, y, 1); ++xx) s += qd[y * W + xx];
                E1[y * W + x] = s;
            }
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                int64_t s = 0, n = 0;
                for (int yy = y - ARM(x, y, 2); yy <= y + ARM(x, y, 3); ++yy) {
                    s += E1[yy * W + x];
                    n += ARM(x, yy, 0) + ARM(x, yy, 1) + 1;
                }
                if (iters == 1)
                    od[y * W + x] = ((float)s / (float)n) * 0x1p-20f;
                else
                    A1[y * W + x] = (s + n / 2) / n;
            }
        if (iters == 1) continue;
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                int64_t s = 0;
                for (int yy = y - ARM(x, y, 2); yy <= y + ARM(x, y, 3); ++yy) s += A1[yy * W + x];
                E2[y * W + x] = s;
            }
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                int64_t s = 0, n = 0;
                for (int xx = x - ARM(x, y, 0); xx <= x + ARM(x, y, 1); ++xx) {
                    s += E2[y * W + xx];
                    n += ARM(xx, y, 2) + ARM(xx, y, 3) + 1;
                }
                od[y * W + x] = ((float)s / (float)n) * 0x1p-20f;
            }
    }
#undef ARM
    free(E1);
    free(A1);
    free(E2);
}

/* Winner-take-all, Eq. 3, and sub-pixel refinement.
 * READING (ties): the smallest d among equal minima.
 * READING (sub-pixel; not in the paper): parabola through the aggregated
 * costs m = A(d*-1), c = A(d*), p = A(d*+1):
 *   num = m - p;  den = (m - c) + (p - c);  delta = num / (2 den)
 * clamped to [-0.5, 0.5]; delta = 0 when d* is 0 or D-1 or den <= 0. */
static float parabola_at(const float* agg, size_t P, size_t i, int D, int d) {
    float del = 0.0f;
    if (d > 0 && d < D - 1) {
        float m = agg[(size_t)(d - 1) * P + i];
        float c = agg[(size_t)d * P + i];
        float p = agg[(size_t)(d + 1) * P + i];
        float num = m - p;
        float den = (m - c) + (p - c);
        if (den > 0.0f) {
            float two_den = 2.0f * den;
            del = num / two_den;
            if (del > 0.5f) del = 0.5f;
            if (del < -0.5f) del = -0.5f;
        }
    }
    return del;
}

void orc_wta(const float* agg, int W, int H, int D, int16_t* dint, float* delta) {
    size_t P = (size_t)W * H;
    for (size_t i = 0; i < P; ++i) {
        int best = 0;
        float bv = agg[i];
        for (int d = 1; d < D; ++d)
            if (agg[(size_t)d * P + i] < bv) {
                bv = agg[(size_t)d * P + i];
                best = d;
            }
        dint[i] = (int16_t)best;
        delta[i] = parabola_at(agg, P, i, D, best);
    }
}

/* Left-right consistency check.  READING (not in the paper, whose outlier
 * step is the Eq. 4 vote): a left pixel is valid when its partner x - dL is
 * inside the image and |dL(x) - dR(x - dL)| <= maxdiff.  The output disparity
 * is dL + delta for a valid pixel and 0 otherwise (0 marks a missing value,
 * as in Eq. 14). */
void orc_lrcheck(const int16_t* dL, const float* deltaL, const int16_t* dR, int W, int H,
                 int maxdiff, int subpixel, float* disp, uint8_t* valid) {
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            int dl = dL[y * W + x];
            int xr = x - dl;
            int ok = xr >= 0 && absi(dl - (int)dR[y * W + xr]) <= maxdiff;
            valid[y * W + x] = (uint8_t)ok;
            float del = subpixel ? deltaL[y * W + x] : 0.0f;
            disp[y * W + x] = ok ? (float)dl + del : 0.0f;
        }
}

/* Disparity refinement by region vote, Eq. 4 (Sec. 4.3).
 * READING (region): N_p is p's stage-1 cross region: for each y' in
 *   [y - u(p), y + dn(p)], the pixels x' in [x - l(x, y'), x + r(x, y')].
 * READING (votes): only valid pixels vote, each with its integer disparity;
 *   a value outside [0, D) counts as invalid.  An invalid pixel is not
 *   changed and stays invalid (-1 in the output).
 * READING (choice): the disparity with the most votes in N_p; among equal
 *   counts the smallest.  A valid p lies in its own region and votes, so it
 *   always has a winner.
 * READING (iterations): `iters` passes; each pass reads only the previous
 *   pass's map, so every pixel of a pass sees the same input.
 * din: H x W int16; valid: H x W uint8; arms: H x W x 4; dout: H x W int16. */
void orc_vote(const int16_t* din, const uint8_t* valid, const uint8_t* arms, int W, int H, int D,
              int iters, int16_t* dout) {
    size_t P = (size_t)W * H;
    int16_t* cur = (int16_t*)malloc(2 * P);
    int16_t* nxt = (int16_t*)malloc(2 * P);
    int* hist = (int*)malloc(sizeof(int) * (size_t)D);
#define ARM(x, y, k) ((int)arms[4 * ((size_t)(y) * W + (x)) + (k)])
    for (size_t i = 0; i < P; ++i)
        cur[i] = (int16_t)(valid[i] && din[i] >= 0 && din[i] < D ? din[i] : -1);
    for (int it = 0; it < iters; ++it) {
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                size_t i = (size_t)y * W + x;
                if (cur[i] < 0) {
                    nxt[i] = -1;
                    continue;
                }
                memset(hist, 0, sizeof(int) * (size_t)D);
                for (int yy = y - ARM(x, y, 2); yy <= y + ARM(x, y, 3); ++yy)
                    for (int xx = x - ARM(x, yy, 0); xx <= x + ARM(x, yy, 1); ++xx) {
                        int v = cur[(size_t)yy * W + xx];
                        if (v >= 0) hist[v]++;
                    }
                int best = 0;
                for (int d = 1; d < D; ++d)
                    if (hist[d] > hist[best]) best = d;
                nxt[i] = (int16_t)best;
            }
        int16_t* t = cur;
        cur = nxt;
        nxt = t;
    }
#undef ARM
    memcpy(dout, cur, 2 * P);
    free(cur);
    free(nxt);
    free(hist);
}

/* Output of the voted map: where dv >= 0, disp = dv plus the parabola offset
 * at dv from the aggregated costs (the sub-pixel READING of orc_wta; 0 when
 * subpixel = 0) and valid = 1; elsewhere disp = 0 and valid = 0. */
void orc_vote_finish(const float* agg, const int16_t* dv, int W, int H, int D, int subpixel,
                     float* disp, uint8_t* valid) {
    size_t P = (size_t)W * H;
    for (size_t i = 0; i < P; ++i) {
        int ok = dv[i] >= 0;
        valid[i] = (uint8_t)ok;
        disp[i] = ok ? (float)dv[i] + (subpixel ? parabola_at(agg, P, i, D, dv[i]) : 0.0f) : 0.0f;
    }
}

/* ------------------------------------------------------------------------
 * Depth contour extraction given the two optical flow fields (Sec. 5).
 * The flows are computed elsewhere (the DIS flow method is not in this library);
 * they arrive on the quarter-size grid w x h as (U, V) pairs, float.
 * ------------------------------------------------------------------------ */

/* Eq. 6-8: r = |I(p)| (FP32, correctly rounded square root); M(p) = max of
 * |r(p_right) - r(p)| and |r(p_bottom) - r(p)|.
 * READING (border): a missing right or bottom neighbour contributes 0. */
static float flow_r(const float* F, int i) {
    float u = F[2 * i], v = F[2 * i + 1];
    return sqrtf(u * u + v * v);
}
static float flow_amp(const float* F, int w, int h, int x, int y) {
    int i = y * w + x;
    float r = flow_r(F, i);
    float gu = x + 1 < w ? fabsf(flow_r(F, i + 1) - r) : 0.0f;
    float gv = y + 1 < h ? fabsf(flow_r(F, i + w) - r) : 0.0f;
    return gu > gv ? gu : gv;
}

/* Eq. 9-11: the change of the flow projected on its own direction at p:
 * e = I(p) / |I(p)|, p1 = p + rint(e), p0 = p - rint(e) (clamped to the
 * grid), f_i = I(p_i) . e, score = f1 - f0.
 * READING (step): p0 and p1 are the nearest pixels one unit along -e and
 * +e; the paper draws them near p without a distance.  A zero flow has no
 * direction and scores 0. */
static float flow_score(const float* F, int w, int h, int x, int y) {
    int i = y * w + x;
    float r = flow_r(F, i);
    if (r == 0.0f) return 0.0f;
    float ex = F[2 * i] / r, ey = F[2 * i + 1] / r;
    int sx = (int)rintf(ex), sy = (int)rintf(ey);
    int x1 = clampi(x + sx, 0, w - 1), y1 = clampi(y + sy, 0, h - 1);
    int x0 = clampi(x - sx, 0, w - 1), y0 = clampi(y - sy, 0, h - 1);
    int j1 = y1 * w + x1, j0 = y0 * w + x0;
    float f1 = F[2 * j1] * ex + F[2 * j1 + 1] * ey;
    float f0 = F[2 * j0] * ex + F[2 * j0 + 1] * ey;
    return f1 - f0;
}

/* The two per-pixel terms of one flow field before fusion: the amplitude M
 * of Eq. 6-8 and the score of Eq. 9-11 (h x w each).  Exposed so that the
 * tests can pin each term on hand-built flows. */
void orc_flow_terms(const float* F, int w, int h, float* M, float* score) {
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            M[y * w + x] = flow_amp(F, w, h, x, y);
            score[y * w + x] = flow_score(F, w, h, x, y);
        }
}

/* Eq. 12 and the box filter of Sec. 5.2, then the normalisation of
 * Sec. 5.3.2: Mfuse = M_past where score_past > score_future, M_future
 * where score_future > score_past; then the mean over the (2R + 1)^2 window
 * clipped to the grid (summed row by row, left to right), then divided by
 * its maximum over the grid (all 0 when the maximum is 0).
 * READING (tie): equal scores keep the larger amplitude.
 * READING (box): the window size is not given; R is a parameter (default 2).
 * past, future: h x w x 2; out: h x w. */
void orc_flow_fuse(const float* past, const float* future, int w, int h, int R, float* out) {
    float* fu = (float*)malloc(sizeof(float) * (size_t)w * h);
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            float mp = flow_amp(past, w, h, x, y), mf = flow_amp(future, w, h, x, y);
            float sp = flow_score(past, w, h, x, y), sf = flow_score(future, w, h, x, y);
            fu[y * w + x] = sp > sf ? mp : (sf > sp ? mf : (mp > mf ? mp : mf));
        }
    float mx = 0.0f;
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            float s = 0.0f;
            int n = 0;
            for (int yy = y - R; yy <= y + R; ++yy)
                for (int xx = x - R; xx <= x + R; ++xx)
                    if (yy >= 0 && yy < h && xx >= 0 && xx < w) {
                        s += fu[yy * w + xx];
                        ++n;
                    }
            out[y * w + x] = s / (float)n;
            if (out[y * w + x] > mx) mx = out[y * w + x];
        }
    for (size_t i = 0; i < (size_t)w * h; ++i) out[i] = mx > 0.0f ? out[i] / mx : 0.0f;
    free(fu);
}

/* Canny with the depth gate (Sec. 5.3) on the full-size grey image Y (W x H,
 * the census grey of reading 1), given the normalised fused amplitude Mn on
 * the quarter grid (w = W / 2, h = H / 2).
 * READING (gradient): 3x3 Sobel on integer grey with replicated borders,
 *   G2 = gx^2 + gy^2 (exact integers); the normalised magnitude of
 *   Sec. 7.2 is sqrt(G2 / max G2), so a threshold T is G2 > T^2 max G2
 *   (compared in double).
 * READING (suppression): the direction of (gx, gy) falls in one of four
 *   sectors: horizontal when 128 |gy| < 53 |gx| (tan 22.5 deg ~ 53/128),
 *   vertical when 128 |gx| < 53 |gy|, else the diagonal given by the sign of
 *   gx gy; p survives when G2(p) > G2 of the neighbour before it along the
 *   direction and G2(p) >= G2 of the neighbour after it.
 * READING (gate): p is dropped when Mn at (min(x / 2, w - 1), min(y / 2,
 *   h - 1)) is below T_depth.
 * Double threshold: strong above T_high, weak above T_low; weak pixels
 * 8-connected (through weak or strong pixels) to a strong one are edges
 * (breadth-first search here).  Outputs the contour B (uint8 0/1) and the
 * normalised magnitude MI = sqrt(G2 / max G2) (FP32; 0 when max G2 = 0). */
void orc_contour(const uint8_t* Y, int W, int H, const float* Mn, int w, int h, float Thigh,
                 float Tlow, float Tdepth, uint8_t* B, float* MI) {
    size_t P = (size_t)W * H;
    int32_t* gx = (int32_t*)malloc(4 * P);
    int32_t* gy = (int32_t*)malloc(4 * P);
    int64_t* G2 = (int64_t*)malloc(8 * P);
    uint8_t* st = (uint8_t*)malloc(P);
    int* queue = (int*)malloc(sizeof(int) * P);
#define YV(xx, yy) ((int)Y[(size_t)clampi(yy, 0, H - 1) * W + clampi(xx, 0, W - 1)])
    int64_t mx = 0;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            int a = YV(x + 1, y - 1) + 2 * YV(x + 1, y) + YV(x + 1, y + 1) - YV(x - 1, y - 1) -
                    2 * YV(x - 1, y) - YV(x - 1, y + 1);
            int b = YV(x - 1, y + 1) + 2 * YV(x, y + 1) + YV(x + 1, y + 1) - YV(x - 1, y - 1) -
                    2 * YV(x, y - 1) - YV(x + 1, y - 1);
            size_t i = (size_t)y * W + x;
            gx[i] = a;
            gy[i] = b;
            G2[i] = (int64_t)a * a + (int64_t)b * b;
            if (G2[i] > mx) mx = G2[i];
        }
#undef YV
    double th = (double)Thigh * (double)Thigh * (double)mx;
    double tl = (double)Tlow * (double)Tlow * (double)mx;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            size_t i = (size_t)y * W + x;
            st[i] = 0;
            int ax = absi(gx[i]), ay = absi(gy[i]);
            int dx, dy;
            if (128 * ay < 53 * ax) { dx = 1; dy = 0; }
            else if (128 * ax < 53 * ay) { dx = 0; dy = 1; }
            else if ((gx[i] > 0) == (gy[i] > 0)) { dx = 1; dy = 1; }
            else { dx = 1; dy = -1; }
            int xa = x - dx, ya = y - dy, xb = x + dx, yb = y + dy;
            int64_t ga = (xa >= 0 && xa < W && ya >= 0 && ya < H) ? G2[(size_t)ya * W + xa] : 0;
            int64_t gb = (xb >= 0 && xb < W && yb >= 0 && yb < H) ? G2[(size_t)yb * W + xb] : 0;
            if (!(G2[i] > ga && G2[i] >= gb)) continue;
            float g = Mn[(size_t)(y / 2 < h ? y / 2 : h - 1) * w + (x / 2 < w ? x / 2 : w - 1)];
            if (g < Tdepth) continue;
            double v = (double)G2[i];
            st[i] = v > th ? 2 : (v > tl ? 1 : 0);
        }
    int qh = 0, qt = 0;
    for (size_t i = 0; i < P; ++i)
        if (st[i] == 2) queue[qt++] = (int)i;
    while (qh < qt) {
        int i = queue[qh++], y = i / W, x = i % W;
        for (int yy = y - 1; yy <= y + 1; ++yy)
            for (int xx = x - 1; xx <= x + 1; ++xx)
                if (yy >= 0 && yy < H && xx >= 0 && xx < W && st[(size_t)yy * W + xx] == 1) {
                    st[(size_t)yy * W + xx] = 2;
                    queue[qt++] = yy * W + xx;
                }
    }
    for (size_t i = 0; i < P; ++i) {
        B[i] = st[i] == 2;
        MI[i] = mx > 0 ? sqrtf((float)((double)G2[i] / (double)mx)) : 0.0f;
    }
    free(gx);
    free(gy);
    free(G2);
    free(st);
    free(queue);
}

/* Quarter-size front end (Sec. 4.4: the disparity is computed on the image
 * reduced to a quarter of its area, then doubled before depth conversion).
 * READING (reduction): each output pixel is the mean of a 2 x 2 block, per
 * channel, rounded half up: (a + b + c + d + 2) >> 2.  The output is
 * (W / 2) x (H / 2); an odd last column or row is dropped.
 * rgb: H x W x 3; out: (H / 2) x (W / 2) x 3. */
void orc_downscale2(const uint8_t* rgb, int W, int H, uint8_t* out) {
    int w = W / 2, h = H / 2;
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x)
            for (int c = 0; c < 3; ++c) {
                int s = rgb[((2 * y) * W + 2 * x) * 3 + c] + rgb[((2 * y) * W + 2 * x + 1) * 3 + c] +
                        rgb[((2 * y + 1) * W + 2 * x) * 3 + c] +
                        rgb[((2 * y + 1) * W + 2 * x + 1) * 3 + c];
                out[(y * w + x) * 3 + c] = (uint8_t)((s + 2) >> 2);
            }
}

/* Full-scale disparity and depth of a quarter-size match (Sec. 4.4).
 * READING: disparity doubled, dfull = 2 * disp (FP32, exact); depth is
 * fB / dfull with fB = focal length x baseline of the rig (not given in the
 * paper: a parameter), in FP32, where the pixel is valid and dfull > 0;
 * elsewhere dfull = 0 and depth = 0 (0 = no depth, as in Eq. 14).
 * All maps H x W of the quarter-size grid. */
void orc_depth_half(const float* disp, const uint8_t* valid, int W, int H, float fB,
                    float* dfull, float* depth) {
    for (size_t i = 0; i < (size_t)W * H; ++i) {
        float d2 = valid[i] ? 2.0f * disp[i] : 0.0f;
        dfull[i] = d2;
        depth[i] = d2 > 0.0f ? fB / d2 : 0.0f;
    }
}

/* The whole plain matcher: grey, census and arms of both views, the cost and
 * aggregated volumes of both views, WTA of both, LR check, and, when
 * vote_iters > 0, the Eq. 4 vote on the LR-valid left disparities with the
 * sub-pixel offset taken again at the voted disparity. */
void orc_match(const uint8_t* rgbL, const uint8_t* rgbR, int W, int H, int D, int cw, int ch,
               int L1, int tau1, float gamma, float eps, float lam_ad, float lam_c, int iters,
               int maxdiff, int subpixel, int vote_iters, float* disp, uint8_t* valid,
               int16_t* dL_out, int16_t* dR_out) {
    size_t P = (size_t)W * H, V = P * D;
    uint8_t* Y = (uint8_t*)malloc(P);
    uint64_t* cL = (uint64_t*)malloc(8 * P);
    uint64_t* cR = (uint64_t*)malloc(8 * P);
    uint8_t* aL = (uint8_t*)malloc(4 * P);
    uint8_t* aR = (uint8_t*)malloc(4 * P);
    int32_t* q = (int32_t*)malloc(4 * V);
    float* agg = (float*)malloc(4 * V);
    int16_t* dL = (int16_t*)malloc(2 * P);
    int16_t* dR = (int16_t*)malloc(2 * P);
    float* delL = (float*)malloc(4 * P);
    float* delR = (float*)malloc(4 * P);
    orc_grey(rgbL, W, H, Y);
    orc_census(Y, W, H, cw, ch, cL);
    orc_grey(rgbR, W, H, Y);
    orc_census(Y, W, H, cw, ch, cR);
    orc_arms(rgbL, W, H, L1, tau1, aL);
    orc_arms(rgbR, W, H, L1, tau1, aR);
    orc_cost(0, rgbL, rgbR, cL, cR, aL, W, H, D, L1, gamma, eps, lam_ad, lam_c, q);
    orc_aggregate(q, aL, W, H, D, iters, agg);
    orc_wta(agg, W, H, D, dL, delL);
    float* aggL = NULL;
    if (vote_iters > 0) {  /* the vote's sub-pixel step needs the left costs */
        aggL = (float*)malloc(4 * V);
        memcpy(aggL, agg, 4 * V);
    }
    orc_cost(1, rgbL, rgbR, cL, cR, aR, W, H, D, L1, gamma, eps, lam_ad, lam_c, q);
    orc_aggregate(q, aR, W, H, D, iters, agg);
    orc_wta(agg, W, H, D, dR, delR);
    orc_lrcheck(dL, delL, dR, W, H, maxdiff, subpixel, disp, valid);
    if (vote_iters > 0) {
        int16_t* dv = (int16_t*)malloc(2 * P);
        orc_vote(dL, valid, aL, W, H, D, vote_iters, dv);
        orc_vote_finish(aggL, dv, W, H, D, subpixel, disp, valid);
        free(dv);
        free(aggL);
    }
    if (dL_out) memcpy(dL_out, dL, 2 * P);
    if (dR_out) memcpy(dR_out, dR, 2 * P);
    free(Y); free(cL); free(cR); free(aL); free(aR); free(q); free(agg);
    free(dL); free(dR); free(delL); free(delR);
}

/* ------------------------------------------------------------------------
 * Differentiable soft-argmin form, in double precision.
 *
 * Forward: the real-valued Eq. 1 cost
 *   c(p,d) = alpha_p (1 - exp(-(s/3)/lambda_ad)) + (1 - alpha_p)(1 - exp(-h/lambda_census))
 * with alpha_p = 1 - exp(-gamma / (Lmin(p) + eps)) and c = 1 where the partner
 * is outside the image; two normalised region means (Eq. 2 twice, no
 * rounding); soft-argmin  dhat_p = sum_d d softmax_d(-A2(p,d) / T).
 * Left view is the reference.
 * ---------------------------------------------------------------------- */

typedef struct {
    int W, H, D;
    const uint8_t* arms;
    double* n1;
    double* n2;
} soft_geom;

static void soft_counts(soft_geom* g) {
    int W = g->W, H = g->H;
    const uint8_t* A = g->arms;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            double n = 0;
            for (int yy = y - A[4 * (y * W + x) + 2]; yy <= y + A[4 * (y * W + x) + 3]; ++yy)
                n += A[4 * (yy * W + x)] + A[4 * (yy * W + x) + 1] + 1;
            g->n1[y * W + x] = n;
            n = 0;
            for (int xx = x - A[4 * (y * W + x)]; xx <= x + A[4 * (y * W + x) + 1]; ++xx)
                n += A[4 * (y * W + xx) + 2] + A[4 * (y * W + xx) + 3] + 1;
            g->n2[y * W + x] = n;
        }
}

/* Raw real-valued costs of slice d, plus dc/dlambda_ad and dc/dlambda_census. */
static void soft_cost_slice(const uint8_t* rgbL, const uint8_t* rgbR, const uint64_t* cL,
                            const uint64_t* cR, const uint8_t* arms, int W, int H, int d,
                            double gamma, double eps, double lam_ad, double lam_c, double* c,
                            double* dc_ad, double* dc_c) {
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            int i = y * W + x;
            if (x - d < 0) {
                c[i] = 1.0;
                if (dc_ad) dc_ad[i] = 0.0, dc_c[i] = 0.0;
                continue;
            }
            const uint8_t* a = rgbL + 3 * i;
            const uint8_t* b = rgbR + 3 * (i - d);
            double s = absi(a[0] - b[0]) + absi(a[1] - b[1]) + absi(a[2] - b[2]);
            uint64_t xr = cL[i] ^ cR[i - d];
            int h = 0;
            for (int k = 0; k < 64; ++k) h += (int)((xr >> k) & 1u);
            double al = 1.0 - exp(-gamma / ((double)lmin_of(arms + 4 * i) + eps));
            double ea = exp(-(s / 3.0) / lam_ad), ec = exp(-(double)h / lam_c);
            c[i] = al * (1.0 - ea) + (1.0 - al) * (1.0 - ec);
            if (dc_ad) {
                dc_ad[i] = -al * ea * (s / 3.0) / (lam_ad * lam_ad);
                dc_c[i] = -(1.0 - al) * ec * (double)h / (lam_c * lam_c);
            }
        }
}

/* Two normalised region means of one slice, straight from the definition. */
static void soft_agg_slice(const soft_geom* g, const double* c, double* tmp1, double* tmp2,
                           double* A2) {
    int W = g->W, H = g->H;
    const uint8_t* A = g->arms;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            double s = 0;
            for (int xx = x - A[4 * (y * W + x)]; xx <= x + A[4 * (y * W + x) + 1]; ++xx)
                s += c[y * W + xx];
            tmp1[y * W + x] = s;
        }
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            double s = 0;
            for (int yy = y - A[4 * (y * W + x) + 2]; yy <= y + A[4 * (y * W + x) + 3]; ++yy)
                s += tmp1[yy * W + x];
            tmp2[y * W + x] = s / g->n1[y * W + x];
        }
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            double s = 0;
            for (int yy = y - A[4 * (y * W + x) + 2]; yy <= y + A[4 * (y * W + x) + 3]; ++yy)
                s += tmp2[yy * W + x];
            tmp1[y * W + x] = s;
        }
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            double s = 0;
            for (int xx = x - A[4 * (y * W + x)]; xx <= x + A[4 * (y * W + x) + 1]; ++xx)
                s += tmp1[y * W + xx];
            A2[y * W + x] = s / g->n2[y * W + x];
        }
}

/* Forward.  Outputs dhat (H x W) and, when non-null, the aggregated volume
 * A2 (D x H x W). */
void orc_soft_forward(const uint8_t* rgbL, const uint8_t* rgbR, const uint64_t* cL,
                      const uint64_t* cR, const uint8_t* armsL, int W, int H, int D,
                      double gamma, double eps, double lam_ad, double lam_c, double T,
                      double* dhat, double* A2_out) {
    size_t P = (size_t)W * H;
    soft_geom g = {W, H, D, armsL, (double*)malloc(8 * P), (double*)malloc(8 * P)};
    soft_counts(&g);
    double* vol = (double*)malloc(8 * P * D);
    double* c = (double*)malloc(8 * P);
    double* t1 = (double*)malloc(8 * P);
    double* t2 = (double*)malloc(8 * P);
    for (int d = 0; d < D; ++d) {
        soft_cost_slice(rgbL, rgbR, cL, cR, armsL, W, H, d, gamma, eps, lam_ad, lam_c, c, NULL,
                        NULL);
        soft_agg_slice(&g, c, t1, t2, vol + (size_t)d * P);
    }
    for (size_t i = 0; i < P; ++i) {
        double mn = vol[i];
        for (int d = 1; d < D; ++d)
            if (vol[(size_t)d * P + i] < mn) mn = vol[(size_t)d * P + i];
        double z = 0, zd = 0;
        for (int d = 0; d < D; ++d) {
            double e = exp(-(vol[(size_t)d * P + i] - mn) / T);
            z += e;
            zd += d * e;
        }
        dhat[i] = zd / z;
    }
    if (A2_out) memcpy(A2_out, vol, 8 * P * D);
    free(vol); free(c); free(t1); free(t2); free(g.n1); free(g.n2);
}

/* Gradient of L = sum_p gdhat_p dhat_p with respect to (lambda_ad,
 * lambda_census, T), by the chain rule written out:
 *   dL/dA2(p,d) = gdhat_p w_pd (dhat_p - d) / T
 *   dL/dT       = sum_p gdhat_p sum_d w_pd (d - dhat_p) A2(p,d) / T^2
 * then the adjoint of each region sum (every output scatters its adjoint back
 * over the same ranges it summed), divided by N where the forward divided,
 * and finally dc/dlambda.  grad[0..2] = (lambda_ad, lambda_census, T). */
static void soft_grad_impl(const uint8_t* rgbL, const uint8_t* rgbR, const uint64_t* cL,
                           const uint64_t* cR, const uint8_t* armsL, int W, int H, int D,
                           double gamma, double eps, double lam_ad, double lam_c, double T,
                           const double* gdhat, int magnitude, double* grad) {
    size_t P = (size_t)W * H;
    soft_geom g = {W, H, D, armsL, (double*)malloc(8 * P), (double*)malloc(8 * P)};
    soft_counts(&g);
    double* vol = (double*)malloc(8 * P * D);
    double* dhat = (double*)malloc(8 * P);
    orc_soft_forward(rgbL, rgbR, cL, cR, armsL, W, H, D, gamma, eps, lam_ad, lam_c, T, dhat, vol);
    double* c = (double*)malloc(8 * P);
    double* dca = (double*)malloc(8 * P);
    double* dcc = (double*)malloc(8 * P);
    double* gA = (double*)malloc(8 * P);
    double* g1 = (double*)malloc(8 * P);
    double* g2 = (double*)malloc(8 * P);
    double* mn = (double*)malloc(8 * P);
    double* z = (double*)malloc(8 * P);
    const uint8_t* A = armsL;
    for (size_t i = 0; i < P; ++i) {
        double m = vol[i];
        for (int d = 1; d < D; ++d)
            if (vol[(size_t)d * P + i] < m) m = vol[(size_t)d * P + i];
        double s = 0;
        for (int d = 0; d < D; ++d) s += exp(-(vol[(size_t)d * P + i] - m) / T);
        mn[i] = m;
        z[i] = s;
    }
    double gad = 0, gc = 0, gT = 0;
    for (int d = 0; d < D; ++d) {
        const double* a2 = vol + (size_t)d * P;
        for (size_t i = 0; i < P; ++i) {
            double w = exp(-(a2[i] - mn[i]) / T) / z[i];
            gA[i] = gdhat[i] * w * (dhat[i] - d) / T;
            double tT = gdhat[i] * w * (d - dhat[i]) * a2[i] / (T * T);
            if (magnitude) gA[i] = fabs(gA[i]), tT = fabs(tT);
            gT += tT;
        }
        /* adjoint of A2 = S2 / N2, S2 = horizontal sum of E2 over p's arms */
        memset(g1, 0, 8 * P);
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                double v = gA[y * W + x] / g.n2[y * W + x];
                for (int xx = x - A[4 * (y * W + x)]; xx <= x + A[4 * (y * W + x) + 1]; ++xx)
                    g1[y * W + xx] += v;
            }
        /* adjoint of E2 = vertical sum of a1 over the column pixel's arms */
        memset(g2, 0, 8 * P);
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x)
                for (int yy = y - A[4 * (y * W + x) + 2]; yy <= y + A[4 * (y * W + x) + 3]; ++yy)
                    g2[yy * W + x] += g1[y * W + x];
        /* adjoint of a1 = S1 / N1, S1 = vertical sum of E1 */
        memset(g1, 0, 8 * P);
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                double v = g2[y * W + x] / g.n1[y * W + x];
                for (int yy = y - A[4 * (y * W + x) + 2]; yy <= y + A[4 * (y * W + x) + 3]; ++yy)
                    g1[yy * W + x] += v;
            }
        /* adjoint of E1 = horizontal sum of c */
        memset(g2, 0, 8 * P);
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x)
                for (int xx = x - A[4 * (y * W + x)]; xx <= x + A[4 * (y * W + x) + 1]; ++xx)
                    g2[y * W + xx] += g1[y * W + x];
        soft_cost_slice(rgbL, rgbR, cL, cR, armsL, W, H, d, gamma, eps, lam_ad, lam_c, c, dca,
                        dcc);
        for (size_t i = 0; i < P; ++i) {
            gad += g2[i] * (magnitude ? fabs(dca[i]) : dca[i]);
            gc += g2[i] * (magnitude ? fabs(dcc[i]) : dcc[i]);
        }
    }
    grad[0] = gad;
    grad[1] = gc;
    grad[2] = gT;
    free(vol); free(dhat); free(c); free(dca); free(dcc); free(gA); free(g1); free(g2);
    free(mn); free(z); free(g.n1); free(g.n2);
}

void orc_soft_grad(const uint8_t* rgbL, const uint8_t* rgbR, const uint64_t* cL,
                   const uint64_t* cR, const uint8_t* armsL, int W, int H, int D, double gamma,
                   double eps, double lam_ad, double lam_c, double T, const double* gdhat,
                   double* grad) {
    soft_grad_impl(rgbL, rgbR, cL, cR, armsL, W, H, D, gamma, eps, lam_ad, lam_c, T, gdhat, 0,
                   grad);
}

/* The same chain with every per-entry term replaced by its magnitude: the
 * seed |dL/dA2|, the temperature terms |.|, and |dc/dlambda|.  The region
 * adjoints are non-negative linear maps, so mag[k] bounds the sum of the
 * absolute values of the terms that add up to grad[k]: the scale against
 * which a float evaluation's rounding error in grad[k] is measured. */
void orc_soft_grad_mag(const uint8_t* rgbL, const uint8_t* rgbR, const uint64_t* cL,
                       const uint64_t* cR, const uint8_t* armsL, int W, int H, int D,
                       double gamma, double eps, double lam_ad, double lam_c, double T,
                       const double* gdhat, double* mag) {
    soft_grad_impl(rgbL, rgbR, cL, cR, armsL, W, H, D, gamma, eps, lam_ad, lam_c, T, gdhat, 1,
                   mag);
}
