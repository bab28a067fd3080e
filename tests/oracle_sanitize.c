/* Driver that runs every public function of the C oracle on small seeded
 * inputs, built together with oracle/dco_oracle.c under AddressSanitizer
 * and UndefinedBehaviorSanitizer (host code only) by a CPU test.  Shapes
 * include the smallest image the census window allows, ragged sizes, a
 * disparity range next to the width, both aggregation forms, short arm
 * limits and the Eq. 4 vote, so that every border branch runs.  Exits 0
 * when no sanitizer fires (the sanitizers abort otherwise). */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void orc_match(const uint8_t* rgbL, const uint8_t* rgbR, int W, int H, int D, int cw, int ch,
               int L1, int tau1, float gamma, float eps, float lam_ad, float lam_c, int iters,
               int maxdiff, int subpixel, int vote_iters, float* disp, uint8_t* valid,
               int16_t* dL_out, int16_t* dR_out);
void orc_flow_terms(const float* F, int w, int h, float* M, float* score);
void orc_flow_fuse(const float* past, const float* future, int w, int h, int R, float* out);
void orc_contour(const uint8_t* Y, int W, int H, const float* Mn, int w, int h, float Thigh,
                 float Tlow, float Tdepth, uint8_t* B, float* MI);
void orc_grey(const uint8_t* rgb, int W, int H, uint8_t* Y);
void orc_census(const uint8_t* Y, int W, int H, int cw, int ch, uint64_t* out);
void orc_arms(const uint8_t* rgb, int W, int H, int L1, int tau1, uint8_t* arms);
void orc_downscale2(const uint8_t* rgb, int W, int H, uint8_t* out);
void orc_depth_half(const float* disp, const uint8_t* valid, int W, int H, float fB,
                    float* dfull, float* depth);
void orc_soft_forward(const uint8_t* rgbL, const uint8_t* rgbR, const uint64_t* cL,
                      const uint64_t* cR, const uint8_t* armsL, int W, int H, int D,
                      double gamma, double eps, double lam_ad, double lam_c, double T,
                      double* dhat, double* A2_out);
void orc_soft_grad(const uint8_t* rgbL, const uint8_t* rgbR, const uint64_t* cL,
                   const uint64_t* cR, const uint8_t* armsL, int W, int H, int D, double gamma,
                   double eps, double lam_ad, double lam_c, double T, const double* gdhat,
                   double* grad);

static uint64_t g_state = 0x9e3779b97f4a7c15ull;
static uint32_t rnd(void) {  /* splitmix64 */
    uint64_t z = (g_state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return (uint32_t)((z ^ (z >> 31)) >> 32);
}

/* blocky texture with flat patches, so that arms reach the limit */
static uint8_t* image(int W, int H, int block) {
    uint8_t* p = (uint8_t*)malloc((size_t)W * H * 3);
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x)
            for (int c = 0; c < 3; ++c) {
                uint32_t v = (uint32_t)(((x / block) * 131 + (y / block) * 71 + c * 29) % 251);
                p[3 * ((size_t)y * W + x) + c] = (uint8_t)(v + (rnd() % 3));
            }
    return p;
}

static void match_case(int W, int H, int D, int L1, int iters, int vote) {
    uint8_t* L = image(W, H, 5);
    uint8_t* R = (uint8_t*)malloc((size_t)W * H * 3);
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            int xs = x + 3 < W ? x + 3 : W - 1;   /* right view: left shifted by 3 */
            memcpy(R + 3 * ((size_t)y * W + x), L + 3 * ((size_t)y * W + xs), 3);
        }
    size_t P = (size_t)W * H;
    float* disp = (float*)malloc(4 * P);
    uint8_t* valid = (uint8_t*)malloc(P);
    int16_t* dL = (int16_t*)malloc(2 * P);
    int16_t* dR = (int16_t*)malloc(2 * P);
    orc_match(L, R, W, H, D, 9, 7, L1, 20, 1.0f, 0.8f, 10.0f, 40.0f, iters, 0, 1, vote, disp,
              valid, dL, dR);
    free(L), free(R), free(disp), free(valid), free(dL), free(dR);
}

static void contour_case(int W, int H) {
    int w = W / 2, h = H / 2;
    float* past = (float*)malloc(sizeof(float) * 2 * w * h);
    float* fut = (float*)malloc(sizeof(float) * 2 * w * h);
    for (int i = 0; i < 2 * w * h; ++i) {
        past[i] = (i % 7 == 0) ? 0.0f : (float)((int)(rnd() % 200) - 100) / 16.0f;
        fut[i] = (float)((int)(rnd() % 200) - 100) / 16.0f;
    }
    float* M = (float*)malloc(sizeof(float) * w * h);
    float* S = (float*)malloc(sizeof(float) * w * h);
    float* Mn = (float*)malloc(sizeof(float) * w * h);
    orc_flow_terms(past, w, h, M, S);
    orc_flow_fuse(past, fut, w, h, 2, Mn);
    uint8_t* rgb = image(W, H, 3);
    uint8_t* Y = (uint8_t*)malloc((size_t)W * H);
    orc_grey(rgb, W, H, Y);
    uint8_t* B = (uint8_t*)malloc((size_t)W * H);
    float* MI = (float*)malloc(sizeof(float) * W * H);
    orc_contour(Y, W, H, Mn, w, h, 0.06f, 0.03f, 0.03f, B, MI);
    free(past), free(fut), free(M), free(S), free(Mn), free(rgb), free(Y), free(B), free(MI);
}

static void half_case(int W, int H) {
    uint8_t* rgb = image(W, H, 4);
    uint8_t* out = (uint8_t*)malloc((size_t)(W / 2) * (H / 2) * 3);
    orc_downscale2(rgb, W, H, out);
    int w = W / 2, h = H / 2;
    float* d = (float*)malloc(sizeof(float) * w * h);
    uint8_t* v = (uint8_t*)malloc((size_t)w * h);
    for (int i = 0; i < w * h; ++i) {
        d[i] = (float)(rnd() % 40) / 4.0f;
        v[i] = (uint8_t)(rnd() & 1);
    }
    float* df = (float*)malloc(sizeof(float) * w * h);
    float* dep = (float*)malloc(sizeof(float) * w * h);
    orc_depth_half(d, v, w, h, 800.0f, df, dep);
    free(rgb), free(out), free(d), free(v), free(df), free(dep);
}

static void soft_case(int W, int H, int D) {
    uint8_t* L = image(W, H, 4);
    uint8_t* R = image(W, H, 4);
    size_t P = (size_t)W * H;
    uint8_t* Y = (uint8_t*)malloc(P);
    uint64_t* cL = (uint64_t*)malloc(8 * P);
    uint64_t* cR = (uint64_t*)malloc(8 * P);
    uint8_t* aL = (uint8_t*)malloc(4 * P);
    orc_grey(L, W, H, Y);
    orc_census(Y, W, H, 9, 7, cL);
    orc_grey(R, W, H, Y);
    orc_census(Y, W, H, 9, 7, cR);
    orc_arms(L, W, H, 17, 20, aL);
    double* dhat = (double*)malloc(8 * P);
    double* vol = (double*)malloc(8 * P * D);
    double* g = (double*)malloc(8 * P);
    for (size_t i = 0; i < P; ++i) g[i] = (double)(rnd() % 3) - 1.0;
    double grad[3];
    orc_soft_forward(L, R, cL, cR, aL, W, H, D, 1.0, 0.8, 10.0, 30.0, 1.0, dhat, vol);
    orc_soft_grad(L, R, cL, cR, aL, W, H, D, 1.0, 0.8, 10.0, 30.0, 1.0, g, grad);
    free(L), free(R), free(Y), free(cL), free(cR), free(aL), free(dhat), free(vol), free(g);
}

int main(void) {
    match_case(9, 7, 1, 17, 2, 0);     /* smallest image the census window allows */
    match_case(9, 7, 8, 17, 1, 2);
    match_case(37, 23, 36, 17, 2, 2);  /* D next to the width */
    match_case(53, 41, 12, 4, 2, 1);   /* short arms */
    match_case(64, 48, 16, 17, 1, 0);
    match_case(70, 19, 20, 0, 2, 2);   /* no arms at all */
    contour_case(30, 22);
    contour_case(31, 17);              /* odd full sizes */
    half_case(33, 21);
    soft_case(26, 18, 8);
    puts("sanitized oracle run: ok");
    return 0;
}
