/* Exhaustive check of the final division of the two-stage aggregation.
 *
 * Claim: for every integer N in [1, NMAX] and every float a in [0, 2^31),
 * with y = RN(1/N), q0 = RN(a y), r = RN(a - q0 N) (one fused multiply-add)
 * and q = RN(q0 + r y) (one fused multiply-add), q == RN(a / N).
 *
 * Reductions (both exact, so checking the reduced set checks the claim):
 *  - N = 2^k N' with N' odd: y = 2^-k RN(1/N') and every step scales by
 *    2^-k, so only odd N are checked;
 *  - a = m 2^e with m an integer in [2^23, 2^24): a y, a - q0 N and
 *    q0 + r y scale by 2^e and nothing leaves the normal range (the kernel
 *    also folds a 2^-20 scale into y and N, which is exact too), so only
 *    m is enumerated; a = 0 gives 0 on both sides.
 * The reference RN(m / N) is the double quotient rounded to float: a p-bit
 * quotient rounded first to 53 >= 2p + 2 bits and then to p bits is the
 * correctly rounded quotient (Figueroa's double-rounding theorem).
 *
 * Usage: div_exhaustive [NMAX] [threads]; prints the count of checks and
 * exits 1 on the first counterexample.  Built with -O2 -mfma
 * -ffp-contract=off so that fmaf is the hardware fused multiply-add and no
 * other product is fused. */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

static int g_nmax = 1225, g_threads = 8;
static volatile int g_fail = 0;

typedef struct {
    int t;
    unsigned long long checks;
} job;

static void* run(void* arg) {
    job* j = (job*)arg;
    for (int N = 1 + 2 * j->t; N <= g_nmax && !g_fail; N += 2 * g_threads) {
        const float n = (float)N;
        const float y = 1.0f / n;
        const double dn = (double)N;
        for (uint32_t m = 1u << 23; m < (1u << 24); ++m) {
            const float a = (float)m;
            const float q0 = a * y;
            const float r = fmaf(-q0, n, a);
            const float q = fmaf(r, y, q0);
            const float want = (float)((double)m / dn);
            if (q != want) {
                printf("counterexample: N=%d m=%u got %a want %a\n", N, m, q, want);
                g_fail = 1;
                break;
            }
        }
        j->checks += 1u << 23;
    }
    return NULL;
}

int main(int argc, char** argv) {
    if (argc > 1) g_nmax = atoi(argv[1]);
    if (argc > 2) g_threads = atoi(argv[2]);
    if (g_threads < 1) g_threads = 1;
    pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * g_threads);
    job* jobs = (job*)calloc(g_threads, sizeof(job));
    for (int t = 0; t < g_threads; ++t) {
        jobs[t].t = t;
        pthread_create(&th[t], NULL, run, &jobs[t]);
    }
    unsigned long long total = 0;
    for (int t = 0; t < g_threads; ++t) {
        pthread_join(th[t], NULL);
        total += jobs[t].checks;
    }
    printf("checks %llu nmax %d fail %d\n", total, g_nmax, g_fail);
    return g_fail ? 1 : 0;
}
