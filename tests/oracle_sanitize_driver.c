/* Exercises every entry point of the CPU oracle (test infrastructure) on small
 * inputs, threads included, so that a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer, or with ThreadSanitizer, can check its memory
 * accesses, arithmetic and thread use.  Exit status 0 and "ok" when every call
 * returns success; the sanitizers report on their own. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../oracle/oracle.h"

#define CHECK(x)                                                          \
    do {                                                                  \
        if ((x) != 0) {                                                   \
            fprintf(stderr, "%s:%d: %s failed\n", __FILE__, __LINE__, #x); \
            return 1;                                                     \
        }                                                                 \
    } while (0)

static oracle_lattice lat(int nx, int nt, double nu, int obs, int anti)
{
    oracle_lattice L;
    memset(&L, 0, sizeof L);
    L.nx = nx;
    L.nt = nt;
    L.nu = nu;
    L.D = 1.0;
    L.a = 1.0;
    L.tau = 1.0;
    L.g = 1.0;
    L.m2 = 0.0;
    L.observable = obs;
    L.antithetic = anti;
    return L;
}

static int run_shape(int nx, int nt, int nthreads)
{
    const int d = nx * nt, k = 3, ns = 1 << k;
    double box_lo[64], box_hi[64];
    for (int j = 0; j < d; ++j) {
        box_lo[j] = -2.0;
        box_hi[j] = 2.0;
    }
    uint64_t *id = malloc(sizeof(uint64_t) * ns), *n = malloc(sizeof(uint64_t) * ns);
    uint64_t *off = malloc(sizeof(uint64_t) * ns);
    double *lo = malloc(sizeof(double) * ns * d), *hi = malloc(sizeof(double) * ns * d);
    double *sums = malloc(sizeof(double) * ns * ORACLE_SUMS_LEN(nx));
    double *split = malloc(sizeof(double) * ns * 2 * d);
    double *res = malloc(sizeof(double) * ORACLE_RESULT_LEN(nx));
    CHECK(oracle_plan_uniform(d, box_lo, box_hi, k, id, lo, hi));
    for (int s = 0; s < ns; ++s) {
        n[s] = 50 + 7 * (uint64_t)s;
        off[s] = (uint64_t)s * 1000003u;
    }
    uint32_t words[64];
    double u[64], R[64], p[64];
    oracle_words(d, 5, id[0], 17, words);
    oracle_point(d, 5, id[0], lo, hi, 17, u);
    for (int obs = 0; obs <= 1; ++obs) {
        for (int anti = 0; anti <= 1; ++anti) {
            oracle_lattice L = lat(nx, nt, 0.7, obs, anti);
            CHECK(oracle_residual(&L, u, R));
            if (!isfinite(oracle_action(&L, u)))
                return 1;
            CHECK(oracle_observable(&L, u, p));
            CHECK(oracle_sums(&L, 3, ns, id, lo, hi, n, off, sums, nthreads));
            CHECK(oracle_finalize(nx, d, ns, lo, hi, sums, res));
            if (!anti)
                CHECK(oracle_split_sums(&L, 3, ns, id, lo, hi, n, off, split, nthreads));
        }
    }
    double S[4];
    double pts[4 * 64];
    for (int i = 0; i < 4; ++i)
        oracle_point(d, 7, id[1], lo + d, hi + d, (uint64_t)i, pts + i * d);
    oracle_lattice L0 = lat(nx, nt, 0.5, 0, 0);
    CHECK(oracle_action_batch(&L0, 4, pts, S));
    if (d <= 32) {
        double *E = malloc(sizeof(double) * d * d);
        double lambda[32], scale[32], log_k, hz;
        int32_t uni[32];
        CHECK(oracle_is_basis(nx, nt, E));
        CHECK(oracle_is_modes(&L0, box_lo, box_hi, lambda, uni, scale, &log_k));
        CHECK(oracle_is_point(&L0, box_lo, box_hi, 9, 3, 11, u, &hz));
        uint64_t sid[4] = {1, 2, (1ull << 63) | 1u, (1ull << 63) | 2u};
        uint64_t sn[4] = {40, 33, 21, 60}, soff[4] = {0, 5, 0, 1ull << 40};
        double *is = malloc(sizeof(double) * 4 * ORACLE_SUMS_LEN(nx));
        CHECK(oracle_is_sums(&L0, 9, box_lo, box_hi, 0.8, 4, sid, sn, soff, is, nthreads));
        free(is);
        free(E);
    }
    free(id);
    free(n);
    free(off);
    free(lo);
    free(hi);
    free(sums);
    free(split);
    free(res);
    return 0;
}

int main(void)
{
    const int shapes[][2] = {{1, 1}, {2, 1}, {3, 2}, {4, 2}, {5, 3}, {10, 2}, {16, 4}};
    for (size_t i = 0; i < sizeof shapes / sizeof shapes[0]; ++i)
        if (run_shape(shapes[i][0], shapes[i][1], 4) != 0)
            return 1;
    double box[3] = {-1.0, -1.0, -1.0}, box_hi[3] = {1.0, 1.0, 1.0}, out[5];
    if (oracle_nsphere(3, 1, 1, box, box_hi, 1000, out) != 0)
        return 1;
    printf("ok\n");
    return 0;
}
