/*
 * Plain FP64 CPU oracle: see oracle.h.  TEST INFRASTRUCTURE ONLY -- loaded by
 * the tests, the smoke check and the benchmark's CPU-baseline leg; never by the
 * product path.
 *
 * Built with -O2 -ffp-contract=off and no fast-math: every operation below is
 * one IEEE double operation in the order written, except the one explicit fma
 * of the point map.
 *
 * Each step follows the paper (Honkonen & Honkonen, arXiv:1803.07560):
 *   action          section 2, Eq. Gen2 and the constants a, tau, nu, D after it;
 *                   periodicity in space and time as stated below Gen2
 *   observables     section 2, Eq. Gen2 (the factors v(t_i,x_k) v(t_i,x_n))
 *   normalisation   section 2 (C computed numerically) and section 4 (each value
 *                   divided by the integral with the velocity factors set to 1)
 *   subvolumes      section 3 (volume subdivided; one extent per dimension)
 *   error bar       section 3, the serial integrand's output (result, absolute error)
 * Philox4x32-10 follows Salmon et al., "Parallel random numbers: as easy as
 * 1, 2, 3" (SC'11).
 */
#include "oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ Philox */

/* Round multipliers and key increments published with Philox4x32. */
static const uint32_t PHILOX_M0 = 0xD2511F53u;
static const uint32_t PHILOX_M1 = 0xCD9E8D57u;
static const uint32_t PHILOX_W0 = 0x9E3779B9u;
static const uint32_t PHILOX_W1 = 0xBB67AE85u;

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { /* key schedule: a Weyl sequence between rounds */
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

void oracle_words(int32_t d, uint64_t seed, uint64_t id, uint64_t index, uint32_t *words)
{
    const int32_t nb = (d + 3) / 4;
    const uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    for (int32_t j = 0; j < nb; ++j) {
        uint64_t q = index * (uint64_t)nb + (uint64_t)j;
        uint32_t ctr[4] = { (uint32_t)q, (uint32_t)(q >> 32), (uint32_t)id, (uint32_t)(id >> 32) };
        uint32_t blk[4];
        oracle_philox4x32_10(ctr, key, blk);
        for (int t = 0; t < 4; ++t)
            if (4 * j + t < d)
                words[4 * j + t] = blk[t];
    }
}

/* --------------------------------------------------------------- the point */

static void box_map(int32_t d, const double *lo, const double *hi, double *scale, double *base)
{
    for (int32_t k = 0; k < d; ++k) {
        scale[k] = (hi[k] - lo[k]) * 0x1p-32;
        base[k] = lo[k] + 0.5 * scale[k];
    }
}

void oracle_point(int32_t d, uint64_t seed, uint64_t id, const double *lo, const double *hi,
                  uint64_t index, double *u)
{
    uint32_t *x = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)d);
    double *scale = (double *)malloc(sizeof(double) * (size_t)d);
    double *base = (double *)malloc(sizeof(double) * (size_t)d);
    oracle_words(d, seed, id, index, x);
    box_map(d, lo, hi, scale, base);
    for (int32_t k = 0; k < d; ++k)
        u[k] = fma((double)x[k], scale[k], base[k]);
    free(x);
    free(scale);
    free(base);
}

/* -------------------------------------------------------------- the action */

static int lattice_ok(const oracle_lattice *lat)
{
    if (!lat || lat->nx < 1 || lat->nt < 1)
        return 0;
    if (!(lat->D > 0) || !(lat->a > 0) || !(lat->tau > 0))
        return 0;
    if (!isfinite(lat->nu) || !isfinite(lat->D) || !isfinite(lat->a) || !isfinite(lat->tau) ||
        !isfinite(lat->g) || !isfinite(lat->m2))
        return 0;
    if (lat->observable != ORACLE_OBS_ANCHOR && lat->observable != ORACLE_OBS_AVERAGED)
        return 0;
    return 1;
}

/* v(t_l, x_m) with both indices taken periodically. */
static double site(const oracle_lattice *lat, const double *u, int32_t l, int32_t m)
{
    int32_t L = lat->nt, M = lat->nx;
    l = ((l % L) + L) % L;
    m = ((m % M) + M) % M;
    return u[l * M + m];
}

int oracle_residual(const oracle_lattice *lat, const double *u, double *R)
{
    if (!lattice_ok(lat) || !u || !R)
        return -1;
    const double a = lat->a, tau = lat->tau, nu = lat->nu, g = lat->g;
    for (int32_t l = 0; l < lat->nt; ++l) {
        for (int32_t m = 0; m < lat->nx; ++m) {
            double v = site(lat, u, l, m);
            double v_next_t = site(lat, u, l + 1, m);
            double v_right = site(lat, u, l, m + 1);
            double v_left = site(lat, u, l, m - 1);
            /* forward time difference */
            double time_diff = v_next_t - v;
            /* central first derivative in space */
            double grad = (v_right - v_left) / (2.0 * a);
            /* three-point Laplacian */
            double lap = (v_right - 2.0 * v + v_left) / (a * a);
            R[l * lat->nx + m] = time_diff + (g * v * grad - nu * lap) * tau;
        }
    }
    return 0;
}

double oracle_action(const oracle_lattice *lat, const double *u)
{
    if (!lattice_ok(lat) || !u)
        return NAN;
    const int32_t d = lat->nx * lat->nt;
    double *R = (double *)malloc(sizeof(double) * (size_t)d);
    oracle_residual(lat, u, R);
    double sum_r2 = 0.0, sum_u2 = 0.0;
    for (int32_t k = 0; k < d; ++k) {
        sum_r2 += R[k] * R[k];
        sum_u2 += u[k] * u[k];
    }
    free(R);
    double S = sum_r2 / (2.0 * lat->D * lat->tau);
    if (lat->m2 != 0.0)
        S += 0.5 * lat->m2 * sum_u2;
    return S;
}

/* Section 4's equal-time correlation <v(t, x) v(t, x + r)>: either the single
 * product the paper writes, or its mean over all nx*nt anchors (the action is
 * invariant under periodic shifts in space and time, so both have the same
 * expectation). */
int oracle_observable(const oracle_lattice *lat, const double *u, double *p)
{
    if (!lattice_ok(lat) || !u || !p)
        return -1;
    const int32_t nx = lat->nx, nt = lat->nt;
    for (int32_t r = 0; r < nx; ++r) {
        if (lat->observable == ORACLE_OBS_ANCHOR) {
            p[r] = site(lat, u, 0, 0) * site(lat, u, 0, r);
            continue;
        }
        double sum = 0.0;
        for (int32_t l = 0; l < nt; ++l)
            for (int32_t m = 0; m < nx; ++m)
                sum += site(lat, u, l, m) * site(lat, u, l, m + r);
        p[r] = sum / ((double)nx * (double)nt);
    }
    return 0;
}

int oracle_action_batch(const oracle_lattice *lat, size_t n, const double *u, double *S)
{
    if (!lattice_ok(lat) || (n && (!u || !S)))
        return -1;
    const size_t d = (size_t)lat->nx * (size_t)lat->nt;
    for (size_t i = 0; i < n; ++i)
        S[i] = oracle_action(lat, u + i * d);
    return 0;
}

/* ----------------------------------------------------- compensated sums */

typedef struct {
    double s, c;
} neumaier;

static void nm_add(neumaier *acc, double x)
{
    double t = acc->s + x;
    if (fabs(acc->s) >= fabs(x))
        acc->c += (acc->s - t) + x;
    else
        acc->c += (x - t) + acc->s;
    acc->s = t;
}

static double nm_value(const neumaier *acc) { return acc->s + acc->c; }

/* ------------------------------------------------- per-subvolume sums */

typedef struct {
    const oracle_lattice *lat;
    uint64_t seed;
    size_t nsub;
    const uint64_t *id;
    const double *lo, *hi;
    const uint64_t *n, *offset;
    double *out;
    int split; /* 0: sums record, 1: split statistics */
    int32_t nthreads, tid;
} sums_job;

static void subvolume_sums(const sums_job *job, size_t s)
{
    const oracle_lattice *lat = job->lat;
    const int32_t nx = lat->nx, d = lat->nx * lat->nt;
    const double *lo = job->lo + s * (size_t)d, *hi = job->hi + s * (size_t)d;
    uint32_t *x = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)d);
    double *u = (double *)malloc(sizeof(double) * (size_t)d);
    double *scale = (double *)malloc(sizeof(double) * (size_t)d);
    double *base = (double *)malloc(sizeof(double) * (size_t)d);
    double *p = (double *)malloc(sizeof(double) * (size_t)nx);
    box_map(d, lo, hi, scale, base);

    /* record layout: n, w, w^2, p_r w, (p_r w)^2, p_r w^2 -- or, for the split
     * statistics, sum_U w and sum_U w^2 per dimension */
    const int32_t len = job->split ? 2 * d : ORACLE_SUMS_LEN(nx);
    neumaier *acc = (neumaier *)calloc((size_t)len, sizeof(neumaier));

    const uint64_t first = job->offset[s], count = job->n[s];
    for (uint64_t i = 0; i < count; ++i) {
        oracle_words(d, job->seed, job->id[s], first + i, x);
        for (int32_t k = 0; k < d; ++k)
            u[k] = fma((double)x[k], scale[k], base[k]);
        double w = exp(-oracle_action(lat, u));
        if (job->split) {
            for (int32_t k = 0; k < d; ++k) {
                if (x[k] >> 31) { /* upper half of the box along k */
                    nm_add(&acc[k], w);
                    nm_add(&acc[d + k], w * w);
                }
            }
            continue;
        }
        nm_add(&acc[0], 1.0);
        nm_add(&acc[1], w);
        nm_add(&acc[2], w * w);
        oracle_observable(lat, u, p);
        for (int32_t r = 0; r < nx; ++r) {
            double pw = p[r] * w;
            nm_add(&acc[3 + r], pw);
            nm_add(&acc[3 + nx + r], pw * pw);
            nm_add(&acc[3 + 2 * nx + r], pw * w);
        }
    }
    double *out = job->out + s * (size_t)len;
    for (int32_t t = 0; t < len; ++t)
        out[t] = nm_value(&acc[t]);
    free(acc);
    free(x);
    free(u);
    free(scale);
    free(base);
    free(p);
}

static void *sums_worker(void *arg)
{
    const sums_job *job = (const sums_job *)arg;
    for (size_t s = (size_t)job->tid; s < job->nsub; s += (size_t)job->nthreads)
        subvolume_sums(job, s);
    return NULL;
}

static int run_sums(const oracle_lattice *lat, uint64_t seed, size_t nsub, const uint64_t *id,
                    const double *lo, const double *hi, const uint64_t *n,
                    const uint64_t *offset, double *out, int32_t nthreads, int split)
{
    if (!lattice_ok(lat))
        return -1;
    if (nsub == 0)
        return 0;
    if (!id || !lo || !hi || !n || !offset || !out)
        return -1;
    const int32_t d = lat->nx * lat->nt;
    for (size_t s = 0; s < nsub; ++s)
        for (int32_t k = 0; k < d; ++k)
            if (!(lo[s * d + k] < hi[s * d + k]) || !isfinite(lo[s * d + k]) ||
                !isfinite(hi[s * d + k]))
                return -1;
    if (nthreads < 1)
        nthreads = 1;
    if ((size_t)nthreads > nsub)
        nthreads = (int32_t)nsub;
    sums_job *jobs = (sums_job *)calloc((size_t)nthreads, sizeof(sums_job));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    for (int32_t t = 0; t < nthreads; ++t) {
        sums_job j = { lat, seed, nsub, id, lo, hi, n, offset, out, split, nthreads, t };
        jobs[t] = j;
    }
    int rc = 0;
    int32_t started = 0;
    for (int32_t t = 1; t < nthreads; ++t) {
        if (pthread_create(&th[t], NULL, sums_worker, &jobs[t]) != 0) {
            rc = -2;
            break;
        }
        ++started;
    }
    if (rc == 0)
        sums_worker(&jobs[0]);
    for (int32_t t = 1; t <= started; ++t)
        pthread_join(th[t], NULL);
    free(jobs);
    free(th);
    return rc;
}

int oracle_sums(const oracle_lattice *lat, uint64_t seed, size_t nsub, const uint64_t *id,
                const double *lo, const double *hi, const uint64_t *n, const uint64_t *offset,
                double *sums, int32_t nthreads)
{
    return run_sums(lat, seed, nsub, id, lo, hi, n, offset, sums, nthreads, 0);
}

int oracle_split_sums(const oracle_lattice *lat, uint64_t seed, size_t nsub, const uint64_t *id,
                      const double *lo, const double *hi, const uint64_t *n,
                      const uint64_t *offset, double *out, int32_t nthreads)
{
    return run_sums(lat, seed, nsub, id, lo, hi, n, offset, out, nthreads, 1);
}

/* ---------------------------------------------------------------- finalize */

int oracle_finalize(int32_t nx, int32_t d, size_t nsub, const double *lo, const double *hi,
                    const double *sums, double *result)
{
    if (nx < 1 || d < nx || !result || (nsub && (!lo || !hi || !sums)))
        return -1;
    const int32_t len = ORACLE_SUMS_LEN(nx);
    double *V = (double *)malloc(sizeof(double) * (nsub ? nsub : 1));
    neumaier Z = { 0, 0 }, varZ = { 0, 0 }, wsq = { 0, 0 }, nev = { 0, 0 };
    for (size_t s = 0; s < nsub; ++s) {
        const double *rec = sums + s * (size_t)len;
        double vol = 1.0;
        for (int32_t k = 0; k < d; ++k)
            vol *= hi[s * d + k] - lo[s * d + k];
        V[s] = vol;
        double n = rec[0];
        if (!(n >= 2.0)) {
            free(V);
            return -1;
        }
        nm_add(&Z, vol * rec[1] / n);
        nm_add(&varZ, vol * vol * (rec[2] - rec[1] * rec[1] / n) / (n * (n - 1.0)));
        nm_add(&wsq, (vol / n) * (vol / n) * rec[2]);
        nm_add(&nev, n);
    }
    const double z = nm_value(&Z);
    result[0] = z;
    result[1] = sqrt(fmax(nm_value(&varZ), 0.0));
    result[2] = log(z);
    result[3] = nm_value(&wsq) > 0 ? z * z / nm_value(&wsq) : 0.0;
    result[4] = nm_value(&nev);
    for (int32_t r = 0; r < nx; ++r) {
        neumaier N = { 0, 0 };
        for (size_t s = 0; s < nsub; ++s) {
            const double *rec = sums + s * (size_t)len;
            nm_add(&N, V[s] * rec[3 + r] / rec[0]);
        }
        const double C = nm_value(&N) / z;
        /* delta method for the ratio N/Z with the per-subvolume covariance */
        neumaier var = { 0, 0 };
        for (size_t s = 0; s < nsub; ++s) {
            const double *rec = sums + s * (size_t)len;
            const double n = rec[0], v2 = V[s] * V[s], nn = n * (n - 1.0);
            const double var_n = v2 * (rec[3 + nx + r] - rec[3 + r] * rec[3 + r] / n) / nn;
            const double var_z = v2 * (rec[2] - rec[1] * rec[1] / n) / nn;
            const double cov = v2 * (rec[3 + 2 * nx + r] - rec[3 + r] * rec[1] / n) / nn;
            nm_add(&var, var_n - 2.0 * C * cov + C * C * var_z);
        }
        result[5 + r] = C;
        result[5 + nx + r] = sqrt(fmax(nm_value(&var), 0.0)) / fabs(z);
    }
    free(V);
    return 0;
}

/* -------------------------------------------------------------- the plan */

int oracle_plan_uniform(int32_t d, const double *box_lo, const double *box_hi, int32_t k,
                        uint64_t *id, double *lo, double *hi)
{
    if (d < 1 || k < 0 || k > 40 || !box_lo || !box_hi || !id || !lo || !hi)
        return -1;
    const uint64_t count = (uint64_t)1 << k;
    for (uint64_t b = 0; b < count; ++b) {
        id[b] = count + b;
        double *l = lo + b * (uint64_t)d, *h = hi + b * (uint64_t)d;
        memcpy(l, box_lo, sizeof(double) * (size_t)d);
        memcpy(h, box_hi, sizeof(double) * (size_t)d);
        /* level t halves dimension t mod d; bit (k-1-t) of b picks the upper half */
        for (int32_t t = 0; t < k; ++t) {
            int32_t dim = t % d;
            double mid = 0.5 * (l[dim] + h[dim]);
            if ((b >> (k - 1 - t)) & 1)
                l[dim] = mid;
            else
                h[dim] = mid;
        }
    }
    return 0;
}

/* --------------------------------------------------------------- N-sphere */

int oracle_nsphere(int32_t dim, uint64_t seed, uint64_t id, const double *lo, const double *hi,
                   uint64_t n, double *out)
{
    if (dim < 1 || n < 2 || !lo || !hi || !out)
        return -1;
    double *u = (double *)malloc(sizeof(double) * (size_t)dim);
    neumaier sf = { 0, 0 }, sf2 = { 0, 0 };
    double vol = 1.0;
    for (int32_t k = 0; k < dim; ++k)
        vol *= hi[k] - lo[k];
    for (uint64_t i = 0; i < n; ++i) {
        oracle_point(dim, seed, id, lo, hi, i, u);
        double r2 = 0.0;
        for (int32_t k = 0; k < dim; ++k)
            r2 += u[k] * u[k];
        double f = r2 < 1.0 ? sqrt(1.0 - r2) : 0.0;
        nm_add(&sf, f);
        nm_add(&sf2, f * f);
    }
    free(u);
    const double nn = (double)n, mean = nm_value(&sf) / nn;
    const double var = (nm_value(&sf2) - nm_value(&sf) * mean) / (nn - 1.0);
    out[0] = nn;
    out[1] = nm_value(&sf);
    out[2] = nm_value(&sf2);
    out[3] = vol * mean;
    out[4] = vol * sqrt(fmax(var, 0.0) / nn);
    return 0;
}
