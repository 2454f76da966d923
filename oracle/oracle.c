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
    if (lat->antithetic != 0 && lat->antithetic != 1)
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
    double gaussian_fraction; /* Gaussian-proposal records only */
    size_t nsub;
    const uint64_t *id;
    const double *lo, *hi;
    const uint64_t *n, *offset;
    double *out;
    int split; /* 0: sums record, 1: split statistics, 2: Gaussian-proposal record */
    int l1;      /* sums records: append sum |p_r w| per r */
    int shifted; /* sums records: weights exp(sigma - S), sigma = the smallest S */
    int32_t nthreads, tid;
} sums_job;

static void is_stream_sums(const sums_job *job, size_t s);

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
    double *ub = (double *)malloc(sizeof(double) * (size_t)d);
    double *pb = (double *)malloc(sizeof(double) * (size_t)nx);
    box_map(d, lo, hi, scale, base);
    const int pairs = lat->antithetic && !job->split;

    /* record layout: n, w, w^2, p_r w, (p_r w)^2, p_r w^2 [, |p_r w|] -- or, for
     * the split statistics, sum_U w and sum_U w^2 per dimension */
    const int32_t len = job->split ? 2 * d : ORACLE_SUMS_LEN(nx) + (job->l1 ? nx : 0);
    neumaier *acc = (neumaier *)calloc((size_t)len, sizeof(neumaier));

    const uint64_t first = job->offset[s], count = job->n[s];
    /* shifted weights: a first pass finds the smallest action of the
     * subvolume's points (both points of a pair), which every weight is taken
     * relative to; plain weights use sigma = 0, and 0 - S is -S exactly */
    double sigma = 0.0;
    if (job->shifted) {
        sigma = INFINITY;
        for (uint64_t i = 0; i < count; ++i) {
            oracle_words(d, job->seed, job->id[s], first + i, x);
            for (int32_t k = 0; k < d; ++k)
                u[k] = fma((double)x[k], scale[k], base[k]);
            sigma = fmin(sigma, oracle_action(lat, u));
            if (pairs) {
                for (int32_t k = 0; k < d; ++k)
                    ub[k] = fma((double)(0xFFFFFFFFu - x[k]), scale[k], base[k]);
                sigma = fmin(sigma, oracle_action(lat, ub));
            }
        }
    }
    for (uint64_t i = 0; i < count; ++i) {
        oracle_words(d, job->seed, job->id[s], first + i, x);
        for (int32_t k = 0; k < d; ++k)
            u[k] = fma((double)x[k], scale[k], base[k]);
        double w = exp(sigma - oracle_action(lat, u));
        if (job->split) {
            for (int32_t k = 0; k < d; ++k) {
                if (x[k] >> 31) { /* upper half of the box along k */
                    nm_add(&acc[k], w);
                    nm_add(&acc[d + k], w * w);
                }
            }
            continue;
        }
        oracle_observable(lat, u, p);
        if (pairs) {
            /* the partner point: the complemented words through the same map */
            for (int32_t k = 0; k < d; ++k)
                ub[k] = fma((double)(0xFFFFFFFFu - x[k]), scale[k], base[k]);
            const double wb = exp(sigma - oracle_action(lat, ub));
            oracle_observable(lat, ub, pb);
            for (int32_t r = 0; r < nx; ++r)
                p[r] = 0.5 * (p[r] * w + pb[r] * wb); /* now the pair's p_r w */
            w = 0.5 * (w + wb);
            nm_add(&acc[0], 1.0);
            nm_add(&acc[1], w);
            nm_add(&acc[2], w * w);
            for (int32_t r = 0; r < nx; ++r) {
                nm_add(&acc[3 + r], p[r]);
                nm_add(&acc[3 + nx + r], p[r] * p[r]);
                nm_add(&acc[3 + 2 * nx + r], p[r] * w);
                if (job->l1)
                    nm_add(&acc[3 + 3 * nx + r], fabs(p[r]));
            }
            continue;
        }
        nm_add(&acc[0], 1.0);
        nm_add(&acc[1], w);
        nm_add(&acc[2], w * w);
        for (int32_t r = 0; r < nx; ++r) {
            double pw = p[r] * w;
            nm_add(&acc[3 + r], pw);
            nm_add(&acc[3 + nx + r], pw * pw);
            nm_add(&acc[3 + 2 * nx + r], pw * w);
            if (job->l1)
                nm_add(&acc[3 + 3 * nx + r], fabs(pw));
        }
    }
    if (job->shifted) {
        /* [n, sigma, the rest of the sums record] */
        double *out = job->out + s * (size_t)(len + 1);
        out[0] = nm_value(&acc[0]);
        out[1] = sigma;
        for (int32_t t = 1; t < len; ++t)
            out[t + 1] = nm_value(&acc[t]);
    } else {
        double *out = job->out + s * (size_t)len;
        for (int32_t t = 0; t < len; ++t)
            out[t] = nm_value(&acc[t]);
    }
    free(acc);
    free(x);
    free(u);
    free(scale);
    free(base);
    free(p);
    free(ub);
    free(pb);
}

static void *sums_worker(void *arg)
{
    const sums_job *job = (const sums_job *)arg;
    for (size_t s = (size_t)job->tid; s < job->nsub; s += (size_t)job->nthreads) {
        if (job->split == 2)
            is_stream_sums(job, s);
        else
            subvolume_sums(job, s);
    }
    return NULL;
}

static int run_sums(const oracle_lattice *lat, uint64_t seed, size_t nsub, const uint64_t *id,
                    const double *lo, const double *hi, const uint64_t *n,
                    const uint64_t *offset, double *out, int32_t nthreads, int split,
                    double gaussian_fraction, int l1, int shifted)
{
    if (!lattice_ok(lat))
        return -1;
    if (split && lat->antithetic) /* pairs: plain sums records only */
        return -1;
    if (nsub == 0)
        return 0;
    if (!id || !lo || !hi || !n || !offset || !out)
        return -1;
    const int32_t d = lat->nx * lat->nt;
    const size_t rows = split == 2 ? 1 : nsub; /* one box for every stream */
    for (size_t s = 0; s < rows; ++s)
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
        sums_job j = { lat, seed, gaussian_fraction, nsub, id, lo, hi, n, offset, out,
                       split, l1, shifted, nthreads, t };
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
    return run_sums(lat, seed, nsub, id, lo, hi, n, offset, sums, nthreads, 0, 0.0, 0, 0);
}

int oracle_sums_l1(const oracle_lattice *lat, uint64_t seed, size_t nsub, const uint64_t *id,
                   const double *lo, const double *hi, const uint64_t *n, const uint64_t *offset,
                   double *sums, int32_t nthreads)
{
    return run_sums(lat, seed, nsub, id, lo, hi, n, offset, sums, nthreads, 0, 0.0, 1, 0);
}

int oracle_sums_shifted(const oracle_lattice *lat, uint64_t seed, size_t nsub,
                        const uint64_t *id, const double *lo, const double *hi, const uint64_t *n,
                        const uint64_t *offset, double *sums, int32_t nthreads)
{
    return run_sums(lat, seed, nsub, id, lo, hi, n, offset, sums, nthreads, 0, 0.0, 0, 1);
}

int oracle_sums_shifted_l1(const oracle_lattice *lat, uint64_t seed, size_t nsub,
                           const uint64_t *id, const double *lo, const double *hi,
                           const uint64_t *n, const uint64_t *offset, double *sums,
                           int32_t nthreads)
{
    return run_sums(lat, seed, nsub, id, lo, hi, n, offset, sums, nthreads, 0, 0.0, 1, 1);
}

int oracle_split_sums(const oracle_lattice *lat, uint64_t seed, size_t nsub, const uint64_t *id,
                      const double *lo, const double *hi, const uint64_t *n,
                      const uint64_t *offset, double *out, int32_t nthreads)
{
    return run_sums(lat, seed, nsub, id, lo, hi, n, offset, out, nthreads, 1, 0.0, 0, 0);
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

/* Shifted records [n, sigma, sums record without n] stand for the plain record
 * with first-order sums times exp(-sigma) and second-order sums times
 * exp(-2 sigma).  Every record is moved to the smallest sigma of the list (a
 * factor exp(sigma_min - sigma) <= 1, squared for second-order sums) and the
 * plain finalize runs on those; Z carries the factor exp(sigma_min), so
 * log Z = log(that Z) - sigma_min, while C(r), its errors and the effective
 * sample size are ratios in which the factor cancels. */
int oracle_finalize_shifted(int32_t nx, int32_t d, size_t nsub, const double *lo,
                            const double *hi, const double *sums, double *result)
{
    if (nx < 1 || d < nx || !result || nsub == 0 || !lo || !hi || !sums)
        return -1;
    const int32_t len = ORACLE_SUMS_LEN(nx), slen = len + 1;
    double smin = INFINITY;
    for (size_t s = 0; s < nsub; ++s)
        smin = fmin(smin, sums[s * (size_t)slen + 1]);
    if (!isfinite(smin))
        return -1;
    double *plain = (double *)malloc(sizeof(double) * nsub * (size_t)len);
    for (size_t s = 0; s < nsub; ++s) {
        const double *rec = sums + s * (size_t)slen;
        double *out = plain + s * (size_t)len;
        const double f1 = exp(smin - rec[1]), f2 = f1 * f1;
        out[0] = rec[0];
        out[1] = rec[2] * f1;
        out[2] = rec[3] * f2;
        for (int32_t r = 0; r < nx; ++r) {
            out[3 + r] = rec[4 + r] * f1;
            out[3 + nx + r] = rec[4 + nx + r] * f2;
            out[3 + 2 * nx + r] = rec[4 + 2 * nx + r] * f2;
        }
    }
    const int rc = oracle_finalize(nx, d, nsub, lo, hi, plain, result);
    free(plain);
    if (rc != 0)
        return rc;
    result[2] -= smin;             /* log Z */
    result[0] = exp(result[2]);    /* Z (may underflow; log Z does not) */
    result[1] *= exp(-smin);       /* Z_err */
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

/* ------------------------------------------- Gaussian-proposal sampling */
/*
 * Importance sampling of exp(-S) over a box with the Gaussian of the action's
 * quadratic part as proposal, mixed with the uniform density of the box.
 * Dropping the nonlinear term of Eq. Gen2 leaves S0 = u.P.u / 2 with
 * P = A^T A / (D tau) + m2 I, A = (T - 1) - (nu tau / a^2) L, T the periodic
 * shift in time and L the periodic second difference in space.  P is a
 * polynomial in the shifts, so the real Fourier basis of the lattice (tensor
 * product of the one-dimensional ones) diagonalises it.  The constant mode
 * (lambda = m2, 0 in the paper) is drawn uniformly over [-R, R] when its
 * Gaussian would be wider than the box (lambda R^2 < 4, R the largest |u| in
 * the box); every other mode is Gaussian with standard deviation
 * scale_j = min(1/sqrt(lambda_j), R) (a mode with lambda near 0, such as the
 * checkerboard at nu tau / a^2 = 1/2, gets the box's width).  With a_j = <u, e_j>
 * and z_j = a_j / scale_j the Gaussian proposal density is
 *     q_G(u) = exp(-sum_gaussian z_j^2 / 2) / K,
 *     K = (2R if the constant mode is uniform) * prod_gaussian sqrt(2 pi) scale_j
 * (every point of the box has |a_0| <= R).  Defensive mixture (Hesterberg,
 * Technometrics 1995): a fraction alpha of the samples comes from q_G, the rest
 * from the uniform density 1/V of the box, and every sample, from either, has
 * the weight
 *     W(u) = 1_box(u) exp(-S(u)) / (alpha q_G(u) + (1 - alpha) / V),
 * whose mean over all samples is Z and which is bounded by V / (1 - alpha):
 * the Gaussian alone gives heavy-tailed weights wherever the nonlinear term
 * cancels the linear residual, S ~ 0 where S0 is large.
 */

/* Vector b of the real orthonormal Fourier basis of period n, component m:
 * b = 0 constant; b = 2k-1 cosine and b = 2k sine of frequency k < n/2; the
 * last vector of an even period alternates in sign.  *k_out = frequency. */
static double fourier_basis(int32_t n, int32_t b, int32_t m, int32_t *k_out)
{
    const double two_pi = 6.283185307179586476925286766559;
    const int32_t k = (b + 1) / 2;
    if (k_out)
        *k_out = k;
    if (b == 0)
        return 1.0 / sqrt((double)n);
    if (n % 2 == 0 && b == n - 1)
        return ((m % 2) ? -1.0 : 1.0) / sqrt((double)n);
    const double angle = two_pi * (double)k * (double)m / (double)n;
    return sqrt(2.0 / (double)n) * ((b % 2) ? cos(angle) : sin(angle));
}

int oracle_is_basis(int32_t nx, int32_t nt, double *E)
{
    if (nx < 1 || nt < 1 || !E)
        return -1;
    const int32_t d = nx * nt;
    for (int32_t bt = 0; bt < nt; ++bt)
        for (int32_t bx = 0; bx < nx; ++bx) {
            const int32_t j = bt * nx + bx;
            for (int32_t l = 0; l < nt; ++l)
                for (int32_t m = 0; m < nx; ++m)
                    E[(size_t)(l * nx + m) * d + j] =
                        fourier_basis(nt, bt, l, NULL) * fourier_basis(nx, bx, m, NULL);
        }
    return 0;
}

static int is_box_ok(int32_t d, const double *lo, const double *hi)
{
    for (int32_t k = 0; k < d; ++k)
        if (!(lo[k] < hi[k]) || !isfinite(lo[k]) || !isfinite(hi[k]))
            return 0;
    return 1;
}

int oracle_is_modes(const oracle_lattice *lat, const double *lo, const double *hi,
                    double *lambda, int32_t *uniform, double *scale, double *log_k)
{
    if (!lattice_ok(lat) || !lo || !hi || !lambda || !uniform || !scale || !log_k)
        return -1;
    const int32_t nx = lat->nx, nt = lat->nt, d = nx * nt;
    if (!is_box_ok(d, lo, hi))
        return -1;
    const double two_pi = 6.283185307179586476925286766559;
    const double c = lat->nu * lat->tau / (lat->a * lat->a);
    double R2 = 0.0;
    for (int32_t k = 0; k < d; ++k)
        R2 += fmax(lo[k] * lo[k], hi[k] * hi[k]);
    const double R = sqrt(R2);
    double lk = 0.0;
    for (int32_t bt = 0; bt < nt; ++bt)
        for (int32_t bx = 0; bx < nx; ++bx) {
            int32_t kt, kx;
            fourier_basis(nt, bt, 0, &kt);
            fourier_basis(nx, bx, 0, &kx);
            /* eigenvalues of the periodic second differences */
            const double mt = 2.0 * cos(two_pi * kt / nt) - 2.0;
            const double mx = 2.0 * cos(two_pi * kx / nx) - 2.0;
            const int32_t j = bt * nx + bx;
            lambda[j] = (-mt - c * mt * mx + c * c * mx * mx) / (lat->D * lat->tau) + lat->m2;
            uniform[j] = j == 0 && lambda[j] * R2 < 4.0;
            if (uniform[j]) {
                scale[j] = R;
                lk += log(2.0 * R);
            } else {
                scale[j] = lambda[j] * R2 <= 1.0 ? R : 1.0 / sqrt(lambda[j]);
                lk += 0.5 * log(two_pi) + log(scale[j]);
            }
        }
    *log_k = lk;
    return 0;
}

/* Words per sample: mode j's normal comes from the Box-Muller pair of words
 * (2 floor(j/2), 2 floor(j/2) + 1), cosine for even j and sine for odd j, so
 * the pairs take 2 ceil(d/2) words; the next word is the uniform constant
 * mode's (whose normal is then drawn and not used). */
static int32_t is_words(int32_t d) { return 2 * ((d + 1) / 2) + 1; }

static void is_sample(const oracle_lattice *lat, const int32_t *uniform, const double *scale,
                      const double *E, uint64_t seed, uint64_t id, uint64_t index, uint32_t *x,
                      double *a, double *u, double *half_z2)
{
    const double two_pi = 6.283185307179586476925286766559;
    const double inv32 = 1.0 / 4294967296.0;
    const int32_t d = lat->nx * lat->nt;
    const int32_t W = is_words(d), nb = (W + 3) / 4;
    for (int32_t j = 0; j < nb; ++j) {
        const uint64_t q = index * (uint64_t)nb + (uint64_t)j;
        const uint32_t ctr[4] = { (uint32_t)q, (uint32_t)(q >> 32), (uint32_t)id,
                                  (uint32_t)(id >> 32) };
        const uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
        uint32_t blk[4];
        oracle_philox4x32_10(ctr, key, blk);
        for (int32_t t = 0; t < 4 && 4 * j + t < W; ++t)
            x[4 * j + t] = blk[t];
    }
    double hz = 0.0, z_pair[2] = { 0.0, 0.0 };
    for (int32_t j = 0; j < d; ++j) {
        if (j % 2 == 0) {
            /* Box-Muller: radius from the first word, angle from the second */
            const double u1 = ((double)x[j] + 0.5) * inv32;
            const double u2 = ((double)x[j + 1] + 0.5) * inv32;
            const double r = sqrt(-2.0 * log(u1));
            z_pair[0] = r * cos(two_pi * u2);
            z_pair[1] = r * sin(two_pi * u2);
        }
        if (uniform[j]) {
            /* uniform over [-R, R]: the word's cell centre */
            const double v = ((double)x[2 * ((d + 1) / 2)] + 0.5) * inv32;
            a[j] = scale[j] * (2.0 * v - 1.0);
            continue;
        }
        const double z = z_pair[j % 2];
        a[j] = scale[j] * z;
        hz += 0.5 * z * z;
    }
    for (int32_t k = 0; k < d; ++k) {
        double v = 0.0;
        for (int32_t j = 0; j < d; ++j)
            v += E[(size_t)k * d + j] * a[j];
        u[k] = v;
    }
    *half_z2 = hz;
}

int oracle_is_point(const oracle_lattice *lat, const double *lo, const double *hi, uint64_t seed,
                    uint64_t id, uint64_t index, double *u, double *half_z2)
{
    if (!lattice_ok(lat) || !u || !half_z2)
        return -1;
    const int32_t d = lat->nx * lat->nt;
    double *lambda = (double *)malloc(sizeof(double) * (size_t)d * 3);
    int32_t *uniform = (int32_t *)malloc(sizeof(int32_t) * (size_t)d);
    double *E = (double *)malloc(sizeof(double) * (size_t)d * (size_t)d);
    uint32_t *x = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(d + 12));
    double lk;
    /* lambda: [eigenvalues (d), scales (d), coefficients (d)] */
    int rc = oracle_is_modes(lat, lo, hi, lambda, uniform, lambda + d, &lk);
    if (rc == 0) {
        oracle_is_basis(lat->nx, lat->nt, E);
        is_sample(lat, uniform, lambda + d, E, seed, id, index, x, lambda + 2 * d, u, half_z2);
    }
    free(lambda);
    free(uniform);
    free(E);
    free(x);
    return rc;
}

/* Stream ids with the top bit set draw from the box's uniform density (the
 * same point map as the plain sampler), the others from the Gaussian. */
#define ORACLE_IS_UNIFORM_STREAM (UINT64_C(1) << 63)

static void is_stream_sums(const sums_job *job, size_t s)
{
    const oracle_lattice *lat = job->lat;
    const int32_t nx = lat->nx, d = lat->nx * lat->nt;
    double *lambda = (double *)malloc(sizeof(double) * (size_t)d);
    double *scale = (double *)malloc(sizeof(double) * (size_t)d);
    int32_t *uniform = (int32_t *)malloc(sizeof(int32_t) * (size_t)d);
    double *E = (double *)malloc(sizeof(double) * (size_t)d * (size_t)d);
    uint32_t *x = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(d + 12));
    double *a = (double *)malloc(sizeof(double) * (size_t)d);
    double *u = (double *)malloc(sizeof(double) * (size_t)d);
    double *p = (double *)malloc(sizeof(double) * (size_t)nx);
    double *mscale = (double *)malloc(sizeof(double) * (size_t)d);
    double *mbase = (double *)malloc(sizeof(double) * (size_t)d);
    double lk;
    oracle_is_modes(lat, job->lo, job->hi, lambda, uniform, scale, &lk);
    oracle_is_basis(nx, lat->nt, E);
    box_map(d, job->lo, job->hi, mscale, mbase);
    double log_v = 0.0;
    for (int32_t k = 0; k < d; ++k)
        log_v += log(job->hi[k] - job->lo[k]);
    /* log of the mixture density times K: log(alpha e^{-hz} + (1 - alpha) K / V) */
    const double alpha = job->gaussian_fraction;
    const double log_ga = alpha > 0.0 ? log(alpha) : -INFINITY;
    const double log_un = alpha < 1.0 ? log(1.0 - alpha) + lk - log_v : -INFINITY;
    const int from_uniform = (job->id[s] & ORACLE_IS_UNIFORM_STREAM) != 0;

    const int32_t len = ORACLE_SUMS_LEN(nx);
    neumaier *acc = (neumaier *)calloc((size_t)len, sizeof(neumaier));
    const uint64_t first = job->offset[s], count = job->n[s];
    for (uint64_t i = 0; i < count; ++i) {
        double hz = 0.0;
        if (from_uniform) {
            oracle_words(d, job->seed, job->id[s], first + i, x);
            for (int32_t k = 0; k < d; ++k)
                u[k] = fma((double)x[k], mscale[k], mbase[k]);
            /* the Gaussian exponent of this point: coefficients along the modes */
            for (int32_t j = 0; j < d; ++j) {
                if (uniform[j])
                    continue;
                double aj = 0.0;
                for (int32_t k = 0; k < d; ++k)
                    aj += E[(size_t)k * d + j] * u[k];
                const double z = aj / scale[j];
                hz += 0.5 * z * z;
            }
        } else {
            is_sample(lat, uniform, scale, E, job->seed, job->id[s], first + i, x, a, u, &hz);
        }
        int inside = 1;
        for (int32_t k = 0; k < d; ++k)
            inside &= job->lo[k] <= u[k] && u[k] <= job->hi[k];
        double w = 0.0;
        if (inside) {
            const double g1 = log_ga - hz, g2 = log_un;
            const double mx = fmax(g1, g2);
            const double log_mix = mx + log(exp(g1 - mx) + exp(g2 - mx));
            w = exp(-oracle_action(lat, u) - log_mix);
        }
        oracle_observable(lat, u, p);
        nm_add(&acc[0], 1.0);
        nm_add(&acc[1], w);
        nm_add(&acc[2], w * w);
        for (int32_t r = 0; r < nx; ++r) {
            const double pw = p[r] * w;
            nm_add(&acc[3 + r], pw);
            nm_add(&acc[3 + nx + r], pw * pw);
            nm_add(&acc[3 + 2 * nx + r], pw * w);
        }
    }
    double *out = job->out + s * (size_t)len;
    for (int32_t t = 0; t < len; ++t)
        out[t] = nm_value(&acc[t]);
    free(acc);
    free(lambda);
    free(scale);
    free(uniform);
    free(E);
    free(x);
    free(a);
    free(u);
    free(p);
    free(mscale);
    free(mbase);
}

int oracle_is_sums(const oracle_lattice *lat, uint64_t seed, const double *lo, const double *hi,
                   double gaussian_fraction, size_t nstream, const uint64_t *id, const uint64_t *n,
                   const uint64_t *offset, double *sums, int32_t nthreads)
{
    if (!(gaussian_fraction >= 0.0 && gaussian_fraction <= 1.0))
        return -1;
    return run_sums(lat, seed, nstream, id, lo, hi, n, offset, sums, nthreads, 2,
                    gaussian_fraction, 0, 0);
}

/* ------------------------------------------------- spherical coordinates */

/*
 * Sampling in spherical coordinates (the paper's discussion proposes switching
 * from cartesian to spherical coordinates to concentrate resolution where the
 * subdivision needs it, on a shell about the origin).  The integration domain
 * is still the cube [-B, B]^d; it is cut into radial shells rho_lo <= |u| <
 * rho_hi about the origin (the outermost reaching the cube's corners,
 * B sqrt(d)), and each shell is sampled uniformly in its own volume:
 *   direction: omega = z / |z| with z_k independent standard normals, uniform on
 *     the unit sphere (the normal density depends on |z| only);
 *   radius: the volume of a shell element is proportional to rho^(d-1) d rho, so
 *     with v uniform on (0, 1), rho^d = rho_lo^d + v (rho_hi^d - rho_lo^d), i.e.
 *     rho = rho_hi (t + v (1 - t))^(1/d), t = (rho_lo / rho_hi)^d;
 *   u = rho omega.
 * A sample weighs exp(-S(u)) inside the cube and 0 outside; the shell's integral
 * is its volume V = pi^(d/2) / Gamma(d/2 + 1) (rho_hi^d - rho_lo^d) times the
 * mean weight, which is the record's finalize with V as the subvolume volume.
 * Words: sample `index` of shell stream `id` takes W = 2 ceil(d/2) + 1 Philox
 * words (counter (lo32 q, hi32 q, lo32 id, hi32 id), q = index * ceil(W/4) + j,
 * key = seed): coordinate k's normal is the cosine (k even) or sine (k odd) of
 * the Box-Muller pair of words 2 floor(k/2), 2 floor(k/2) + 1 (radius
 * sqrt(-2 ln u1), angle 2 pi u2, u = (x + 1/2) 2^-32), and word 2 ceil(d/2)
 * gives v = (x + 1/2) 2^-32.
 */

double oracle_sph_volume(int32_t d, double rho_lo, double rho_hi)
{
    if (d < 1 || !(rho_lo >= 0.0) || !(rho_hi > rho_lo) || !isfinite(rho_hi))
        return -1.0;
    /* unit-ball volume pi^(d/2) / Gamma(d/2 + 1), by logs; then the shell */
    const double log_pi = 1.14472988584940017414342735135305871; /* ln pi */
    const double log_unit = 0.5 * d * log_pi - lgamma(0.5 * d + 1.0);
    const double t = pow(rho_lo / rho_hi, (double)d);
    return exp(log_unit + d * log(rho_hi)) * (1.0 - t);
}

int oracle_sph_point(int32_t d, uint64_t seed, uint64_t id, double rho_lo, double rho_hi,
                     uint64_t index, double *u)
{
    if (d < 1 || d > 64 || !u || !(rho_lo >= 0.0) || !(rho_hi > rho_lo) || !isfinite(rho_hi))
        return -1;
    const int32_t pairs = (d + 1) / 2, words = 2 * pairs + 1, nb = (words + 3) / 4;
    uint32_t x[68];
    for (int32_t j = 0; j < nb; ++j) {
        const uint64_t q = index * (uint64_t)nb + (uint64_t)j;
        const uint32_t ctr[4] = { (uint32_t)q, (uint32_t)(q >> 32), (uint32_t)id,
                                  (uint32_t)(id >> 32) };
        const uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
        oracle_philox4x32_10(ctr, key, x + 4 * j);
    }
    const double two_pi = 6.283185307179586476925286766559;
    double norm2 = 0.0;
    for (int32_t k = 0; k < d; ++k) {
        const int32_t p = k / 2;
        const double u1 = ((double)x[2 * p] + 0.5) * 0x1p-32;
        const double u2 = ((double)x[2 * p + 1] + 0.5) * 0x1p-32;
        const double r = sqrt(-2.0 * log(u1));
        u[k] = (k % 2 == 0) ? r * cos(two_pi * u2) : r * sin(two_pi * u2);
        norm2 += u[k] * u[k];
    }
    const double v = ((double)x[2 * pairs] + 0.5) * 0x1p-32;
    const double t = pow(rho_lo / rho_hi, (double)d);
    const double rho = rho_hi * pow(t + v * (1.0 - t), 1.0 / d);
    const double f = rho / sqrt(norm2);
    for (int32_t k = 0; k < d; ++k)
        u[k] *= f;
    return 0;
}

int oracle_sph_sums(const oracle_lattice *lat, uint64_t seed, double box, size_t nshell,
                    const uint64_t *id, const double *rho_lo, const double *rho_hi,
                    const uint64_t *n, const uint64_t *offset, double *sums)
{
    if (!lattice_ok(lat) || !(box > 0.0) || !isfinite(box) || (nshell && (!id || !rho_lo ||
        !rho_hi || !n || !offset || !sums)) || lat->antithetic)
        return -1;
    const int32_t nx = lat->nx, d = nx * lat->nt, len = ORACLE_SUMS_LEN(nx);
    if (nx > 64 || d > 64)
        return -1;
    double *u = (double *)malloc(sizeof(double) * (size_t)d);
    double *p = (double *)malloc(sizeof(double) * (size_t)nx);
    int rc = 0;
    for (size_t s = 0; s < nshell && rc == 0; ++s) {
        neumaier acc[3 + 3 * 64];
        memset(acc, 0, sizeof(acc));
        for (uint64_t i = 0; i < n[s] && rc == 0; ++i) {
            rc = oracle_sph_point(d, seed, id[s], rho_lo[s], rho_hi[s], offset[s] + i, u);
            int inside = 1;
            for (int32_t k = 0; k < d; ++k)
                inside = inside && fabs(u[k]) <= box;
            const double w = inside ? exp(-oracle_action(lat, u)) : 0.0;
            oracle_observable(lat, u, p);
            nm_add(&acc[0], 1.0);
            nm_add(&acc[1], w);
            nm_add(&acc[2], w * w);
            for (int32_t r = 0; r < nx; ++r) {
                const double pw = p[r] * w;
                nm_add(&acc[3 + r], pw);
                nm_add(&acc[3 + nx + r], pw * pw);
                nm_add(&acc[3 + 2 * nx + r], pw * w);
            }
        }
        for (int32_t t = 0; t < len; ++t)
            sums[s * (size_t)len + t] = nm_value(&acc[t]);
    }
    free(u);
    free(p);
    return rc;
}
