/*
 * Plain FP64 CPU oracle for the Monte Carlo lattice functional integral of
 * Burgers' equation (Honkonen & Honkonen, arXiv:1803.07560).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, obviously correct
 * statement of what the GPU path computes.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark load it.  It shares no code,
 * header, constant or helper with the HIP library, and the HIP library never
 * links or calls it.
 *
 * Lattice: nt time slices (the paper's L) by nx space sites (the paper's M);
 * variable k = l*nx + m holds v(t_l, x_m), 0-based (paper section 2, Eq. Gen2).
 *
 * Every function that can fail returns 0 on success and a negative value on
 * invalid arguments; nothing aborts.
 */
#ifndef BURGERS_ORACLE_H
#define BURGERS_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Parameters of the discretised action (Eq. Gen2 and the constants after it).
 * g multiplies the nonlinear term (1 in the paper; 0 gives the Gaussian case)
 * and m2 adds (m2/2)*sum(u^2) (0 in the paper; a regulator for closed forms).
 * observable selects the per-sample product p_r behind C(r) (oracle_observable).
 * antithetic = 1 turns each sample index into a pair of points (see
 * ORACLE_SUMS_LEN). */
typedef struct {
    int32_t nx, nt;
    double nu, D, a, tau;
    double g, m2;
    int32_t observable;
    int32_t antithetic;
} oracle_lattice;

/* p_r as the section 4 correlation is written: the product of the velocity at
 * the first site of the first time slice with the one r sites to its right. */
#define ORACLE_OBS_ANCHOR 0
/* The same product averaged over every anchor (t_l, x_m) of the lattice.  Its
 * expectation under exp(-S) is the anchored one, because the action of Eq. Gen2
 * is unchanged by periodic shifts in space and in time. */
#define ORACLE_OBS_AVERAGED 1

/* Number of doubles in one per-subvolume sums record:
 * [n, sum w, sum w^2, sum p_r w (nx), sum (p_r w)^2 (nx), sum p_r w^2 (nx)]
 * with p_r from oracle_observable.
 * Antithetic pairs (lattice antithetic = 1; antithetic variates applied to the
 * plain estimate of section 3): sample index i gives the point u of its words x
 * and the point u' of the complemented words 0xFFFFFFFF - x, which the same map
 * places at lo + hi - u (the reflection through the subvolume's centre).  The
 * record then runs over pairs: n counts pairs, w stands for the pair mean
 * (w(u) + w(u'))/2 and p_r w for (p_r(u) w(u) + p_r(u') w(u'))/2; the products
 * are those of these means.  Each pair is two integrand evaluations. */
#define ORACLE_SUMS_LEN(nx) (3 + 3 * (nx))

/* Number of doubles in the finalize output:
 * [Z, Z_err, log_Z, ess, n_evals, C (nx), C_err (nx)]. */
#define ORACLE_RESULT_LEN(nx) (5 + 2 * (nx))

/* Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11). */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* The d uniform 32-bit words of sample `index` of subvolume `id`:
 * block j uses counter (lo32(q), hi32(q), lo32(id), hi32(id)) with
 * q = index*ceil(d/4) + j, key = (lo32(seed), hi32(seed)). */
void oracle_words(int32_t d, uint64_t seed, uint64_t id, uint64_t index, uint32_t *words);

/* Map words to the point u in the box [lo, hi): u_k = lo_k + (x_k + 1/2) * (hi_k - lo_k) / 2^32,
 * evaluated as fma(x, scale, base) with scale = (hi-lo)*2^-32 and base = lo + scale/2. */
void oracle_point(int32_t d, uint64_t seed, uint64_t id, const double *lo, const double *hi,
                  uint64_t index, double *u);

/* Residual R_{l,m} of the discretised Burgers equation at every site (the
 * bracket squared in Eq. Gen2), periodic in space and time. R has nt*nx entries. */
int oracle_residual(const oracle_lattice *lat, const double *u, double *R);

/* The action S[u] = sum R^2 / (2 D tau) + (m2/2) sum u^2 (exponent of Eq. Gen2). */
double oracle_action(const oracle_lattice *lat, const double *u);

/* The products p_r, r = 0 .. nx-1, of one configuration u (d = nx*nt values):
 * anchored:  p_r = u(t_0, x_0) u(t_0, x_r);
 * averaged:  p_r = (1/(nx nt)) sum over l, m of u(t_l, x_m) u(t_l, x_{m+r}),
 * space index periodic. */
int oracle_observable(const oracle_lattice *lat, const double *u, double *p);

/* S for n points stored row-major (n x d). */
int oracle_action_batch(const oracle_lattice *lat, size_t n, const double *u, double *S);

/* Per-subvolume Monte Carlo sums over samples offset[s] .. offset[s]+n[s]-1 of
 * subvolume s (boxes lo/hi row-major nsub x d).  Sums are Neumaier-compensated
 * and taken in sample order; threads split the subvolume list only. */
int oracle_sums(const oracle_lattice *lat, uint64_t seed, size_t nsub, const uint64_t *id,
                const double *lo, const double *hi, const uint64_t *n, const uint64_t *offset,
                double *sums, int32_t nthreads);

/* oracle_sums with nx more fields per record: sum |p_r w| (pairs: the absolute
 * value of the pair's mean p_r w), the L1 scale against which the signed sums
 * and C(r) are compared.  Record length ORACLE_SUMS_LEN(nx) + nx; the first
 * ORACLE_SUMS_LEN(nx) fields are oracle_sums' own. */
int oracle_sums_l1(const oracle_lattice *lat, uint64_t seed, size_t nsub, const uint64_t *id,
                   const double *lo, const double *hi, const uint64_t *n, const uint64_t *offset,
                   double *sums, int32_t nthreads);

/* Shifted weights: per subvolume sigma = the smallest action S of its samples
 * (a first pass over them), then the sums record of w = exp(sigma - S), which
 * cannot underflow for every sample of a subvolume at once.  Record:
 * [n, sigma, sum w, sum w^2, sum p_r w (nx), sum (p_r w)^2 (nx), sum p_r w^2 (nx)]
 * (ORACLE_SUMS_LEN(nx) + 1 doubles); the true first-order sums are these times
 * exp(-sigma), the second-order ones times exp(-2 sigma). */
int oracle_sums_shifted(const oracle_lattice *lat, uint64_t seed, size_t nsub,
                        const uint64_t *id, const double *lo, const double *hi, const uint64_t *n,
                        const uint64_t *offset, double *sums, int32_t nthreads);

/* oracle_sums_shifted with nx more fields, sum |p_r w| of the shifted weights
 * (true values: times exp(-sigma)); record length ORACLE_SUMS_LEN(nx) + 1 + nx. */
int oracle_sums_shifted_l1(const oracle_lattice *lat, uint64_t seed, size_t nsub,
                           const uint64_t *id, const double *lo, const double *hi,
                           const uint64_t *n, const uint64_t *offset, double *sums,
                           int32_t nthreads);

/* Split statistics for one subvolume list: for every dimension j, the sums of w
 * and w^2 over the samples in the upper half of the box along j (word j has its
 * top bit set).  out is nsub x 2d: [sum_U w (d), sum_U w^2 (d)]. */
int oracle_split_sums(const oracle_lattice *lat, uint64_t seed, size_t nsub, const uint64_t *id,
                      const double *lo, const double *hi, const uint64_t *n,
                      const uint64_t *offset, double *out, int32_t nthreads);

/* Combine per-subvolume sums into Z, C(r) = N(r)/Z and their standard errors. */
int oracle_finalize(int32_t nx, int32_t d, size_t nsub, const double *lo, const double *hi,
                    const double *sums, double *result);

/* oracle_finalize over shifted records (oracle_sums_shifted): log Z is finite
 * whenever some weight is, even where Z itself underflows. */
int oracle_finalize_shifted(int32_t nx, int32_t d, size_t nsub, const double *lo,
                            const double *hi, const double *sums, double *result);

/* Uniform split of a box into 2^k subvolumes by bisecting dims 0..k-1 in turn;
 * heap ids 2^k .. 2^(k+1)-1 in increasing order. */
int oracle_plan_uniform(int32_t d, const double *box_lo, const double *box_hi, int32_t k,
                        uint64_t *id, double *lo, double *hi);

/* Gaussian-proposal importance sampling of exp(-S) over one box.
 *
 * Proposal: the Gaussian of the action's quadratic part S0 = u.P.u/2 (the
 * nonlinear term dropped), P = A^T A/(D tau) + m2 I with A = (T - 1) -
 * (nu tau/a^2) L, diagonal in the real Fourier basis of the lattice; the
 * constant mode is uniform over [-R, R] when lambda_0 R^2 < 4 (R = the largest
 * |u| in the box), every other mode Gaussian with standard deviation
 * min(1/sqrt(lambda), R).
 * Defensive mixture: a fraction alpha (gaussian_fraction) of the samples comes
 * from it and the rest from the uniform density 1/V of the box; every sample
 * has the weight W = 1_box(u) exp(-S(u)) / (alpha q_G(u) + (1 - alpha)/V) with
 * q_G(u) = exp(-sum z^2/2)/K, so W <= V/(1 - alpha) and the mean of W is Z.
 *
 * oracle_is_basis: the d x d orthonormal basis E (row = lattice variable
 *   k = l*nx + m, column = mode j = bt*nx + bx; column j is the product of the
 *   time vector bt and the space vector bx; vector b of period n: 0 constant,
 *   2k-1 cosine and 2k sine of frequency k < n/2, n-1 alternating for even n).
 * oracle_is_modes: per mode the eigenvalue lambda_j of P, whether it is drawn
 *   uniformly (only the constant mode j = 0 can be), its scale (R for the
 *   uniform mode, min(1/sqrt(lambda), R) for Gaussian ones), and
 *   log K = (log 2R if mode 0 is uniform) + sum_gaussian log(sqrt(2 pi) scale).
 * oracle_is_point: sample `index` of stream `id`.  Words come from Philox4x32-10
 *   with counter (lo32(q), hi32(q), lo32(id), hi32(id)), q = index*ceil(W/4) + j,
 *   key = seed, W = 2 ceil(d/2) + 1 words: mode j's normal is the cosine (j
 *   even) or sine (j odd) of the Box-Muller pair of words 2 floor(j/2) and
 *   2 floor(j/2) + 1 (radius sqrt(-2 ln u1), angle 2 pi u2, u = (x + 1/2) 2^-32);
 *   a uniform constant mode takes word 2 ceil(d/2).  *half_z2 = sum over
 *   Gaussian modes of z^2/2.
 * oracle_is_sums: per stream the sums record of W/K (n, sum w, ...) over
 *   samples offset .. offset+n-1, one box lo/hi (d each) for every stream.
 *   Streams whose id has bit 63 set draw from the uniform density with the
 *   plain sampler's words and point map (oracle_point); the others from the
 *   Gaussian (oracle_is_point).  Returns -1 unless 0 <= gaussian_fraction <= 1. */
int oracle_is_basis(int32_t nx, int32_t nt, double *E);
int oracle_is_modes(const oracle_lattice *lat, const double *lo, const double *hi,
                    double *lambda, int32_t *uniform, double *scale, double *log_k);
int oracle_is_point(const oracle_lattice *lat, const double *lo, const double *hi, uint64_t seed,
                    uint64_t id, uint64_t index, double *u, double *half_z2);
int oracle_is_sums(const oracle_lattice *lat, uint64_t seed, const double *lo, const double *hi,
                   double gaussian_fraction, size_t nstream, const uint64_t *id, const uint64_t *n,
                   const uint64_t *offset, double *sums, int32_t nthreads);

/* Sampling in spherical coordinates over the cube [-box, box]^d, cut into
 * radial shells rho_lo <= |u| < rho_hi (the paper's proposed change from
 * cartesian to spherical coordinates).  Each shell is sampled uniformly in its
 * volume: direction z/|z| from d standard normals, radius rho = rho_hi
 * (t + v (1 - t))^(1/d) with t = (rho_lo/rho_hi)^d.  Words of sample `index` of
 * stream `id`: W = 2 ceil(d/2) + 1 Philox words (counter (lo32 q, hi32 q,
 * lo32 id, hi32 id), q = index * ceil(W/4) + j, key = seed); coordinate k's
 * normal is the cosine (k even) or sine (k odd) of the Box-Muller pair of words
 * 2 floor(k/2), 2 floor(k/2) + 1 (u = (x + 1/2) 2^-32, radius sqrt(-2 ln u1),
 * angle 2 pi u2); v comes from word 2 ceil(d/2) the same way.
 * oracle_sph_volume: the shell's volume pi^(d/2)/Gamma(d/2 + 1) (rho_hi^d -
 *   rho_lo^d) (-1 on invalid arguments).
 * oracle_sph_point: the point of one sample (d <= 64).
 * oracle_sph_sums: per shell, the sums record (ORACLE_SUMS_LEN(nx)) of
 *   w = exp(-S(u)) for u inside the cube (|u_k| <= box), 0 outside; finalize
 *   with the shell volumes in place of box volumes. */
double oracle_sph_volume(int32_t d, double rho_lo, double rho_hi);
int oracle_sph_point(int32_t d, uint64_t seed, uint64_t id, double rho_lo, double rho_hi,
                     uint64_t index, double *u);
int oracle_sph_sums(const oracle_lattice *lat, uint64_t seed, double box, size_t nshell,
                    const uint64_t *id, const double *rho_lo, const double *rho_hi,
                    const uint64_t *n, const uint64_t *offset, double *sums);

/* Plain Monte Carlo of the N-sphere integrand f(x) = sqrt(1 - |x|^2) (0 outside
 * the unit ball) over a box: out = [n, sum f, sum f^2, result, abserr]. */
int oracle_nsphere(int32_t dim, uint64_t seed, uint64_t id, const double *lo, const double *hi,
                   uint64_t n, double *out);

#ifdef __cplusplus
}
#endif
#endif
