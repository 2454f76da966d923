/*
 * bfi.h -- C ABI of the MI355X (gfx950) library for Monte Carlo evaluation of
 * the lattice functional integral of Burgers' equation (Honkonen & Honkonen,
 * "Modelling turbulence via numerical functional integration using Burgers'
 * equation", arXiv:1803.07560).
 *
 * What is computed (section 2, Eq. Gen2): over a box of d = nx*nt lattice
 * variables v(t_l, x_m), periodic in space and time, the normalisation
 *     Z = integral of exp(-S[u]) du
 * and the equal-time two-point correlation
 *     C(r) = integral of u_{0,0} u_{0,r} exp(-S[u]) du / Z,   r = 0 .. nx-1,
 * normalised as in section 4 (divided by the same integral with the velocity
 * factors set to 1).  S is the discretised action of Eq. Gen2:
 *     R_{l,m} = v_{l+1,m} - v_{l,m}
 *             + tau [ g v_{l,m} (v_{l,m+1} - v_{l,m-1}) / (2a)
 *                     - nu (v_{l,m+1} - 2 v_{l,m} + v_{l,m-1}) / a^2 ],
 *     S = sum_{l,m} R_{l,m}^2 / (2 D tau) + (m2/2) sum u^2,
 * with g = 1 and m2 = 0 in the paper (the two knobs exist for closed-form checks).
 * The box is split into subvolumes, each an extent per dimension (section 3),
 * integrated by plain Monte Carlo; the error bar of a subvolume is V s / sqrt(n)
 * (the serial integrand's "result, absolute error" of section 3).
 *
 * Points.  Sample i of subvolume `id` takes ceil(d/4) Philox4x32-10 blocks
 * (Salmon et al., SC'11), block j with key (lo32(seed), hi32(seed)) and counter
 * (lo32(q), hi32(q), lo32(id), hi32(id)), q = i*ceil(d/4) + j; word k maps to
 *     u_k = fma((double)x_k, scale_k, base_k),
 *     scale_k = (hi_k - lo_k) * 2^-32,  base_k = lo_k + scale_k / 2,
 * so u_k lies strictly inside (lo_k, hi_k).  Variable k = l*nx + m.
 *
 * Conventions for every entry point:
 *   - Host pointers are caller-owned and only read (or written, for outputs)
 *     during the call; nothing is retained unless stated.
 *   - Device pointers (suffix _dev) are caller-owned device memory that must
 *     stay valid until the work enqueued on the given stream has completed.
 *   - A stream argument is a hipStream_t passed as void*; NULL selects the
 *     context's own stream.
 *   - Every call returns a bfi_status; on failure bfi_last_error() returns a
 *     thread-local message.  Nothing aborts, nothing throws across the ABI.
 *   - A context is not thread-safe; the server API is.
 */
#ifndef BFI_H
#define BFI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BFI_OK = 0,
    BFI_EINVAL = -1,       /* invalid argument (shape, parameter, box, count) */
    BFI_ENOMEM = -2,       /* device or host allocation failed */
    BFI_EDEVICE = -3,      /* a HIP runtime call failed */
    BFI_EUNSUPPORTED = -4, /* lattice shape or option not compiled in */
    BFI_EBUSY = -5,        /* server full: no slot or memory for the request now */
    BFI_ECANCELLED = -6,   /* request was cancelled */
    BFI_EBUDGET = -7,      /* adaptive run stopped at its evaluation budget */
    BFI_ENOTFOUND = -8     /* unknown ticket */
} bfi_status;

/* Arithmetic of the action and the weight.  Sums are FP64 in both forms. */
typedef enum {
    BFI_FP64 = 0,         /* action, exp(-S) and sums in FP64 */
    BFI_FP32_SHIFTED = 1, /* action and exp in FP32 with a per-thread shift sigma:
                             w = exp(sigma - S), sums in FP64 relative to exp(-sigma) */
    BFI_FP64_SHIFTED = 2  /* action, exp and sums in FP64 with the same per-thread
                             shift (sigma = an action of the thread's samples, moved
                             when a later one is more than 64 below it): no weight
                             underflows relative to the largest one, so Z and C(r)
                             stay defined where every plain exp(-S) is 0 (S > ~745);
                             bfi_result.log_Z carries Z then.  Not supported by the
                             Gaussian-proposal sampler (EUNSUPPORTED). */
} bfi_precision;

/* The per-sample product p_r behind N(r) and C(r) = N(r)/Z (section 4's
 * equal-time correlation). */
typedef enum {
    BFI_OBS_ANCHOR = 0,   /* p_r = u_{0,0} u_{0,r}: first time slice, sites 0 and r */
    BFI_OBS_AVERAGED = 1  /* p_r = (1/(nx nt)) sum_{l,m} u_{l,m} u_{l,m+r} (space index
                             periodic): the anchored product averaged over every
                             anchor.  The action of Eq. Gen2 is invariant under
                             periodic shifts in space and time, so N(r) and C(r) keep
                             their expectation while their variance drops; p_r is
                             exactly symmetric in r <-> nx - r.  Costs nx (nx/2 + 1)
                             multiply-adds per time slice per sample. */
} bfi_observable;

/* Lattice and parameters of Eq. Gen2.  nx = space sites (the paper's M),
 * nt = time slices (L); the paper's run is nx = 10, nt = 2, a = tau = nu = D = 1. */
typedef struct {
    int32_t nx, nt;
    double nu, D, a, tau;
    double g;            /* nonlinear coupling, 1 for Burgers */
    double m2;           /* mass term, 0 for Burgers */
    int32_t observable;  /* bfi_observable; 0 (anchored) is the paper's product */
    int32_t antithetic;  /* 0: one point per sample index (the paper's plain Monte
                            Carlo, section 3).  1: antithetic pairs: sample index i
                            gives the point of its Philox words x and the point of
                            the complemented words 0xFFFFFFFF - x, which the same map
                            puts at lo + hi - u (the reflection through the
                            subvolume's centre); records then run over pairs (n
                            counts pairs, w and p_r w are the pair means) and each
                            pair is two integrand evaluations.  The two points share
                            one Philox evaluation; their weights are nearly
                            uncorrelated on subvolumes that are not centred at 0 (on
                            a box centred at 0, u' = -u only flips the sign of the
                            nonlinear term).  Supported by bfi_eval (without split
                            statistics), plans, bfi_integrate, bfi_finalize and the
                            server, for d <= 32; the other entry points return
                            EUNSUPPORTED. */
} bfi_lattice;

/* A list of subvolumes (host arrays, caller-owned).
 *   id[i]      heap id (root box 1, children 2k and 2k+1); keys the Philox stream
 *   lo, hi     count x d row-major extents, lo < hi, finite
 *   n[i]       samples, >= 2
 *   offset[i]  index of the first sample (a subvolume continues its own stream
 *              when evaluated again at offset = samples already taken) */
typedef struct {
    size_t count;
    const uint64_t *id;
    const double *lo;
    const double *hi;
    const uint64_t *n;
    const uint64_t *offset;
} bfi_subvolumes;

/* Launch shape.  A NULL bfi_launch* takes the tuned (else default) shape for
 * the lattice and precision; in a given struct, samples_per_thread = 0,
 * block = 0 and persistent = -1 each take the tuned value.  Work items hold
 * samples_per_thread * block consecutive samples of one subvolume. */
typedef struct {
    int32_t samples_per_thread; /* K: samples each thread takes per work item */
    int32_t block;              /* threads per block: 64, 128, 256, 512 or 1024
                                   (split statistics: 256; the Gaussian-proposal
                                   and N-sphere samplers: 64, 128 or 256) */
    int32_t persistent;         /* 1: persistent kernel draining a device queue;
                                   0: one block per work item; -1: tuned */
    int32_t use_graph;          /* 1: replay a captured hipGraph (plans only) */
} bfi_launch;

/* Number of doubles in one partial record:
 *   [n, sigma, S_w, S_w2, S_pw[nx], S_pw2[nx], S_pww[nx]]
 * with sums over the samples of w = exp(-S) scaled by exp(sigma) (first-order
 * sums: S_w, S_pw) or exp(2 sigma) (second-order: S_w2, S_pw2 = sum (p_r w)^2,
 * S_pww = sum p_r w^2), p_r as selected by the lattice's observable.  sigma is 0
 * in BFI_FP64. */
#define BFI_PARTIAL_LEN(nx) (4 + 3 * (nx))
/* Split statistics per subvolume: [sigma, S_U w (d), S_U w^2 (d)], sums over the
 * samples in the upper half of the subvolume along each dimension (Philox word
 * with its top bit set), scaled like the partial record of the same sigma. */
#define BFI_SPLIT_LEN(d) (1 + 2 * (d))

#define BFI_MAX_NX 64
#define BFI_MAX_D 64

typedef struct {
    double Z, Z_err;        /* Z and its standard error (may over/underflow; see log_Z) */
    double log_Z;           /* natural log of Z, finite whenever some weight is nonzero */
    double ess;             /* effective sample size (sum W)^2 / sum W^2 */
    double n_evals;         /* integrand evaluations in the estimate */
    int32_t nx;             /* number of valid entries of C and C_err */
    double C[BFI_MAX_NX];     /* C(r) = N(r)/Z */
    double C_err[BFI_MAX_NX]; /* delta-method standard error of C(r) */
} bfi_result;

typedef struct bfi_context bfi_context;
typedef struct bfi_plan bfi_plan;
typedef struct bfi_server bfi_server;

const char *bfi_status_string(bfi_status s);
/* Message of the last failure on this thread (empty if none). */
const char *bfi_last_error(void);
/* BFI_OK if (nx, nt) has compiled kernels, BFI_EUNSUPPORTED otherwise. */
bfi_status bfi_shape_supported(int32_t nx, int32_t nt);
/* Writes up to `cap` supported shapes as (nx, nt) pairs; *count = number supported. */
bfi_status bfi_supported_shapes(int32_t *pairs, int32_t cap, int32_t *count);

/* Context on one HIP device: owns a stream, staging buffers and the tuned
 * launch table.  Errors: EINVAL (bad device), EDEVICE. */
bfi_status bfi_context_create(int32_t device, bfi_context **out);
bfi_status bfi_context_destroy(bfi_context *ctx);

/* Evaluate per-subvolume partial records (paper section 3: the integral over
 * each subvolume separately).  partials: host, count x BFI_PARTIAL_LEN(nx);
 * split: host, count x BFI_SPLIT_LEN(d), or NULL to skip split statistics
 * (supported for d <= 32).  Blocking.  Errors: EINVAL, EUNSUPPORTED, ENOMEM,
 * EDEVICE. */
bfi_status bfi_eval(bfi_context *ctx, const bfi_lattice *lat, bfi_precision prec,
                    uint64_t seed, const bfi_subvolumes *subs, const bfi_launch *launch,
                    double *partials, double *split);

/* bfi_eval for callers that cannot allocate: code under stream capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Same arguments, validation,
 * launch resolution, kernels and results as bfi_eval (with the same launch
 * shape the records are bitwise equal); blocking on the context's stream.  It
 * calls no hipMalloc, hipFree or other allocating routine: the copied
 * subvolume list, point maps, work items, item and subvolume records and the
 * queue head live in one static device array of BFI_NOALLOC_SCRATCH_BYTES per
 * device, held from library load until the process ends (its device address is
 * taken when a context is created on the device).  Layout, 256-byte aligned
 * regions: ids, n, offsets (8 B each per subvolume), lo, hi and the FP64 map
 * (8 B each per subvolume and dimension), the FP32 map (4 B each), the
 * parameter block, (count + 1) first-item indices, work items (32 B), item
 * records (BFI_PARTIAL_LEN(nx) doubles each, plus 2d with split statistics),
 * subvolume records (plus BFI_SPLIT_LEN(d) with split statistics), the queue
 * head.  Items hold samples_per_thread * block samples of one subvolume.
 * Every call on a device shares that device's array: calls that overlap in
 * time on one device (from two threads or two contexts) race.  Errors: those
 * of bfi_eval, and EINVAL (with the bytes needed) when the layout exceeds the
 * array; EDEVICE if the array's address could not be taken. */
#define BFI_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
bfi_status bfi_eval_noalloc(bfi_context *ctx, const bfi_lattice *lat, bfi_precision prec,
                            uint64_t seed, const bfi_subvolumes *subs, const bfi_launch *launch,
                            double *partials, double *split);

/* Plans: the subvolume list uploaded once, work items and buffers resident in
 * device memory, optionally a captured graph; run many times. */
bfi_status bfi_plan_create(bfi_context *ctx, const bfi_lattice *lat, bfi_precision prec,
                           const bfi_subvolumes *subs, const bfi_launch *launch,
                           bfi_plan **out);
/* Enqueue one evaluation of the whole plan on `stream` (NULL: the context's
 * stream).  partials_dev: device, count x BFI_PARTIAL_LEN(nx), written when the
 * stream reaches it; NULL keeps them in the plan's own buffer.  With use_graph,
 * the sequence is captured once per (stream, partials_dev) pair and replayed
 * (the four pairs used last are kept), so a caller may alternate output buffers
 * to overlap reading one run's records with the next run.  Runs of one plan
 * share its work buffers: they must not overlap in time (one stream, or events
 * ordering the streams). */
bfi_status bfi_plan_run(bfi_plan *plan, uint64_t seed, double *partials_dev, void *stream);
/* Wait for the plan's last run and copy its partial records to host. */
bfi_status bfi_plan_partials(bfi_plan *plan, double *partials);
/* Work items of the plan and the launch shape it resolved to. */
bfi_status bfi_plan_info(const bfi_plan *plan, uint64_t *n_items, uint64_t *n_evals,
                         bfi_launch *resolved);
/* Duration in milliseconds of the plan's last run on the device, from HIP
 * events on the run's stream (waits for it): the Monte Carlo kernel alone for
 * direct launches, the whole replay (queue reset, kernel, merge) for graphs. */
bfi_status bfi_plan_kernel_ms(bfi_plan *plan, double *ms);
bfi_status bfi_plan_destroy(bfi_plan *plan);

/* Merge partial records of disjoint sample ranges of the same subvolumes
 * (section 3: a subvolume's estimate from more samples), record by record:
 * acc[i] <- acc[i] (+) more[i], both count x BFI_PARTIAL_LEN(nx), host,
 * caller-owned.  Counts add; the result takes the smaller shift sigma, with
 * first-order sums rescaled by exp(sigma - sigma_old) and second-order sums by
 * its square.  A record with n = 0 is empty (its other fields are ignored).
 * With counter-based points, the records of [offset, offset + n) and
 * [offset + n, offset + n + m) merge into an estimate over n + m samples: this
 * is how a run is checkpointed (subvolumes, sample counts, records) and resumed.
 * Host only.  Errors: EINVAL (nx out of range, NULL arrays, a count that is not
 * a whole number in [0, 2^53], a non-finite shift in a non-empty record, a
 * merged count above 2^53); acc is left unchanged on error. */
bfi_status bfi_partials_merge(int32_t nx, size_t count, double *acc, const double *more);

/* Combine partial records into Z, C(r) and their errors (section 4's
 * normalisation; delta method for the ratio).  Host only.  The subvolume list
 * supplies the volumes; n_evals counts two evaluations per record sample when
 * lat->antithetic is set.  Errors: EINVAL (n < 2, bad box). */
bfi_status bfi_finalize(const bfi_lattice *lat, const bfi_subvolumes *subs,
                        const double *partials, bfi_result *out);

/* Convenience: split [box_lo, box_hi] into 2^split_log2 subvolumes by bisecting
 * dims 0, 1, ... in turn (dim t mod d at level t; heap ids 2^k .. 2^(k+1)-1),
 * give subvolume i (id order) floor(budget/2^k) + (i < budget mod 2^k) samples
 * from offset 0, evaluate and finalize.  box_lo/box_hi: host, d doubles.  The
 * budget counts integrand evaluations: with antithetic pairs, budget/2 (rounded
 * down) sample indices are split that way. */
bfi_status bfi_integrate(bfi_context *ctx, const bfi_lattice *lat, bfi_precision prec,
                         uint64_t seed, const double *box_lo, const double *box_hi,
                         int32_t split_log2, uint64_t budget, const bfi_launch *launch,
                         bfi_result *out);

/* Error-driven adaptive refinement (section 3: subvolumes are subdivided until a
 * convergence criterion holds).  Starts from the uniform 2^split_log2 partition
 * with n_min samples each; every round ranks leaves by their contribution to the
 * variance of C, and either splits a leaf at the midpoint of the dimension
 * minimising sigma_lower + sigma_upper (children start fresh streams) or doubles
 * its samples (continuing its stream), until max_r sigma_C(r)/|C(0)| <= target
 * with an effective sample size (sum W)^2 / sum W^2 of at least min_ess, or
 * max_evals is spent; a round's planned samples are scaled up to round_evals.
 * Leaves keep n_min <= n <= n_max.  The effective-size floor guards the stop:
 * when a few points carry all the weight the delta-method error of C(r) is
 * itself unreliable (one point alone gives sigma_C = 0).  out gets the estimate;
 * the final partition is written to the caller's arrays when non-NULL
 * (capacity `cap` leaves; *n_leaves gets the count).  Returns BFI_EBUDGET (with a
 * valid estimate) if the budget ran out first. */
/* Progress of an adaptive run, reported once per round after the leaves are
 * analysed and after every holdout pass (see bfi_adaptive_config.progress). */
typedef struct {
    int32_t round;           /* rounds completed */
    int32_t holdout_checks;  /* holdout passes run so far */
    uint64_t leaves;
    uint64_t evals;          /* evaluations spent so far, holdout passes included */
    double rel_err;          /* running max_r sigma_C(r)/|C(0)| */
    double holdout_rel_err;  /* of the last holdout pass (0: none yet) */
} bfi_adaptive_progress;
typedef void (*bfi_adaptive_progress_fn)(const bfi_adaptive_progress *p, void *user);

typedef struct {
    double target_rel_err;  /* on max_r sigma_C(r) / |C(0)| */
    uint64_t max_evals;
    uint64_t n_min, n_max;  /* per-leaf sample bounds, n_min >= 2 */
    int32_t split_log2;     /* initial uniform partition */
    int32_t max_rounds;
    double refine_fraction; /* share of the total variance refined per round, (0, 1] */
    uint64_t round_evals;   /* work floor per round: when the refined leaves' planned
                               samples fall short of it, their counts are scaled up by a
                               power of two (within n_max); 0: no floor */
    double min_ess;         /* effective sample size the stop requires; 0: 100 */
    uint64_t split_samples; /* the split statistics (and the leaf spread they are
                               compared with) cover the first split_samples samples of
                               each leaf's stream, which run through the kernel variant
                               that accumulates them; later samples run through the
                               plain kernel.  0: all samples; else >= 2 */
    int32_t holdout;        /* 0: stop when the running estimate meets the target.
                               1: confirm it on a holdout pass first -- every leaf's n
                               samples drawn afresh under seed + k * 0x9E3779B97F4A7C15
                               (k = 1, 2, ... per check), which no refinement decision
                               has seen.  The run stops when the holdout estimate meets
                               the target (out then holds that estimate); otherwise the
                               running target is tightened by min(1/2, target / holdout
                               error) and refinement goes on: at most one check per
                               round, so a failed check is never redrawn on the same
                               leaves.  Holdout evaluations count against max_evals. */
    bfi_adaptive_progress_fn progress; /* called on the caller's thread during the run
                                   (NULL: none); must not call back into the library */
    void *progress_user;        /* passed to progress unchanged */
} bfi_adaptive_config;

typedef struct {
    int32_t rounds;
    uint64_t leaves;
    uint64_t evals;
    double rel_err;         /* achieved max_r sigma_C(r)/|C(0)| */
    int32_t holdout_checks; /* holdout passes run (holdout = 1) */
    int32_t holdout_used;   /* 1: out holds the last holdout pass's estimate, whose
                               samples are the partition's leaves (offset 0, n) under
                               holdout_seed */
    uint64_t holdout_seed;
    double holdout_rel_err; /* max_r sigma_C(r)/|C(0)| of the last holdout pass (0: none) */
    double device_seconds;  /* time the device spent on the run's evaluations (events
                               around each replay of the captured round sequence) */
    int32_t graph_instantiations; /* executable graphs built: one per kernel variant
                                     unless an in-place update was refused */
    int32_t graph_updates;  /* replays after an in-place update of the captured
                               sequence (one per evaluated list after the first) */
} bfi_adaptive_stats;

bfi_status bfi_integrate_adaptive(bfi_context *ctx, const bfi_lattice *lat, bfi_precision prec,
                                  uint64_t seed, const double *box_lo, const double *box_hi,
                                  const bfi_adaptive_config *cfg, const bfi_launch *launch,
                                  bfi_result *out, bfi_adaptive_stats *stats,
                                  uint64_t *leaf_id, double *leaf_lo, double *leaf_hi,
                                  uint64_t *leaf_n, uint64_t *leaf_offset, size_t cap,
                                  size_t *n_leaves);

/* One refinement decision of the adaptive policy, exposed for host-side tests.
 * For each leaf: partial record (BFI_PARTIAL_LEN(nx)) of its current samples,
 * which ranks it, and split statistics (BFI_SPLIT_LEN(d)) with split_base, the
 * partial record of the samples they cover (its shift, count, sum of w and of
 * w^2 give the spread the split is judged against).  split_base NULL: the
 * statistics cover the same samples as `partials`.  action[i] is set to -1
 * (keep), 0 (double the samples) or 1 + j (split along dimension j). */
bfi_status bfi_adaptive_decide(const bfi_lattice *lat, const bfi_subvolumes *leaves,
                               const double *partials, const double *split,
                               const double *split_base, const bfi_adaptive_config *cfg,
                               int32_t *action);

/* Single integrands on the paper's integrand protocol (section 3): for each
 * subvolume, the integral over it (result), its absolute error V s / sqrt(n),
 * and a suggested split dimension (the dimension minimising sigma_lower +
 * sigma_upper of the integrand over the two halves).
 *   BFI_INTEGRAND_NSPHERE: f(x) = sqrt(1 - |x|^2) (0 outside the unit ball) over
 *     `dim` <= 16 dimensions, FP64: half the volume of the unit (dim+1)-ball over
 *     [-1,1]^dim (section 3, Listings 1 and 2).
 *   BFI_INTEGRAND_BURGERS_Z: exp(-S) of Eq. Gen2 (the normalisation), d <= 32.
 *   BFI_INTEGRAND_BURGERS_N: u_{0,0} u_{0,r} exp(-S), r = `distance` (the
 *     un-normalised correlation; section 4 divides it by the BURGERS_Z integral);
 *     its split suggestion uses the statistics of exp(-S).
 * Points are those of bfi_eval (Philox keyed by seed, id, index). */
typedef enum {
    BFI_INTEGRAND_NSPHERE = 0,
    BFI_INTEGRAND_BURGERS_Z = 1,
    BFI_INTEGRAND_BURGERS_N = 2
} bfi_integrand_kind;

typedef struct {
    int32_t kind;       /* bfi_integrand_kind */
    int32_t dim;        /* N-sphere: dimensions; ignored for the lattice kinds */
    bfi_lattice lat;    /* lattice kinds */
    int32_t prec;       /* lattice kinds: bfi_precision */
    int32_t distance;   /* BURGERS_N: r in [0, nx) */
} bfi_integrand;

/* One evaluation per listed subvolume; result, abserr (double) and split_dim
 * (int32, 0-based) are host arrays of subs->count.  Blocking. */
bfi_status bfi_integrand_eval(bfi_context *ctx, const bfi_integrand *f, uint64_t seed,
                              const bfi_subvolumes *subs, const bfi_launch *launch,
                              double *result, double *abserr, int32_t *split_dim);

/* The paper's subdivision (section 3, with the ranges of section 4): every open
 * subvolume is evaluated twice, with n_initial samples and then with
 * sample_factor times more (continuing its stream); it is accepted (result and
 * error of the second evaluation) when one of the criteria holds --
 *   1. |r2 - r1| <= (rel_diff - 1) max(|r1|, |r2|)      (rel_diff e.g. 1.025 .. 1.085)
 *   2. |r2 - r1| <= abs_diff                             (e.g. 0.5 .. 2)
 *   3. max(|r1|, |r2|) <= max_abs                        (e.g. 0.5 .. 2)
 * (a non-positive threshold disables its criterion) -- else it is split in two
 * along the suggested dimension and both halves start fresh streams.  A
 * subvolume at max_depth below the initial partition, or whose children would
 * exceed max_evals, is accepted unconverged.  All open subvolumes of a
 * generation are evaluated in one batch.  *result = sum of accepted results,
 * *abserr = root sum of squares of their errors.  Returns BFI_EBUDGET (with a
 * valid result) when the budget forced unconverged acceptances. */
typedef struct {
    uint64_t n_initial;
    double sample_factor;
    double rel_diff;
    double abs_diff;
    double max_abs;
    int32_t split_log2;
    int32_t max_depth;
    uint64_t max_evals;
} bfi_hdi_config;

typedef struct {
    uint64_t evals;
    uint64_t accepted;
    uint64_t unconverged;
    int32_t generations;
    int32_t depth;        /* deepest accepted level below the initial partition */
} bfi_hdi_stats;

bfi_status bfi_integrate_hdi(bfi_context *ctx, const bfi_integrand *f, uint64_t seed,
                             const double *box_lo, const double *box_hi,
                             const bfi_hdi_config *cfg, const bfi_launch *launch, double *result,
                             double *abserr, bfi_hdi_stats *stats);

/* Gaussian-proposal importance sampling over a cube [box_lo, box_hi]^d, an
 * extension beyond the paper's plain sampler (d <= 32).
 *
 * Dropping the nonlinear term of Eq. Gen2 leaves S0 = u.P.u/2 with
 * P = A^T A/(D tau) + m2 I, A = (T - 1) - (nu tau/a^2) L (T the periodic time
 * shift, L the periodic second difference in space), diagonal in the real
 * Fourier basis of the lattice: mode j = bt*nx + bx is the product of time
 * vector bt and space vector bx (vector b of period n: 0 constant, 2k-1 cosine
 * and 2k sine of frequency k < n/2, n-1 alternating for even n, normalised),
 * with eigenvalue lambda_j = (-mt - c mt mx + c^2 mx^2)/(D tau) + m2,
 * c = nu tau/a^2, mt = 2 cos(2 pi kt/nt) - 2, mx = 2 cos(2 pi kx/nx) - 2.
 * Proposal: a_j = scale_j z_j, z_j standard normal by Box-Muller,
 * scale_j = min(1/sqrt(lambda_j), R), R = sqrt(d) max(|box_lo|, |box_hi|);
 * the constant mode is instead uniform over [-R, R] when lambda_0 R^2 < 4.
 * A fraction alpha (gaussian_fraction) of the samples comes from it and the
 * rest from the cube's uniform density 1/V (a defensive mixture: the Gaussian
 * alone has heavy-tailed weights where the nonlinear term cancels the linear
 * residual); every sample of either component weighs
 *     W = K exp(-S) / (alpha exp(-sum_gaussian z^2/2) + (1 - alpha) K/V) <= V/(1 - alpha),
 *     K = (2R if mode 0 is uniform) * prod_gaussian sqrt(2 pi) scale_j,
 * and Z is the mean of W over all samples, C(r) the W-weighted mean of p_r.
 *
 * Streams: stream id s keys Philox as a subvolume id does.  Ids with bit 63
 * set draw from the uniform component with the plain sampler's words and point
 * map over the cube; the others from the Gaussian: sample i takes
 * ceil((2 ceil(d/2) + 1)/4) Philox blocks, q = i*blocks + j; mode j's normal is
 * the cosine (j even) or sine (j odd) of the Box-Muller pair of words
 * 2 floor(j/2), 2 floor(j/2) + 1 (radius sqrt(-2 ln u1), angle 2 pi u2,
 * u = (x + 1/2) 2^-32); a uniform constant mode takes word 2 ceil(d/2).
 * BFI_FP32_SHIFTED computes the normals with the hardware log2, square root and
 * sine/cosine, the transforms, action and weight in FP32; sums are FP64.
 *
 * bfi_is_modes: the mode table (d entries each; uniform[j] = 1 for a uniform
 *   constant mode) and log K.  Host only.
 * bfi_is_eval: partial records (count x BFI_PARTIAL_LEN(nx), same layout as
 *   bfi_eval's) of W/K over samples offset .. offset + n - 1 (n >= 2) of each
 *   stream, for the given alpha (which enters every weight).
 * bfi_integrate_is: round(alpha budget) samples over Gaussian streams
 *   1 .. streams and the rest over uniform streams 2^63 + 1 .. 2^63 + streams,
 *   each share split floor(b/S) + (i < b mod S) (every stream needs 2 samples);
 *   result as bfi_finalize's, Z = K sum(W/K)/budget, with the two components as
 *   strata of the variance.  BFI_EINVAL for a non-finite or empty cube, alpha
 *   outside [0, 1], or too small a budget; BFI_EUNSUPPORTED for d > 32.
 * bfi_debug_is_points: the points (n x d, FP64) and sum z^2/2 of one stream at
 *   the given indices (test hook). */
bfi_status bfi_is_modes(const bfi_lattice *lat, double box_lo, double box_hi, double *lambda,
                        int32_t *uniform, double *scale, double *log_k);
bfi_status bfi_is_eval(bfi_context *ctx, const bfi_lattice *lat, bfi_precision prec, uint64_t seed,
                       double box_lo, double box_hi, double gaussian_fraction, size_t count,
                       const uint64_t *stream_id, const uint64_t *n, const uint64_t *offset,
                       const bfi_launch *launch, double *partials);
bfi_status bfi_integrate_is(bfi_context *ctx, const bfi_lattice *lat, bfi_precision prec,
                            uint64_t seed, double box_lo, double box_hi, double gaussian_fraction,
                            uint32_t streams, uint64_t budget, const bfi_launch *launch,
                            bfi_result *out);
bfi_status bfi_debug_is_points(bfi_context *ctx, const bfi_lattice *lat, bfi_precision prec,
                               uint64_t seed, double box_lo, double box_hi, uint64_t stream_id,
                               const uint64_t *index, uint64_t n, double *u_out,
                               double *half_z2_out);

/* Monte Carlo in spherical coordinates (the paper's discussion proposes
 * switching from cartesian to spherical coordinates to concentrate resolution
 * on the shell about the origin where the subdivision gathers).  The
 * integration domain stays the cube [-box, box]^d; it is cut into radial
 * shells rho_lo <= |u| < rho_hi about the origin, and each shell is sampled
 * uniformly in its volume: direction z/|z| from d standard normals, radius
 * rho = rho_hi (t + v (1 - t))^(1/d) with t = (rho_lo/rho_hi)^d and v uniform.
 * A sample weighs exp(-S) inside the cube and 0 outside; a shell's integral is
 * its volume pi^(d/2) / Gamma(d/2 + 1) (rho_hi^d - rho_lo^d) times the mean
 * weight.  Words of sample i of stream `id`: W = 2 ceil(d/2) + 1 Philox words,
 * block j with counter (lo32 q, hi32 q, lo32 id, hi32 id), q = i * ceil(W/4) + j,
 * key = seed; coordinate k's normal is the cosine (k even) or sine (k odd) of
 * the Box-Muller pair of words 2 floor(k/2), 2 floor(k/2) + 1 (u = (x + 1/2)
 * 2^-32, radius sqrt(-2 ln u1), angle 2 pi u2); word 2 ceil(d/2) gives v.
 * d <= 32, single points, BFI_FP64 or BFI_FP32_SHIFTED (BFI_FP64_SHIFTED:
 * EUNSUPPORTED); both observables.
 *
 * A list of shells (host arrays, caller-owned): stream id, radii (0 <= rho_lo <
 * rho_hi, finite), sample count (>= 2) and first sample index per shell. */
typedef struct {
    size_t count;
    const uint64_t *id;
    const double *rho_lo;
    const double *rho_hi;
    const uint64_t *n;
    const uint64_t *offset;
} bfi_shells;

/* Per-shell partial records (count x BFI_PARTIAL_LEN(nx), host) of the weight
 * exp(-S) 1_cube over each shell's samples.  Blocking.  launch: NULL or a
 * shape (default 256 samples per thread, 256-thread persistent blocks).
 * Errors: EINVAL, EUNSUPPORTED, ENOMEM, EDEVICE. */
bfi_status bfi_sph_eval(bfi_context *ctx, const bfi_lattice *lat, bfi_precision prec,
                        uint64_t seed, double box, const bfi_shells *shells,
                        const bfi_launch *launch, double *partials);
/* Z, C(r) and their errors from per-shell records, each shell weighted by its
 * volume.  Host only.  Errors: EINVAL. */
bfi_status bfi_sph_finalize(const bfi_lattice *lat, const bfi_shells *shells,
                            const double *partials, bfi_result *out);
/* Two-stage estimate over `nshells` equal-width shells from the centre to the
 * cube's corners (rho up to box sqrt(d); shell s has stream id s + 1): a pilot
 * pass of floor(pilot_fraction budget / nshells) samples per shell, then the
 * rest of the budget allocated in proportion to shell volume times the pilot's
 * standard deviation of the weight (Neyman's allocation), each shell continuing
 * its stream after its pilot samples; records merged, finalized.  Errors:
 * EINVAL (pilot below 2 samples per shell, bad fraction or count), and those
 * of bfi_sph_eval. */
bfi_status bfi_integrate_sph(bfi_context *ctx, const bfi_lattice *lat, bfi_precision prec,
                             uint64_t seed, double box, int32_t nshells, uint64_t budget,
                             double pilot_fraction, const bfi_launch *launch, bfi_result *out);
/* Test hook: the points (n x d, host) of shell [rho_lo, rho_hi) of stream id
 * at sample indices index[0 .. n-1], as the kernel computes them. */
bfi_status bfi_debug_sph_points(bfi_context *ctx, const bfi_lattice *lat, bfi_precision prec,
                                uint64_t seed, uint64_t id, double rho_lo, double rho_hi,
                                uint64_t n, const uint64_t *index, double *out);

/* Continuous-batching request server on one context.  Requests are admitted
 * while their device state fits `memory_budget` bytes and a slot is free; their
 * partial sums stay resident on the device; every scheduling step packs chunks
 * of all admitted requests into persistent kernels, one per lattice shape. */
typedef struct {
    uint64_t memory_budget;     /* bytes of request state on the device */
    int32_t max_requests;       /* admitted requests at once */
    int32_t chunks_per_step;    /* work items per request per step, at least */
    int32_t max_pending;        /* submitted but not admitted; EBUSY beyond it */
    uint64_t step_evals;        /* target evaluations per step, shared equally by the
                                   active requests (0: 2^25); bounds the wait of a
                                   newly admitted request for the running step */
    int32_t max_samples_per_thread; /* cap on the tuned samples per thread of served
                                   work items (0: 128).  An item is the unit of a
                                   request's progress: small items spread a small
                                   request over many blocks, which keeps its latency
                                   low, where batch runs prefer large ones */
} bfi_server_config;

typedef struct {
    bfi_lattice lat;
    bfi_precision prec;
    uint64_t seed;
    double box;               /* box [-box, box]^d */
    int32_t split_log2;       /* uniform partition */
    uint64_t budget;          /* total integrand evaluations (antithetic pairs: budget/2
                                 sample indices, split as in bfi_integrate) */
} bfi_request;

typedef struct {
    uint64_t submitted, completed, cancelled, rejected;
    uint64_t steps, evals;
    double busy_seconds;      /* time with kernels in flight */
} bfi_server_stats;

bfi_status bfi_server_create(bfi_context *ctx, const bfi_server_config *cfg, bfi_server **out);
/* Non-blocking.  Errors: EINVAL, EUNSUPPORTED, EBUSY (pending queue full). */
bfi_status bfi_server_submit(bfi_server *srv, const bfi_request *req, uint64_t *ticket);
/* *done = 1 when finished; then out holds the result and the ticket is released.
 * latency_s (optional) gets submit-to-completion seconds.  A finished request
 * that failed returns its own status (with *done = 1) and releases the ticket,
 * e.g. ECANCELLED after bfi_server_cancel, EDEVICE when a HIP call failed or its
 * sums came out non-finite (an action beyond the range of the precision).  A
 * failed request affects no other. */
bfi_status bfi_server_poll(bfi_server *srv, uint64_t ticket, bfi_result *out, int32_t *done,
                           double *latency_s);
/* Blocks until done or timeout_s elapses (*done = 0). */
bfi_status bfi_server_wait(bfi_server *srv, uint64_t ticket, double timeout_s, bfi_result *out,
                           int32_t *done, double *latency_s);
bfi_status bfi_server_cancel(bfi_server *srv, uint64_t ticket);
bfi_status bfi_server_stats_get(bfi_server *srv, bfi_server_stats *out);
bfi_status bfi_server_destroy(bfi_server *srv);

/* Autotuner: time candidate launch shapes (samples_per_thread in 16..1024 x
 * block in 64..1024 x persistent) on a synthetic uniform partition of the lattice with about
 * `evals_per_trial` evaluations, keep the fastest for (shape, precision, single
 * points or antithetic pairs, observable -- lat->antithetic, lat->observable) in
 * the context, and return it with its rate.  A plan without an entry of its own
 * takes the anchored-product entry of its sampler, then the single-point one.
 * Blocking. */
bfi_status bfi_autotune(bfi_context *ctx, const bfi_lattice *lat, bfi_precision prec,
                        uint64_t evals_per_trial, bfi_launch *best, double *best_evals_per_s);
/* Save / load the context's tuned table as JSON (keyed by device architecture;
 * entries for another architecture are ignored on load). */
bfi_status bfi_tune_save(const bfi_context *ctx, const char *path);
bfi_status bfi_tune_load(bfi_context *ctx, const char *path);

/* Test hooks for bit-exact parity.
 * bfi_debug_points: the points of samples index[0..n) of one subvolume as the
 * kernels generate them, FP64 (or, for BFI_FP32_SHIFTED, the FP32 point widened
 * to double); out: host n x d.  d <= BFI_MAX_D.
 * bfi_debug_action: S for n points (host, n x d) with the kernels' action
 * (FP32 form: points rounded to float, S widened); out_S: host, n. */
bfi_status bfi_debug_points(bfi_context *ctx, int32_t d, bfi_precision prec, uint64_t seed,
                            uint64_t id, const double *lo, const double *hi,
                            const uint64_t *index, uint64_t n, double *out);
bfi_status bfi_debug_action(bfi_context *ctx, const bfi_lattice *lat, bfi_precision prec,
                            uint64_t n, const double *points, double *out_S);

#ifdef __cplusplus
}
#endif
#endif
