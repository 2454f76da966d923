// Error-driven adaptive refinement of the subvolume partition (paper section 3:
// the volume is subdivided into smaller and smaller subvolumes until the
// result converges; the integrand suggests the dimension to split).
//
// Policy of one round, over the current leaves:
//   1. Finalize all leaves; each leaf's contribution to the variance of C is
//      e_s = sum_r [Var N_s(r) - 2 C(r) Cov_s(r) + C(r)^2 Var Z_s] / Z^2.
//   2. Leaves are ranked by e_s (descending, ties by lower id) and taken until
//      their contributions reach `refine_fraction` of the total (at least one).
//   3. A taken leaf is split at the midpoint of the dimension j* minimising
//      sigma_lower(j) + sigma_upper(j) -- the standard deviations of the weight
//      in the two halves, from the split statistics of m samples (each half holds
//      m/2 in expectation) -- when that sum is below kSplitGain * 2 sigma_leaf
//      (sigma_leaf over the same m samples) or when doubling would exceed n_max;
//      otherwise its samples are doubled by continuing its own Philox stream.
//      Ties in j* go to the lower dimension.  m is the leaf's sample count, or
//      at most `split_samples`: the statistics then come from the first samples
//      of the stream only, and the rest run through the plain kernel.
//   4. Children get fresh streams (ids 2 id and 2 id + 1) with
//      clamp(n_leaf, n_min, n_max) samples each; the parent's samples are dropped.
//   5. If the round's planned samples fall short of `round_evals`, every planned
//      count (children, doubled leaves) is multiplied by the smallest power of
//      two reaching it, within n_max, so each round keeps the chip busy and the
//      extra samples go where the variance is.
// Rounds repeat until max_r sigma_C(r) / |C(0)| <= target, the evaluation budget
// or the round limit is reached.  Every round's work list (uneven sample counts)
// is drained by the persistent kernel through the device queue; the leaves'
// records stay in device memory, where each round's records are folded into
// them and step 1 runs (the host takes the decisions of steps 2-5 from each
// leaf's e_s, j* and gain).
//
// The running estimate is judged on the samples that steered the refinement:
// leaves whose samples happened to miss the rare large weights look quiet and
// are left alone, so its error bar is optimistic when the weights are heavy
// tailed.  With `holdout` the stop is confirmed on the same leaves sampled
// afresh under another seed; a failed check tightens the running target.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <type_traits>
#include <limits>
#include <numeric>
#include <optional>

#include "runtime.h"

using namespace bfi;

namespace {

constexpr double kSplitGain = 0.9;

// Product of the extents, in dimension order (the finalize's own volume).
double box_volume(const double *lo, const double *hi, int d)
{
    double v = 1.0;
    for (int k = 0; k < d; ++k)
        v *= hi[k] - lo[k];
    return v;
}

// Contribution of every leaf to the variance of C (NaN counts 0), and the
// estimate itself, from the finalize's two passes over host records.
bfi_status analyse(int nx, int d, size_t count, const double *lo, const double *hi,
                   const double *partials, std::vector<double> *e_out, bfi_result *res)
{
    e_out->resize(count);
    BFI_TRY(finalize_records(nx, d, count, lo, hi, partials, res, 1, e_out->data()));
    double *ev = e_out->data();
    parallel_range(count, size_t(1) << 16, [ev](size_t s) { ev[s] = ev[s] >= 0.0 ? ev[s] : 0.0; });
    return BFI_OK;
}

// Split statistics of the leaves: `split` (BFI_SPLIT_LEN(d) per leaf) and `base`,
// the record of the samples they cover (the whole leaf, or its first
// split_samples samples).
struct SplitStats {
    int d, rec_len;
    const double *split, *base;
};

struct SplitChoice {
    int best_dim;  // j*
    double gain;   // (sigma_L + sigma_U)(j*) / (2 sigma)
};

// j* and the gain of leaf s, in the shift of the covered samples (the split
// record shares it).  The device analysis of a run's leaves does the same
// arithmetic (leaf_kernels.hip).
SplitChoice split_choice(const SplitStats &st, size_t s)
{
    const int d = st.d;
    const double *sp = st.split + s * BFI_SPLIT_LEN(d), *base = st.base + s * st.rec_len;
    const double S = base[2], Q = base[3], m = base[0], half = 0.5 * m;
    const double sigma = std::sqrt(std::max(Q / m - (S / m) * (S / m), 0.0));
    double best = std::numeric_limits<double>::infinity();
    int best_j = 0;
    for (int j = 0; j < d; ++j) {
        const double su = sp[1 + j], qu = sp[1 + d + j];
        const double sl = S - su, ql = Q - qu;
        const double vu = std::max(qu / half - (su / half) * (su / half), 0.0);
        const double vl = std::max(ql / half - (sl / half) * (sl / half), 0.0);
        const double sj = std::sqrt(vu) + std::sqrt(vl);
        if (sj < best) {
            best = sj;
            best_j = j;
        }
    }
    return SplitChoice{best_j, sigma > 0 ? best / (2.0 * sigma) : 1.0};
}

double rel_err(const bfi_result &r)
{
    double m = 0.0;
    for (int k = 0; k < r.nx; ++k)
        m = std::max(m, r.C_err[k]);
    return r.C[0] != 0.0 ? m / std::fabs(r.C[0]) : std::numeric_limits<double>::infinity();
}

bool can_split(uint64_t id) { return id < (uint64_t(1) << 62); }

// Action of a refined leaf: split along j* when that halves the spread well
// enough or doubling would exceed n_max, else double; -1 if neither is possible.
int32_t action_of(const SplitChoice &c, uint64_t id, uint64_t n, const bfi_adaptive_config &cfg)
{
    const bool doubling_ok = n <= cfg.n_max / 2;
    if (can_split(id) && (c.gain < kSplitGain || !doubling_ok))
        return 1 + c.best_dim;
    return doubling_ok ? 0 : -1;
}

// A growable array of trivially copyable elements on malloc/realloc: past the
// allocator's mmap threshold, growth remaps pages instead of copying them, so a
// leaf set of gigabytes grows without being copied; new elements are not
// initialised.
template <class T>
class GrowArray {
public:
    GrowArray() = default;
    GrowArray(const GrowArray &) = delete;
    GrowArray &operator=(const GrowArray &) = delete;
    ~GrowArray() { std::free(p_); }
    size_t size() const { return n_; }
    size_t capacity() const { return cap_; }
    T *data() { return p_; }
    const T *data() const { return p_; }
    T &operator[](size_t i) { return p_[i]; }
    const T &operator[](size_t i) const { return p_[i]; }
    T *begin() { return p_; }
    T *end() { return p_ + n_; }
    const T *begin() const { return p_; }
    const T *end() const { return p_ + n_; }
    void resize(size_t n)
    {
        if (n > cap_) {
            const size_t c = std::max(n, 2 * cap_);
            void *q = std::realloc(p_, c * sizeof(T));
            if (!q)
                throw std::bad_alloc();
            p_ = static_cast<T *>(q);
            cap_ = c;
        }
        n_ = n;
    }
    template <class It>
    void assign(It b, It e)
    {
        resize(static_cast<size_t>(e - b));
        std::copy(b, e, p_);
    }

private:
    static_assert(std::is_trivially_copyable<T>::value, "plain data only");
    T *p_ = nullptr;
    size_t n_ = 0, cap_ = 0;
};

// Leaves in ranking order (descending contribution e, ties by lower id), built
// lazily: for e >= 0 the IEEE bit pattern orders like the value, so one
// parallel pass counts the leaves per bucket of its top bits; a read at rank i
// gathers whole buckets from the top (at least twice what was gathered before)
// and sorts only those.  Whole buckets keep the order exact: the result is the
// full sort's, but a round that refines the top few percent of millions of
// leaves never sorts the rest.
class Ranking {
public:
    Ranking(const double *e, size_t n, const uint64_t *ids) : e_(e), n_(n), ids_(ids)
    {
        nchunks_ = (n + kChunk - 1) / kChunk;
        part_.assign(nchunks_, {});
        bucket_.resize(n);
        std::vector<double> sums(nchunks_, 0.0);
        for_chunks(nchunks_, [&](size_t c) {
            part_[c].assign(kBuckets, 0);
            const size_t i1 = std::min(n, (c + 1) * kChunk);
            double sum = 0.0;
            for (size_t s = c * kChunk; s < i1; ++s) {
                const uint16_t b = bucket(e[s]);
                bucket_[s] = b;
                ++part_[c][b];
                sum += e[s];
            }
            sums[c] = sum;
        });
        hist_.assign(kBuckets, 0);
        constexpr size_t kHistGrain = 1024;
        for_chunks(kBuckets / kHistGrain, [&](size_t g) {
            for (const auto &h : part_)
                for (size_t b = g * kHistGrain; b < (g + 1) * kHistGrain; ++b)
                    hist_[b] += h[b];
        });
        total_ = 0.0;
        for (double x : sums)
            total_ += x;
        top_ = kBuckets;
    }
    size_t size() const { return n_; }
    // sum of e over every leaf (per-chunk sums in chunk order)
    double total() const { return total_; }
    // the leaf at rank i
    size_t operator[](size_t i)
    {
        if (i >= keys_.size())
            extend(i + 1);
        return keys_[i].leaf;
    }
    // ranks read so far (every rank below it is final)
    size_t sorted() const { return keys_.size(); }
    // make ranks [0, n) readable in one extension (reading them one at a time
    // grows the sorted part in doublings)
    void gather(size_t n)
    {
        n = std::min(n, n_);
        if (n > keys_.size())
            extend(n);
    }

private:
    static constexpr size_t kBuckets = size_t(1) << 15;  // sign bit 0: 15 top bits
    static constexpr size_t kChunk = size_t(1) << 16;
    struct Key {
        double e;
        uint64_t id;
        size_t leaf;
    };
    static uint16_t bucket(double e)
    {
        uint64_t bits;
        std::memcpy(&bits, &e, sizeof bits);
        return static_cast<uint16_t>(bits >> 48);  // e >= 0 and not NaN (analyse)
    }
    static bool before(const Key &x, const Key &y)
    {
        return x.e != y.e ? x.e > y.e : x.id < y.id;
    }
    // Append buckets [lo, top_) in descending bucket order: every key goes
    // straight to its place (bucket offset + the counts of earlier chunks in that
    // bucket), then each bucket is sorted on its own; chunks and buckets run in
    // parallel.
    void extend(size_t want)
    {
        TraceRange tr("adaptive: ranking extension");
        const size_t n = n_;
        const size_t target = std::min(n, std::max({want, 2 * keys_.size(), size_t(4096)}));
        size_t have = keys_.size(), lo = top_;
        while (lo > 0 && have < target)
            have += hist_[--lo];
        const size_t hi = top_, start = keys_.size(), span = hi - lo;
        std::vector<size_t> first(span + 1);  // start of bucket hi-1-k at first[k]
        first[0] = start;
        for (size_t k = 0; k < span; ++k)
            first[k + 1] = first[k] + hist_[hi - 1 - k];
        keys_.resize(first[span]);
        for_chunks(nchunks_, [&](size_t c) {
            std::vector<size_t> at(span);
            for (size_t k = 0; k < span; ++k) {
                size_t o = first[k];
                for (size_t cc = 0; cc < c; ++cc)
                    o += part_[cc][hi - 1 - k];
                at[k] = o;
            }
            const size_t i1 = std::min(n, (c + 1) * kChunk);
            for (size_t s = c * kChunk; s < i1; ++s) {
                const size_t b = bucket_[s];
                if (b >= lo && b < hi)
                    keys_[at[hi - 1 - b]++] = Key{e_[s], ids_[s], s};
            }
        });
        // each bucket sorted on its own, consecutive buckets in runs of about
        // 1/64 of the keys per task (the top buckets are many and sparse)
        const size_t per_run = std::max<size_t>((first[span] - start) / 64, 1024);
        std::vector<size_t> run_first{0};
        for (size_t k = 0, cnt = 0; k < span; ++k) {
            cnt += first[k + 1] - first[k];
            if (cnt >= per_run || k + 1 == span) {
                run_first.push_back(k + 1);
                cnt = 0;
            }
        }
        for_chunks(run_first.size() - 1, [&](size_t r) {
            for (size_t k = run_first[r]; k < run_first[r + 1]; ++k)
                if (first[k + 1] - first[k] > 1)
                    std::sort(keys_.begin() + first[k], keys_.begin() + first[k + 1], before);
        });
        top_ = lo;
    }
    const double *e_;
    size_t n_;
    const uint64_t *ids_;
    size_t nchunks_ = 0;
    std::vector<std::vector<uint32_t>> part_;  // per chunk: leaves per bucket
    std::vector<uint16_t> bucket_;             // per leaf
    std::vector<uint32_t> hist_;
    GrowArray<Key> keys_;  // grown without initialising: the scatter writes every key
    double total_ = 0.0;
    size_t top_;  // buckets at or above it are in keys_
};

// Decide actions: -1 keep, 0 double, 1 + j split along j, for the leaves in
// ranking order until their contributions e reach refine_fraction of the
// total; act(s) gives leaf s's action.  Returns the number of ranks examined;
// the refined leaves are among them.
template <class Act>
size_t decide(const double *e, size_t count, Act &&act, const bfi_adaptive_config &cfg,
              int32_t *action, Ranking &order)
{
    const double total = order.total();
    parallel_range(count, size_t(1) << 18, [&](size_t s) { action[s] = -1; });
    // the ranks taken (in order, until their contributions reach the fraction);
    // reading them gathers them into the ranking, so the per-leaf decisions
    // below only read it and run in parallel
    double taken = 0.0;
    size_t i = 0;
    for (; i < count; ++i) {
        const size_t s = order[i];
        if (i > 0 && taken >= cfg.refine_fraction * total)
            break;
        if (e[s] <= 0.0 && i > 0)
            break;
        taken += e[s];
    }
    parallel_range(i, size_t(1) << 10, [&](size_t k) {
        const size_t s = order[k];
        action[s] = act(s);
    });
    return i;
}

bfi_status check_config(const bfi_adaptive_config *cfg)
{
    if (!cfg)
        return fail(BFI_EINVAL, "config is NULL");
    if (!(cfg->target_rel_err > 0) || !std::isfinite(cfg->target_rel_err))
        return fail(BFI_EINVAL, "target_rel_err must be positive");
    if (cfg->n_min < 2 || cfg->n_max < cfg->n_min)
        return fail(BFI_EINVAL, "need 2 <= n_min <= n_max");
    if (cfg->split_log2 < 0 || cfg->split_log2 > 24)
        return fail(BFI_EINVAL, "split_log2 must be in [0, 24]");
    if (!(cfg->refine_fraction > 0) || cfg->refine_fraction > 1)
        return fail(BFI_EINVAL, "refine_fraction must be in (0, 1]");
    if (cfg->max_rounds < 0)
        return fail(BFI_EINVAL, "max_rounds must be >= 0");
    if (!(cfg->min_ess >= 0) || !std::isfinite(cfg->min_ess))
        return fail(BFI_EINVAL, "min_ess must be finite and >= 0");
    if (cfg->split_samples == 1)
        return fail(BFI_EINVAL, "split_samples must be 0 (all samples) or >= 2");
    if (cfg->holdout != 0 && cfg->holdout != 1)
        return fail(BFI_EINVAL, "holdout must be 0 or 1");
    return BFI_OK;
}

// Merge record b into a (disjoint samples of the same subvolume): both move to
// the smaller shift; counts add, first-order sums scale by the shift factor,
// second-order sums by its square.  first/second list the field ranges.
void merge_shifted(double *a, const double *b, int sigma_at, const std::vector<int> &first,
                   const std::vector<int> &second, int count_at)
{
    const double sig = std::min(a[sigma_at], b[sigma_at]);
    const double fa = std::exp(sig - a[sigma_at]), fb = std::exp(sig - b[sigma_at]);
    for (int i : first)
        a[i] = fa * a[i] + fb * b[i];
    for (int i : second)
        a[i] = fa * fa * a[i] + fb * fb * b[i];
    if (count_at >= 0)
        a[count_at] += b[count_at];
    a[sigma_at] = sig;
}

// Field ranges of a partial record: first-order sums (S_w, S_pw) and
// second-order sums (S_w2, S_pw2, S_pww).
void record_fields(int nx, std::vector<int> *first, std::vector<int> *second)
{
    *first = {2};
    *second = {3};
    for (int r = 0; r < nx; ++r) {
        first->push_back(4 + r);
        second->push_back(4 + nx + r);
        second->push_back(4 + 2 * nx + r);
    }
}

// The host side of the leaf set: ids, sample counts, boxes and volumes.  The
// records stay in device memory (DeviceLeaves).
struct LeafSet {
    int d = 0, nx = 0;
    GrowArray<uint64_t> id, n;
    GrowArray<double> lo, hi;
    GrowArray<double> vol;  // product of the extents, computed once per leaf
    size_t size() const { return id.size(); }
};

// Device buffer grown geometrically, keeping its first `keep` elements (copied
// on the stream, which is then drained before the old buffer goes).
template <class T>
hipError_t grow_keep(T **p, size_t *cap, size_t need, size_t keep, hipStream_t st)
{
    if (need <= *cap && *p)
        return hipSuccess;
    const size_t n = std::max<size_t>({need, 2 * *cap, 1024});
    T *q = nullptr;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(&q), n * sizeof(T));
    if (e != hipSuccess)
        return e;
    if (*p) {
        if (keep > 0)
            e = hipMemcpyAsync(q, *p, keep * sizeof(T), hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess)
            e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            (void)hipFree(q);
            return e;
        }
        (void)hipFree(*p);
    }
    *p = q;
    *cap = n;
    return hipSuccess;
}

// Pinned host buffer grown geometrically (contents not kept).
template <class T>
hipError_t grow_pinned_buf(T **p, size_t *cap, size_t need)
{
    if (need <= *cap && *p)
        return hipSuccess;
    const size_t n = std::max<size_t>({need, 2 * *cap, 1024});
    if (*p)
        (void)hipHostFree(*p);
    *p = nullptr;
    *cap = 0;
    hipError_t e = hipHostMalloc(reinterpret_cast<void **>(p), n * sizeof(T), hipHostMallocDefault);
    if (e == hipSuccess)
        *cap = n;
    return e;
}

// The leaves' records in device memory: per leaf the record of all its
// samples, its split statistics and the record of the samples they cover, and
// its volume.  A round's records are folded in on the device and every leaf is
// analysed there (leaf_kernels.hip); the host reads back each leaf's
// contribution e, split choice and gain, and the estimate's totals.  Buffers
// grow geometrically; nothing is allocated in a round that adds no capacity.
class DeviceLeaves {
public:
    DeviceLeaves(bfi_context *ctx, int nx, int d)
        : ctx_(ctx), nx_(nx), d_(d), rec_len_(BFI_PARTIAL_LEN(nx)), split_len_(BFI_SPLIT_LEN(d))
    {
    }
    DeviceLeaves(const DeviceLeaves &) = delete;
    DeviceLeaves &operator=(const DeviceLeaves &) = delete;
    ~DeviceLeaves()
    {
        (void)hipStreamSynchronize(ctx_->stream);
        for (void *p : {static_cast<void *>(rec_), static_cast<void *>(split_),
                        static_cast<void *>(base_), static_cast<void *>(vol_),
                        static_cast<void *>(e_d_), static_cast<void *>(gain_d_),
                        static_cast<void *>(best_d_), static_cast<void *>(scratch_),
                        static_cast<void *>(totals_d_), static_cast<void *>(fold_d_)})
            if (p)
                (void)hipFree(p);
        for (void *p : {static_cast<void *>(h_e_), static_cast<void *>(h_gain_),
                        static_cast<void *>(h_best_), static_cast<void *>(h_totals_),
                        static_cast<void *>(h_fold_)})
            if (p)
                (void)hipHostFree(p);
        for (hipEvent_t ev : {ev_f0_, ev_f1_, ev_a0_, ev_e_, ev_a1_})
            if (ev)
                (void)hipEventDestroy(ev);
    }
    // room for n leaves; the first `keep` leaves' records are kept
    bfi_status reserve(size_t n, size_t keep)
    {
        if (n > 0xFFFFFFFFull)
            return fail(BFI_EINVAL, "more than 2^32 leaves");
        if (n <= cap_ && rec_)
            return BFI_OK;
        // capacities in elements; every per-leaf buffer grows to the same count
        // of leaves (cap_), so each is reallocated when the leaves outgrow it
        hipStream_t st = ctx_->stream;
        const size_t leaves = std::max<size_t>({n, 2 * cap_, 1024});
        size_t c_rec = cap_ * rec_len_, c_split = cap_ * split_len_, c_base = cap_ * rec_len_,
               c_vol = cap_;
        BFI_HIP(grow_keep(&rec_, &c_rec, leaves * rec_len_, keep * rec_len_, st));
        BFI_HIP(grow_keep(&split_, &c_split, leaves * split_len_, keep * split_len_, st));
        BFI_HIP(grow_keep(&base_, &c_base, leaves * rec_len_, keep * rec_len_, st));
        BFI_HIP(grow_keep(&vol_, &c_vol, leaves, keep, st));
        size_t c_e = cap_, c_g = cap_, c_b = cap_;
        BFI_HIP(grow_keep(&e_d_, &c_e, leaves, 0, st));
        BFI_HIP(grow_keep(&gain_d_, &c_g, leaves, 0, st));
        BFI_HIP(grow_keep(&best_d_, &c_b, leaves, 0, st));
        cap_ = leaves;
        return BFI_OK;
    }
    // pinned room for a round's fold entries
    bfi_status stage_fold(size_t count)
    {
        BFI_HIP(grow_pinned_buf(&h_fold_, &cap_hfold_, count));
        return BFI_OK;
    }
    FoldEntry *fold_entries() { return h_fold_; }
    // fold entries [0, count) into the leaves, queued after the replays on the
    // context's stream (their records: with_rec/with_split and plain_rec)
    bfi_status fold(size_t count, const double *with_rec, const double *with_split,
                    const double *plain_rec)
    {
        if (count == 0)
            return BFI_OK;
        if (count > 0xFFFFFFFFull)
            return fail(BFI_EINVAL, "more than 2^32 entries in one round");
        hipStream_t st = ctx_->stream;
        BFI_TRY(events());
        BFI_HIP(grow_keep(&fold_d_, &cap_dfold_, count, 0, st));
        BFI_HIP(hipEventRecord(ev_f0_, st));
        BFI_HIP(hipMemcpyAsync(fold_d_, h_fold_, count * sizeof(FoldEntry), hipMemcpyHostToDevice,
                               st));
        FoldArgs fa{fold_d_, static_cast<uint32_t>(count), with_rec, with_split, plain_rec,
                    rec_,    split_,    base_,     vol_,      nx_,       d_};
        BFI_HIP(launch_fold(fa, st));
        BFI_HIP(hipEventRecord(ev_f1_, st));
        folded_ = true;
        return BFI_OK;
    }
    // analyse leaves [0, count): the estimate into res, each leaf's e, split
    // choice and gain into host memory (e(), best(), gain()); device_ms gets the
    // device time of the last fold and this analysis
    bfi_status analyse(size_t count, bfi_result *res, double *device_ms)
    {
        if (count == 0 || count > 0xFFFFFFFFull)
            return fail(BFI_EINVAL, "leaf count out of range");
        hipStream_t st = ctx_->stream;
        BFI_TRY(events());
        BFI_HIP(grow_keep(&scratch_, &cap_scratch_,
                          analysis_scratch_doubles(static_cast<uint32_t>(count), nx_), 0, st));
        const size_t ntot = 1 + 4 + 2 * static_cast<size_t>(nx_);
        BFI_HIP(grow_keep(&totals_d_, &cap_totals_, ntot, 0, st));
        BFI_HIP(grow_pinned_buf(&h_totals_, &cap_htotals_, ntot));
        BFI_HIP(grow_pinned_buf(&h_e_, &cap_he_, count));
        BFI_HIP(grow_pinned_buf(&h_gain_, &cap_hg_, count));
        BFI_HIP(grow_pinned_buf(&h_best_, &cap_hb_, count));
        BFI_HIP(hipEventRecord(ev_a0_, st));
        LeafAnalysisArgs la{rec_,   split_,   base_,     vol_,   static_cast<uint32_t>(count),
                            nx_,    d_,       scratch_,  totals_d_, e_d_,
                            gain_d_, best_d_};
        BFI_HIP(launch_leaf_analysis(la, st));
        BFI_HIP(hipMemcpyAsync(h_totals_, totals_d_, ntot * sizeof(double), hipMemcpyDeviceToHost,
                               st));
        BFI_HIP(hipMemcpyAsync(h_e_, e_d_, count * sizeof(double), hipMemcpyDeviceToHost, st));
        BFI_HIP(hipEventRecord(ev_e_, st));
        // the split choices come back while the host ranks the leaves by e
        // (wait_choices before reading them)
        BFI_HIP(hipMemcpyAsync(h_gain_, gain_d_, count * sizeof(double), hipMemcpyDeviceToHost, st));
        BFI_HIP(hipMemcpyAsync(h_best_, best_d_, count * sizeof(int32_t), hipMemcpyDeviceToHost,
                               st));
        BFI_HIP(hipEventRecord(ev_a1_, st));
        choices_pending_ = true;
        BFI_HIP(hipEventSynchronize(ev_e_));
        // the estimate from the totals, as the finalize forms it
        std::memset(res, 0, sizeof(*res));
        res->nx = nx_;
        const double *T = h_totals_;
        const double sig = T[0], z = T[1];
        if (!std::isfinite(sig))
            return fail(BFI_EINVAL, "partial records carry no finite shift");
        res->log_Z = std::log(z) - sig;
        res->Z = std::exp(res->log_Z);
        res->Z_err = std::sqrt(std::max(T[2], 0.0)) * std::exp(-sig);
        res->ess = T[3] > 0 ? z * z / T[3] : 0.0;
        res->n_evals = T[4];
        for (int r = 0; r < nx_; ++r) {
            res->C[r] = T[5 + r] / z;
            res->C_err[r] = std::sqrt(std::max(T[5 + nx_ + r], 0.0)) / std::fabs(z);
        }
        return BFI_OK;
    }
    // wait for the last analysis's split choices (best(), gain()); its device
    // time, and the fold's before it, go to device_ms
    bfi_status wait_choices(double *device_ms)
    {
        if (!choices_pending_)
            return BFI_OK;
        choices_pending_ = false;
        BFI_HIP(hipEventSynchronize(ev_a1_));
        float ms = 0.0f;
        BFI_HIP(hipEventElapsedTime(&ms, ev_a0_, ev_a1_));
        if (device_ms)
            *device_ms += ms;
        if (folded_) {
            BFI_HIP(hipEventElapsedTime(&ms, ev_f0_, ev_f1_));
            if (device_ms)
                *device_ms += ms;
            folded_ = false;
        }
        return BFI_OK;
    }
    const double *e() const { return h_e_; }
    const int32_t *best() const { return h_best_; }
    const double *gain() const { return h_gain_; }

private:
    bfi_status events()
    {
        if (!ev_f0_)
            for (hipEvent_t *ev : {&ev_f0_, &ev_f1_, &ev_a0_, &ev_e_, &ev_a1_})
                BFI_HIP(hipEventCreate(ev));
        return BFI_OK;
    }
    bfi_context *ctx_;
    int nx_, d_, rec_len_, split_len_;
    size_t cap_ = 0;  // leaves
    double *rec_ = nullptr, *split_ = nullptr, *base_ = nullptr, *vol_ = nullptr;
    double *e_d_ = nullptr, *gain_d_ = nullptr, *scratch_ = nullptr, *totals_d_ = nullptr;
    int32_t *best_d_ = nullptr;
    FoldEntry *fold_d_ = nullptr, *h_fold_ = nullptr;
    size_t cap_scratch_ = 0, cap_totals_ = 0, cap_dfold_ = 0, cap_hfold_ = 0;
    double *h_e_ = nullptr, *h_gain_ = nullptr, *h_totals_ = nullptr;
    int32_t *h_best_ = nullptr;
    size_t cap_he_ = 0, cap_hg_ = 0, cap_hb_ = 0, cap_htotals_ = 0;
    hipEvent_t ev_f0_ = nullptr, ev_f1_ = nullptr, ev_a0_ = nullptr, ev_e_ = nullptr,
               ev_a1_ = nullptr;
    bool choices_pending_ = false;
    bool folded_ = false;
};

// The resident evaluators of a run: the kernel variant with split statistics
// and the plain kernel, each with its buffers and captured graph kept from
// round to round (records left in device memory for the fold), and a plain one
// for holdout checks, whose records come back to the host.
struct Evaluators {
    ResidentEval with, without, holdout;
    bool holdout_ready = false;
    double device_ms = 0.0;  // device time of every list, fold and analysis so far
};

constexpr size_t kGrain = 2048;  // entries per chunk of the parallel host loops

// Where a work list's entries went: entry w's samples below split_samples are
// row wpos[w] of the split-statistics pass, the rest row opos[w] of the plain
// pass (-1: no such samples).
struct ListPos {
    std::vector<int64_t> wpos, opos;
    int64_t nw = 0, no = 0;
};

// Stage a work list and queue its two passes on the context's stream: the
// samples below index `split_samples` of each stream (all of them when 0)
// through the kernel variant with split statistics, the rest through the
// plain kernel.
bfi_status launch_list(Evaluators *ev, const bfi_lattice &lat, uint64_t seed, const SubList &work,
                       uint64_t split_samples, ListPos *pos)
{
    const int d = lat.nx * lat.nt;
    const size_t count = work.size();
    {
        TraceRange tr("adaptive: stage");
        pos->wpos.resize(count);
        pos->opos.resize(count);
        std::vector<uint64_t> cut(count);
        // rows in list order: each chunk counts its entries of either pass,
        // then numbers them from the chunk's start
        const size_t nch = (count + kGrain - 1) / kGrain;
        std::vector<int64_t> cw(nch + 1, 0), co(nch + 1, 0);
        for_chunks(nch, [&](size_t c) {
            int64_t kw = 0, ko = 0;
            for (size_t w = c * kGrain; w < std::min(count, (c + 1) * kGrain); ++w) {
                const uint64_t off = work.offset[w], end = off + work.n[w];
                cut[w] = split_samples == 0 ? end : std::min(std::max(split_samples, off), end);
                kw += cut[w] > off;
                ko += end > cut[w];
            }
            cw[c + 1] = kw;
            co[c + 1] = ko;
        });
        for (size_t c = 0; c < nch; ++c) {
            cw[c + 1] += cw[c];
            co[c + 1] += co[c];
        }
        for_chunks(nch, [&](size_t c) {
            int64_t kw = cw[c], ko = co[c];
            for (size_t w = c * kGrain; w < std::min(count, (c + 1) * kGrain); ++w) {
                const uint64_t off = work.offset[w], end = off + work.n[w];
                pos->wpos[w] = cut[w] > off ? kw++ : -1;
                pos->opos[w] = end > cut[w] ? ko++ : -1;
            }
        });
        const int64_t nw = cw[nch], no = co[nch];
        pos->nw = nw;
        pos->no = no;
        if (nw > std::numeric_limits<int32_t>::max() || no > std::numeric_limits<int32_t>::max())
            return fail(BFI_EINVAL, "more than 2^31 entries in one pass");
        BFI_TRY(ev->with.stage(static_cast<size_t>(nw)));
        BFI_TRY(ev->without.stage(static_cast<size_t>(no)));
        // every entry of the split pass; the plain pass's counts only (its
        // boxes are written while the split pass runs)
        parallel_range(count, kGrain, [&](size_t w) {
            const uint64_t off = work.offset[w], end = off + work.n[w];
            if (pos->wpos[w] >= 0)
                ev->with.set(static_cast<size_t>(pos->wpos[w]), work.id[w], off, cut[w] - off,
                             &work.lo[w * d], &work.hi[w * d]);
            if (pos->opos[w] >= 0)
                ev->without.set_counts(static_cast<size_t>(pos->opos[w]), work.id[w], cut[w],
                                       end - cut[w]);
        });
    }
    {
        // both replays prepared (allocation, capture and update while the
        // device is idle), the split pass queued first
        TraceRange tr("adaptive: prepare and launch");
        if (pos->nw > 0)
            BFI_TRY(ev->with.prepare(seed));
        if (pos->no > 0)
            BFI_TRY(ev->without.prepare(seed));
        if (pos->nw > 0)
            BFI_TRY(ev->with.launch());
    }
    if (pos->no > 0) {
        {
            TraceRange tr("adaptive: plain pass boxes (while the split pass runs)");
            parallel_range(count, kGrain, [&](size_t w) {
                if (pos->opos[w] >= 0)
                    ev->without.set_box(static_cast<size_t>(pos->opos[w]), &work.lo[w * d],
                                        &work.hi[w * d]);
            });
        }
        BFI_TRY(ev->without.launch());
    }
    return BFI_OK;
}

// Wait for a list's passes (their replay times go to device_ms).
bfi_status finish_list(Evaluators *ev, const ListPos &pos)
{
    if (pos.nw > 0) {
        TraceRange tr("adaptive: samples with split statistics");
        double ms = 0.0;
        BFI_TRY(ev->with.finish(nullptr, nullptr, &ms));
        ev->device_ms += ms;
    }
    if (pos.no > 0) {
        TraceRange tr("adaptive: samples through the plain kernel");
        double ms = 0.0;
        BFI_TRY(ev->without.finish(nullptr, nullptr, &ms));
        ev->device_ms += ms;
    }
    return BFI_OK;
}

}  // namespace

extern "C" {

bfi_status bfi_integrate_adaptive(bfi_context *ctx, const bfi_lattice *lat, bfi_precision prec,
                                  uint64_t seed, const double *box_lo, const double *box_hi,
                                  const bfi_adaptive_config *cfg, const bfi_launch *launch,
                                  bfi_result *out, bfi_adaptive_stats *stats, uint64_t *leaf_id,
                                  double *leaf_lo, double *leaf_hi, uint64_t *leaf_n,
                                  uint64_t *leaf_offset, size_t cap, size_t *n_leaves)
{
    return guarded([&]() -> bfi_status {
        TraceRange trace("bfi_integrate_adaptive");
        if (!ctx || !box_lo || !box_hi || !out)
            return fail(BFI_EINVAL, "arguments must be non-NULL");
        if (!known_precision(prec))
            return fail(BFI_EINVAL, "unknown precision");
        BFI_TRY(check_lattice(lat));
        BFI_TRY(check_config(cfg));
        if (lat->antithetic)
            return fail(BFI_EUNSUPPORTED, "adaptive refinement uses single points (antithetic = 0)");
        const int nx = lat->nx, d = nx * lat->nt;
        if (d > 32)
            return fail(BFI_EUNSUPPORTED, "adaptive refinement needs d <= 32 (split statistics)");
        for (int k = 0; k < d; ++k)
            if (!std::isfinite(box_lo[k]) || !std::isfinite(box_hi[k]) || !(box_lo[k] < box_hi[k]))
                return fail(BFI_EINVAL, "box dim %d: need finite lo < hi", k);
        const int rec_len = BFI_PARTIAL_LEN(nx);

        // initial uniform partition with n_min samples per leaf
        SubList init = uniform_split(d, box_lo, box_hi, cfg->split_log2, 0);
        std::fill(init.n.begin(), init.n.end(), cfg->n_min);
        uint64_t evals = static_cast<uint64_t>(init.size()) * cfg->n_min;
        if (evals > cfg->max_evals)
            return fail(BFI_EINVAL, "initial partition exceeds max_evals");
        LeafSet L;
        L.d = d;
        L.nx = nx;
        L.id.assign(init.id.begin(), init.id.end());
        L.n.assign(init.n.begin(), init.n.end());
        L.lo.assign(init.lo.begin(), init.lo.end());
        L.hi.assign(init.hi.begin(), init.hi.end());
        L.vol.resize(L.size());
        for (size_t s = 0; s < L.size(); ++s)
            L.vol[s] = box_volume(&L.lo[s * d], &L.hi[s * d], d);
        BFI_HIP(hipSetDevice(ctx->device));
        Evaluators ev;
        BFI_TRY(ev.with.init(ctx, *lat, prec, true, launch));
        BFI_TRY(ev.without.init(ctx, *lat, prec, false, launch));
        ev.with.set_copy_records(false);
        ev.without.set_copy_records(false);
        DeviceLeaves DL(ctx, nx, d);
        BFI_TRY(DL.reserve(L.size(), 0));
        ListPos pos;
        {
            // every entry of the initial list becomes the leaf of its index
            BFI_TRY(DL.stage_fold(init.size()));
            BFI_TRY(launch_list(&ev, *lat, seed, init, cfg->split_samples, &pos));
            FoldEntry *fe = DL.fold_entries();
            parallel_range(init.size(), kGrain, [&](size_t w) {
                fe[w] = FoldEntry{static_cast<uint32_t>(w), 1, static_cast<int32_t>(pos.wpos[w]),
                                  static_cast<int32_t>(pos.opos[w]), L.vol[w]};
            });
            BFI_TRY(DL.fold(init.size(), ev.with.device_records(), ev.with.device_split_records(),
                            ev.without.device_records()));
            BFI_TRY(finish_list(&ev, pos));
        }

        bfi_status status = BFI_OK;
        const double min_ess = cfg->min_ess > 0 ? cfg->min_ess : 100.0;
        int rounds = 0, checks = 0;
        bool holdout_used = false;
        uint64_t holdout_seed = 0;
        double holdout_err = 0.0;
        double run_target = cfg->target_rel_err;  // tightened by failed holdout checks
        bfi_result res{};
        auto report = [&](double running) {
            if (!cfg->progress)
                return;
            bfi_adaptive_progress p{rounds, checks, L.size(), evals, running, holdout_err};
            cfg->progress(&p, cfg->progress_user);
        };
        // round buffers, kept between rounds (their pages stay mapped)
        struct Origin {
            size_t leaf;
            int kind;  // 0 continuation, 1 lower child, 2 upper child
        };
        SubList work;
        std::vector<Origin> origin;
        std::vector<size_t> first_entry, dst, refined;
        std::vector<int32_t> action;
        std::vector<uint64_t> target;
        for (;;) {
            TracePhases phase("adaptive: analyse");
            BFI_TRY(DL.analyse(L.size(), &res, &ev.device_ms));
            const double *e = DL.e();
            const int32_t *best = DL.best();
            const double *gain = DL.gain();
            report(rel_err(res));
            // stop check; with holdout, a failed check tightens the running target
            // and refinement goes on: the next check comes after at least one more
            // round, never on the same leaves again (a fresh draw over unchanged
            // leaves until one meets the target would select among draws)
            bool stop = false;
            if (rel_err(res) <= run_target && res.ess >= min_ess) {
                if (!cfg->holdout) {
                    stop = true;
                } else {
                    phase.next("adaptive: holdout pass");
                    // holdout check: the same leaves, samples drawn afresh under a
                    // seed of their own, so no refinement decision has seen them
                    uint64_t cost = 0;
                    for (uint64_t n : L.n)
                        cost += n;
                    if (cost > cfg->max_evals - evals) {
                        status = BFI_EBUDGET;
                        stop = true;
                    } else {
                        ++checks;
                        const uint64_t hseed =
                            seed + static_cast<uint64_t>(checks) * 0x9E3779B97F4A7C15ull;
                        std::vector<double> hrec(L.size() * rec_len);
                        if (!ev.holdout_ready) {
                            BFI_TRY(ev.holdout.init(ctx, *lat, prec, false, launch));
                            ev.holdout_ready = true;
                        }
                        BFI_TRY(ev.holdout.stage(L.size()));
                        parallel_range(L.size(), kGrain, [&](size_t s) {
                            ev.holdout.set(s, L.id[s], 0, L.n[s], &L.lo[s * d], &L.hi[s * d]);
                        });
                        double hms = 0.0;
                        BFI_TRY(ev.holdout.run(hseed, hrec.data(), nullptr, &hms));
                        ev.device_ms += hms;
                        evals += cost;
                        bfi_result hres{};
                        BFI_TRY(finalize_records(nx, d, L.size(), L.lo.data(), L.hi.data(),
                                                 hrec.data(), &hres, 1, nullptr, L.vol.data()));
                        const double herr = rel_err(hres);
                        holdout_err = herr;
                        report(rel_err(res));
                        if (herr <= cfg->target_rel_err && hres.ess >= min_ess) {
                            res = hres;
                            holdout_used = true;
                            holdout_seed = hseed;
                            stop = true;
                        } else {
                            // the running estimate was optimistic: ask more of it
                            run_target *= std::min(0.5, cfg->target_rel_err / herr);
                        }
                    }
                }
            }
            if (stop)
                break;
            // every action costs samples (a doubling at least n, a split at least
            // 2 n_min): with the budget spent the trim below would drop them all
            if (rounds >= cfg->max_rounds || evals >= cfg->max_evals) {
                status = BFI_EBUDGET;
                break;
            }
            phase.next("adaptive: decide and plan");
            action.resize(L.size());
            // a leaf's action from its split choice (the device analysis made it)
            auto act = [&](size_t s) {
                return action_of(SplitChoice{best[s], gain[s]}, L.id[s], L.n[s], *cfg);
            };
            std::optional<TraceRange> sub(std::in_place, "adaptive: rank and decide");
            Ranking order(e, L.size(), L.id.data());
            BFI_TRY(DL.wait_choices(&ev.device_ms));
            const size_t examined = decide(e, L.size(), act, *cfg, action.data(), order);
            // the refined leaves in rank order (planning loops over these only)
            refined.clear();
            for (size_t i = 0; i < examined; ++i)
                if (action[order[i]] >= 0)
                    refined.push_back(order[i]);

            // planned sample counts: children clamp(n, n_min, n_max) each, doubled
            // leaves 2n; scaled by a power of two up to the round's work floor
            // planned count of a refined leaf at scale factor f (within n_max):
            // children clamp(n, n_min, n_max) each, doubled leaves 2n, times f
            target.resize(L.size());  // new per-leaf (or per-child) count, refined leaves
            // planned count of a leaf with action `act` and n samples at factor
            // f = 2^fs (a power of two: shifts, not divisions)
            auto target_of = [&](int32_t act, uint64_t n, unsigned fs) {
                const uint64_t base =
                    act == 0 ? 2 * n : std::min(std::max(n, cfg->n_min), cfg->n_max);
                const uint64_t cap = std::max(cfg->n_max, base);
                return base > (cap >> fs) ? cap : std::max(base, std::min(base << fs, cap));
            };
            auto cost_of = [](int32_t act, uint64_t n, uint64_t t) {
                return act == 0 ? t - n : 2 * t;
            };
            // whether the count would still grow at 2f
            auto grows_of = [&](int32_t act, uint64_t n, unsigned fs, uint64_t t) {
                return fs < 63 && target_of(act, n, fs + 1) > t;
            };
            unsigned fs = 0;
            uint64_t planned = 0;
            size_t growable = 0;
            // actions and counts of the leaves the work floor takes, in the order
            // taken (refined[pending + i]); written to the leaves' arrays in parallel
            // before they are read
            std::vector<int32_t> pend_act;
            std::vector<uint64_t> pend_target;
            size_t pending = refined.size();
            auto flush = [&]() {
                parallel_range(pend_act.size(), kGrain, [&](size_t i) {
                    const size_t s = refined[pending + i];
                    action[s] = pend_act[i];
                    target[s] = pend_target[i];
                });
                pending = refined.size();
                pend_act.clear();
                pend_target.clear();
            };
            // every refined leaf at factor f: per-chunk integer sums, so the
            // totals do not depend on the chunking
            std::vector<uint64_t> chunk_planned;
            std::vector<size_t> chunk_growable;
            auto plan_all = [&]() {
                const size_t nr = refined.size(), nch = (nr + kGrain - 1) / kGrain;
                chunk_planned.assign(nch, 0);
                chunk_growable.assign(nch, 0);
                for_chunks(nch, [&](size_t c) {
                    uint64_t p = 0;
                    size_t g = 0;
                    for (size_t i = c * kGrain; i < std::min(nr, (c + 1) * kGrain); ++i) {
                        const size_t s = refined[i];
                        const uint64_t t = target_of(action[s], L.n[s], fs);
                        target[s] = t;
                        p += cost_of(action[s], L.n[s], t);
                        g += grows_of(action[s], L.n[s], fs, t);
                    }
                    chunk_planned[c] = p;
                    chunk_growable[c] = g;
                });
                planned = 0;
                growable = 0;
                for (size_t c = 0; c < nch; ++c) {
                    planned += chunk_planned[c];
                    growable += chunk_growable[c];
                }
            };
            sub.reset();
            sub.emplace("adaptive: work floor");
            plan_all();
            // work floor: scale the refined leaves by powers of two; once n_max caps
            // them all, refine further leaves in variance order (each at the current
            // factor; the next pass doubles again if one of them can still grow)
            size_t next_leaf = 0;
            // the next candidates in rank order, a batch at a time: leaf, decision
            // (each depends on its own leaf only; kHasAction for a leaf that
            // decide() gave an action) and sample count, gathered in parallel so
            // that the scan below reads them in order; ranks [batch_lo, + size).
            // Which decisions a batch computes ahead changes no result.
            constexpr int32_t kHasAction = std::numeric_limits<int32_t>::min();
            // with, for a leaf the floor may take, its count, cost and whether it
            // would grow at twice the factor, all at factor 2^plan_fs (pure
            // functions of the decision, n and the factor: computed with the
            // batch, again for the batch's rest when the factor changes)
            struct Candidate {
                size_t leaf;
                int32_t act;
                uint64_t n, t, cost;
                bool grows;
            };
            std::vector<Candidate> batch;
            size_t batch_lo = 0;
            unsigned plan_fs = 0;
            auto plan_batch = [&](size_t k0) {
                parallel_range(batch.size() - k0, size_t(1) << 9, [&](size_t i) {
                    Candidate &c = batch[k0 + i];
                    if (c.act < 0)
                        return;
                    c.t = target_of(c.act, c.n, fs);
                    c.cost = cost_of(c.act, c.n, c.t);
                    c.grows = grows_of(c.act, c.n, fs, c.t);
                });
                plan_fs = fs;
            };
            auto candidate = [&](size_t rank) -> const Candidate & {
                if (rank < batch_lo || rank >= batch_lo + batch.size()) {
                    // a leaf adds at most 2 n_max samples (counts stay within n_max):
                    // the round needs at least this many more leaves
                    const uint64_t left = cfg->round_evals - planned;
                    const uint64_t need = cfg->n_max <= std::numeric_limits<uint64_t>::max() / 2
                                              ? left / (2 * cfg->n_max) + 1
                                              : 1;
                    const size_t len = static_cast<size_t>(std::min<uint64_t>(
                        order.size() - rank, std::max<uint64_t>(4096, need)));
                    order.gather(rank + len);  // the ranks first (one extension)
                    batch.resize(len);
                    batch_lo = rank;
                    parallel_range(len, size_t(1) << 9, [&](size_t k) {
                        const size_t s = order[rank + k];
                        batch[k] = Candidate{s, action[s] == -1 ? act(s) : kHasAction, L.n[s],
                                             0, 0, false};
                    });
                    plan_batch(0);
                } else if (plan_fs != fs) {
                    plan_batch(rank - batch_lo);
                }
                return batch[rank - batch_lo];
            };
            while (cfg->round_evals > 0 && planned < cfg->round_evals) {
                if (growable > 0) {
                    TraceRange tr("adaptive: replan at twice the factor");
                    ++fs;
                    flush();
                    plan_all();
                    continue;
                }
                // the scan only moves forward and a batch holds ranks from the
                // scan's position on, so its view of which leaves have an action
                // (those decide() gave one) stays current
                const Candidate *c = nullptr;
                while (next_leaf < order.size() && (c = &candidate(next_leaf))->act == kHasAction)
                    ++next_leaf;
                if (next_leaf == order.size())
                    break;
                ++next_leaf;
                if (c->act < 0)
                    continue;  // neither split nor doubling possible: skip it
                refined.push_back(c->leaf);
                pend_act.push_back(c->act);
                pend_target.push_back(c->t);
                planned += c->cost;
                growable += c->grows;
            }
            flush();
            sub.reset();
            sub.emplace("adaptive: budget trim");
            // trim to the evaluation budget in priority order (every refined leaf
            // lies in the part of the ranking read so far); `planned` is the
            // plan's whole cost, so a plan within the budget needs no pass
            uint64_t cost = 0;
            if (evals <= cfg->max_evals && planned <= cfg->max_evals - evals) {
                cost = planned;
            } else {
                for (size_t i = 0; i < order.sorted(); ++i) {
                    const size_t s = order[i];
                    if (action[s] < 0)
                        continue;
                    const uint64_t c = action[s] == 0 ? target[s] - L.n[s] : 2 * target[s];
                    if (evals + cost + c > cfg->max_evals)
                        action[s] = -1;
                    else
                        cost += c;
                }
            }
            sub.reset();
            if (cost == 0) {
                status = BFI_EBUDGET;
                break;
            }

            // work list: children (fresh streams) and continuations, each refined
            // leaf's entries at a precomputed position, filled in parallel
            phase.next("adaptive: work list");
            // entry offsets: counts per chunk of leaves, the chunks' starts in
            // order, then each chunk's offsets from its start
            first_entry.resize(L.size());
            const size_t nfc = (L.size() + kGrain - 1) / kGrain;
            std::vector<size_t> chunk_start(nfc + 1, 0);
            auto entries_of = [&](size_t s) -> size_t {
                return action[s] < 0 ? 0 : action[s] == 0 ? 1 : 2;
            };
            for_chunks(nfc, [&](size_t c) {
                size_t k = 0;
                for (size_t s = c * kGrain; s < std::min(L.size(), (c + 1) * kGrain); ++s)
                    k += entries_of(s);
                chunk_start[c + 1] = k;
            });
            for (size_t c = 0; c < nfc; ++c)
                chunk_start[c + 1] += chunk_start[c];
            const size_t entries = chunk_start[nfc];
            for_chunks(nfc, [&](size_t c) {
                size_t k = chunk_start[c];
                for (size_t s = c * kGrain; s < std::min(L.size(), (c + 1) * kGrain); ++s) {
                    first_entry[s] = k;
                    k += entries_of(s);
                }
            });
            work.d = d;
            work.id.resize(entries);
            work.n.resize(entries);
            work.offset.resize(entries);
            work.lo.resize(entries * d);
            work.hi.resize(entries * d);
            origin.resize(entries);
            parallel_range(L.size(), kGrain, [&](size_t s) {
                if (action[s] < 0)
                    return;
                const double *lo = &L.lo[s * d], *hi = &L.hi[s * d];
                const size_t e = first_entry[s];
                if (action[s] == 0) {
                    work.id[e] = L.id[s];
                    work.n[e] = target[s] - L.n[s];
                    work.offset[e] = L.n[s];
                    std::copy(lo, lo + d, &work.lo[e * d]);
                    std::copy(hi, hi + d, &work.hi[e * d]);
                    origin[e] = {s, 0};
                    return;
                }
                const int j = action[s] - 1;
                const double mid = 0.5 * (lo[j] + hi[j]);
                for (int half = 0; half < 2; ++half) {
                    const size_t w = e + half;
                    work.id[w] = 2 * L.id[s] + half;
                    work.n[w] = target[s];
                    work.offset[w] = 0;
                    std::copy(lo, lo + d, &work.lo[w * d]);
                    std::copy(hi, hi + d, &work.hi[w * d]);
                    if (half == 0)
                        work.hi[w * d + j] = mid;
                    else
                        work.lo[w * d + j] = mid;
                    origin[w] = {s, 1 + half};
                }
            });
            // destinations: a doubled leaf merges its continuation, a split leaf
            // becomes its lower child and its upper child is appended; capacity
            // grows geometrically and by remapping (an exact reserve, or a copying
            // one, would move the whole leaf set, gigabytes at millions of leaves,
            // every round)
            std::optional<TraceRange> grow_range(std::in_place, "adaptive: leaf set growth");
            dst.resize(origin.size());
            const size_t before = L.size();
            // upper children numbered from `before` in list order: counts per
            // chunk of entries, the chunks' starts, then each chunk's numbers
            const size_t nwc = (origin.size() + kGrain - 1) / kGrain;
            std::vector<size_t> upper_start(nwc + 1, 0);
            for_chunks(nwc, [&](size_t c) {
                size_t k = 0;
                for (size_t w = c * kGrain; w < std::min(origin.size(), (c + 1) * kGrain); ++w)
                    k += origin[w].kind == 2;
                upper_start[c + 1] = k;
            });
            upper_start[0] = before;
            for (size_t c = 0; c < nwc; ++c)
                upper_start[c + 1] += upper_start[c];
            for_chunks(nwc, [&](size_t c) {
                size_t next = upper_start[c];
                for (size_t w = c * kGrain; w < std::min(origin.size(), (c + 1) * kGrain); ++w)
                    dst[w] = origin[w].kind == 2 ? next++ : origin[w].leaf;
            });
            const size_t grown = upper_start[nwc];
            L.id.resize(grown);
            L.n.resize(grown);
            L.lo.resize(grown * d);
            L.hi.resize(grown * d);
            L.vol.resize(grown);
            {
                TraceRange tr("adaptive: device leaf buffers");
                BFI_TRY(DL.reserve(grown, before));
            }
            grow_range.reset();
            phase.next("adaptive: evaluate and fold");
            // pinned room for the fold entries first: freeing a pinned buffer
            // waits for the device, which must not happen behind the passes
            BFI_TRY(DL.stage_fold(origin.size()));
            BFI_TRY(launch_list(&ev, *lat, seed, work, cfg->split_samples, &pos));
            {
                // while the device evaluates: the fold entries and the host side
                // of the leaves (every entry has a leaf of its own)
                TraceRange tr("adaptive: fold entries");
                FoldEntry *fe = DL.fold_entries();
                parallel_range(origin.size(), kGrain, [&](size_t w) {
                    const size_t s = dst[w];
                    double vol = 0.0;
                    if (origin[w].kind == 0) {
                        L.n[s] = target[s];
                    } else {
                        L.id[s] = work.id[w];
                        L.n[s] = work.n[w];
                        std::copy(&work.lo[w * d], &work.lo[w * d] + d, &L.lo[s * d]);
                        std::copy(&work.hi[w * d], &work.hi[w * d] + d, &L.hi[s * d]);
                        vol = box_volume(&L.lo[s * d], &L.hi[s * d], d);
                        L.vol[s] = vol;
                    }
                    fe[w] = FoldEntry{static_cast<uint32_t>(s), origin[w].kind,
                                      static_cast<int32_t>(pos.wpos[w]),
                                      static_cast<int32_t>(pos.opos[w]), vol};
                });
            }
            BFI_TRY(DL.fold(origin.size(), ev.with.device_records(), ev.with.device_split_records(),
                            ev.without.device_records()));
            BFI_TRY(finish_list(&ev, pos));
            evals += cost;
            ++rounds;
        }

        BFI_TRY(DL.wait_choices(&ev.device_ms));
        *out = res;
        if (stats) {
            stats->rounds = rounds;
            stats->leaves = L.size();
            stats->evals = evals;
            stats->rel_err = rel_err(res);
            stats->holdout_checks = checks;
            stats->holdout_used = holdout_used ? 1 : 0;
            stats->holdout_seed = holdout_seed;
            stats->holdout_rel_err = holdout_err;
            stats->device_seconds = ev.device_ms * 1e-3;
            stats->graph_instantiations = ev.with.instantiations() + ev.without.instantiations();
            stats->graph_updates = ev.with.updates() + ev.without.updates();
        }
        if (n_leaves)
            *n_leaves = L.size();
        // the partition out, in parallel chunks (hundreds of megabytes at a
        // million leaves, into pages the caller has mostly not touched yet)
        const size_t m = std::min(cap, L.size());
        const size_t nout = (m + kGrain - 1) / kGrain;
        for_chunks(nout, [&](size_t c) {
            const size_t b = c * kGrain, e = std::min(m, b + kGrain);
            if (leaf_id)
                std::memcpy(leaf_id + b, &L.id[b], (e - b) * sizeof(uint64_t));
            if (leaf_n)
                std::memcpy(leaf_n + b, &L.n[b], (e - b) * sizeof(uint64_t));
            if (leaf_offset)
                std::memset(leaf_offset + b, 0, (e - b) * sizeof(uint64_t));
            if (leaf_lo)
                std::memcpy(leaf_lo + b * d, &L.lo[b * d], (e - b) * d * sizeof(double));
            if (leaf_hi)
                std::memcpy(leaf_hi + b * d, &L.hi[b * d], (e - b) * d * sizeof(double));
        });
        if (status == BFI_EBUDGET)
            fail(BFI_EBUDGET, "stopped after %d rounds at relative error %.3g (target %.3g)", rounds,
                 rel_err(res), cfg->target_rel_err);
        return status;
    });
}

bfi_status bfi_adaptive_decide(const bfi_lattice *lat, const bfi_subvolumes *leaves,
                               const double *partials, const double *split,
                               const double *split_base, const bfi_adaptive_config *cfg,
                               int32_t *action)
{
    return guarded([&]() -> bfi_status {
        if (!lat || !leaves || !partials || !split || !action)
            return fail(BFI_EINVAL, "arguments must be non-NULL");
        BFI_TRY(check_config(cfg));
        if (lat->antithetic)
            return fail(BFI_EUNSUPPORTED, "adaptive refinement uses single points (antithetic = 0)");
        if (lat->nx < 1 || lat->nt < 1 || lat->nx * lat->nt > 32)
            return fail(BFI_EINVAL, "adaptive refinement needs 1 <= d <= 32");
        if (leaves->count == 0)
            return fail(BFI_EINVAL, "no leaves");
        if (!leaves->id || !leaves->lo || !leaves->hi || !leaves->n)
            return fail(BFI_EINVAL, "leaf arrays must be non-NULL");
        const int d = lat->nx * lat->nt;
        std::vector<double> e;
        bfi_result res;
        BFI_TRY(analyse(lat->nx, d, leaves->count, leaves->lo, leaves->hi, partials, &e, &res));
        const SplitStats st{d, BFI_PARTIAL_LEN(lat->nx), split, split_base ? split_base : partials};
        Ranking order(e.data(), e.size(), leaves->id);
        decide(
            e.data(), e.size(),
            [&](size_t s) {
                return action_of(split_choice(st, s), leaves->id[s], leaves->n[s], *cfg);
            },
            *cfg, action, order);
        return BFI_OK;
    });
}

bfi_status bfi_partials_merge(int32_t nx, size_t count, double *acc, const double *more)
{
    return guarded([&]() -> bfi_status {
        if (nx < 1 || nx > BFI_MAX_NX)
            return fail(BFI_EINVAL, "nx must be in [1, %d]", BFI_MAX_NX);
        if (count == 0)
            return BFI_OK;
        if (!acc || !more)
            return fail(BFI_EINVAL, "record arrays must be non-NULL");
        const size_t len = BFI_PARTIAL_LEN(nx);
        constexpr double kMaxCount = 9007199254740992.0;  // 2^53: counts stay exact
        for (size_t i = 0; i < count; ++i) {
            const double *a = acc + i * len, *b = more + i * len;
            for (const double *r : {a, b}) {
                if (!(r[0] >= 0) || !(r[0] <= kMaxCount) || r[0] != std::floor(r[0]))
                    return fail(BFI_EINVAL, "record %zu: sample count must be a whole number >= 0",
                                i);
                if (r[0] > 0 && !std::isfinite(r[1]))
                    return fail(BFI_EINVAL, "record %zu: shift must be finite", i);
            }
            if (a[0] + b[0] > kMaxCount)
                return fail(BFI_EINVAL, "record %zu: merged sample count exceeds 2^53", i);
        }
        std::vector<int> first, second;
        record_fields(nx, &first, &second);
        for (size_t i = 0; i < count; ++i) {
            double *a = acc + i * len;
            const double *b = more + i * len;
            if (b[0] == 0)
                continue;
            if (a[0] == 0) {
                std::memcpy(a, b, len * sizeof(double));
                continue;
            }
            merge_shifted(a, b, 1, first, second, 0);
        }
        return BFI_OK;
    });
}

}  // extern "C"
