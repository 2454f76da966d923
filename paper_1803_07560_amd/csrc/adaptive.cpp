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
// is drained by the persistent kernel through the device queue.
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

struct LeafAnalysis {
    double e = 0.0;        // contribution to the variance of C
    int best_dim = 0;      // j*
    double gain = 1.0;     // (sigma_L + sigma_U)(j*) / (2 sigma)
};

// Contribution of every leaf to the variance of C, and the estimate itself
// (both from the finalize's two passes over the records).
bfi_status analyse(int nx, int d, size_t count, const double *lo, const double *hi,
                   const double *partials, std::vector<LeafAnalysis> *out, bfi_result *res,
                   const double *vol = nullptr)
{
    thread_local std::vector<double> e;  // reused across rounds
    if (e.size() < count)
        e.resize(count);
    BFI_TRY(finalize_records(nx, d, count, lo, hi, partials, res, 1, e.data(), vol));
    out->resize(count);
    const double *ev = e.data();
    LeafAnalysis *ov = out->data();
    parallel_range(count, size_t(1) << 16, [ev, ov](size_t s) {
        ov[s] = LeafAnalysis{ev[s] >= 0.0 ? ev[s] : 0.0, 0, 1.0};  // NaN ranks last
    });
    return BFI_OK;
}

// Split statistics of the leaves: `split` (BFI_SPLIT_LEN(d) per leaf) and `base`,
// the record of the samples they cover (the whole leaf, or its first
// split_samples samples).
struct SplitStats {
    int d, rec_len;
    const double *split, *base;
};

// j* and the gain of leaf s, in the shift of the covered samples (the split
// record shares it).
void split_choice(const SplitStats &st, size_t s, LeafAnalysis *a)
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
    a->best_dim = best_j;
    a->gain = sigma > 0 ? best / (2.0 * sigma) : 1.0;
}

double rel_err(const bfi_result &r)
{
    double m = 0.0;
    for (int k = 0; k < r.nx; ++k)
        m = std::max(m, r.C_err[k]);
    return r.C[0] != 0.0 ? m / std::fabs(r.C[0]) : std::numeric_limits<double>::infinity();
}

bool can_split(uint64_t id) { return id < (uint64_t(1) << 62); }

// Action of refined leaf s: split along j* when that halves the spread well
// enough or doubling would exceed n_max, else double; -1 if neither is possible.
// The split analysis is done here, for the leaves that are refined only.
int32_t leaf_action(std::vector<LeafAnalysis> &an, const SplitStats &st, size_t s, uint64_t id,
                    uint64_t n, const bfi_adaptive_config &cfg)
{
    const bool doubling_ok = n <= cfg.n_max / 2;
    if (can_split(id)) {
        split_choice(st, s, &an[s]);
        if (an[s].gain < kSplitGain || !doubling_ok)
            return 1 + an[s].best_dim;
    }
    return doubling_ok ? 0 : -1;
}

// Leaves in ranking order (descending contribution e, ties by lower id), built
// lazily: for e >= 0 the IEEE bit pattern orders like the value, so one
// parallel pass counts the leaves per bucket of its top bits; a read at rank i
// gathers whole buckets from the top (at least twice what was gathered before)
// and sorts only those.  Whole buckets keep the order exact: the result is the
// full sort's, but a round that refines the top few percent of millions of
// leaves never sorts the rest.
class Ranking {
public:
    Ranking(const std::vector<LeafAnalysis> &an, const uint64_t *ids) : an_(an), ids_(ids)
    {
        const size_t n = an.size();
        nchunks_ = (n + kChunk - 1) / kChunk;
        part_.assign(nchunks_, {});
        bucket_.resize(n);
        std::vector<double> sums(nchunks_, 0.0);
        for_chunks(nchunks_, [&](size_t c) {
            part_[c].assign(kBuckets, 0);
            const size_t i1 = std::min(n, (c + 1) * kChunk);
            double sum = 0.0;
            for (size_t s = c * kChunk; s < i1; ++s) {
                const uint16_t b = bucket(an[s].e);
                bucket_[s] = b;
                ++part_[c][b];
                sum += an[s].e;
            }
            sums[c] = sum;
        });
        hist_.assign(kBuckets, 0);
        for (const auto &h : part_)
            for (size_t b = 0; b < kBuckets; ++b)
                hist_[b] += h[b];
        total_ = 0.0;
        for (double x : sums)
            total_ += x;
        top_ = kBuckets;
    }
    size_t size() const { return an_.size(); }
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
        const size_t n = an_.size();
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
                    keys_[at[hi - 1 - b]++] = Key{an_[s].e, ids_[s], s};
            }
        });
        for_chunks(span, [&](size_t k) {
            if (first[k + 1] - first[k] > 1)
                std::sort(keys_.begin() + static_cast<std::ptrdiff_t>(first[k]),
                          keys_.begin() + static_cast<std::ptrdiff_t>(first[k + 1]), before);
        });
        top_ = lo;
    }
    const std::vector<LeafAnalysis> &an_;
    const uint64_t *ids_;
    size_t nchunks_ = 0;
    std::vector<std::vector<uint32_t>> part_;  // per chunk: leaves per bucket
    std::vector<uint16_t> bucket_;             // per leaf
    std::vector<uint32_t> hist_;
    std::vector<Key> keys_;
    double total_ = 0.0;
    size_t top_;  // buckets at or above it are in keys_
};

// Decide actions: -1 keep, 0 double, 1 + j split along j, for the leaves in
// ranking order until their contributions reach refine_fraction of the total.
// Returns the number of ranks examined; the refined leaves are among them.
size_t decide(std::vector<LeafAnalysis> &an, const SplitStats &st, const uint64_t *ids,
              const uint64_t *n, const bfi_adaptive_config &cfg, int32_t *action, Ranking &order)
{
    const size_t count = an.size();
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
        if (an[s].e <= 0.0 && i > 0)
            break;
        taken += an[s].e;
    }
    parallel_range(i, size_t(1) << 10, [&](size_t k) {
        const size_t s = order[k];
        action[s] = leaf_action(an, st, s, ids[s], n[s], cfg);
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

struct LeafSet {
    int d = 0, nx = 0;
    GrowArray<uint64_t> id, n;
    // rec: all samples; split and base: split statistics and the record of the
    // samples they cover (the first split_samples of the leaf's stream)
    GrowArray<double> lo, hi, rec, split, base;
    GrowArray<double> vol;  // product of the extents, computed once per leaf
    size_t size() const { return id.size(); }
};

// Merge record b into a when both may be empty (count 0: nothing to add).
void merge_record(double *a, const double *b, int len, const std::vector<int> &first,
                  const std::vector<int> &second)
{
    if (b[0] == 0)
        return;
    if (a[0] == 0) {
        std::copy(b, b + len, a);
        return;
    }
    merge_shifted(a, b, 1, first, second, 0);
}

// The two resident evaluators of a run: the kernel variant with split
// statistics and the plain kernel, each with its buffers and captured graph
// kept from round to round.
struct Evaluators {
    ResidentEval with, without;
    double device_ms = 0.0;  // replay time of every list so far
};

// The record of all of an entry's samples from the records of its two parts
// (either may be absent).
void combine_parts(double *R, const double *with, const double *plain, int rec_len,
                   const std::vector<int> &first, const std::vector<int> &second)
{
    if (with)
        std::copy(with, with + rec_len, R);
    else
        std::fill(R, R + rec_len, 0.0);
    if (plain)
        merge_record(R, plain, rec_len, first, second);
}

// Copy len values, or zeros when src is absent.
void copy_or_zero(double *dst, const double *src, int len)
{
    if (src)
        std::copy(src, src + len, dst);
    else
        std::fill(dst, dst + len, 0.0);
}

constexpr size_t kGrain = 2048;  // entries per chunk of the parallel host loops

// Evaluate a work list on the device.  The samples below index `split_samples`
// of each stream (all of them when 0) go through the kernel variant with split
// statistics, the rest through the plain kernel.  Entry w's results go to
// sink(w, with, split, plain), called in parallel over the entries: the record
// and the split statistics of its samples below split_samples and the record of
// the rest, each NULL if the entry has no such samples, read where the replays
// left them (pinned host memory, valid until the next list).
template <class Sink>
bfi_status eval_list(Evaluators *ev, const bfi_lattice &lat, uint64_t seed, const SubList &work,
                     uint64_t split_samples, Sink &&sink)
{
    const int d = lat.nx * lat.nt, rec_len = BFI_PARTIAL_LEN(lat.nx), split_len = BFI_SPLIT_LEN(d);
    const size_t count = work.size();
    std::optional<TraceRange> stage_range(std::in_place, "adaptive: stage");
    // entry w's covered part [offset, min(end, P)) goes to the first list at
    // wpos[w], the rest to the second at opos[w] (-1: no such part)
    std::vector<int64_t> wpos(count, -1), opos(count, -1);
    std::vector<uint64_t> cut(count);
    int64_t nw = 0, no = 0;
    for (size_t w = 0; w < count; ++w) {
        const uint64_t off = work.offset[w], end = off + work.n[w];
        cut[w] = split_samples == 0 ? end : std::min(std::max(split_samples, off), end);
        if (cut[w] > off)
            wpos[w] = nw++;
        if (end > cut[w])
            opos[w] = no++;
    }
    BFI_TRY(ev->with.stage(static_cast<size_t>(nw)));
    BFI_TRY(ev->without.stage(static_cast<size_t>(no)));
    parallel_range(count, kGrain, [&](size_t w) {
        const uint64_t off = work.offset[w], end = off + work.n[w];
        const double *lo = &work.lo[w * d], *hi = &work.hi[w * d];
        if (wpos[w] >= 0)
            ev->with.set(static_cast<size_t>(wpos[w]), work.id[w], off, cut[w] - off, lo, hi);
        if (opos[w] >= 0)
            ev->without.set(static_cast<size_t>(opos[w]), work.id[w], cut[w], end - cut[w], lo, hi);
    });
    stage_range.reset();
    // both replays prepared, then queued back to back on the stream
    {
        TraceRange tr("adaptive: prepare and launch");
        if (nw > 0)
            BFI_TRY(ev->with.prepare(seed));
        if (no > 0)
            BFI_TRY(ev->without.prepare(seed));
        if (nw > 0)
            BFI_TRY(ev->with.launch());
        if (no > 0)
            BFI_TRY(ev->without.launch());
    }
    if (nw > 0) {
        TraceRange tr("adaptive: samples with split statistics");
        double ms = 0.0;
        BFI_TRY(ev->with.finish(nullptr, nullptr, &ms));
        ev->device_ms += ms;
    }
    if (no > 0) {
        TraceRange tr("adaptive: samples through the plain kernel");
        double ms = 0.0;
        BFI_TRY(ev->without.finish(nullptr, nullptr, &ms));
        ev->device_ms += ms;
    }
    const double *r_with = ev->with.records(), *sp_with = ev->with.split_records(),
                 *r_without = ev->without.records();
    TraceRange tr("adaptive: take the records");
    parallel_range(count, kGrain, [&](size_t w) {
        const size_t i = static_cast<size_t>(wpos[w]), o = static_cast<size_t>(opos[w]);
        sink(w, wpos[w] >= 0 ? &r_with[i * rec_len] : nullptr,
             wpos[w] >= 0 ? &sp_with[i * split_len] : nullptr,
             opos[w] >= 0 ? &r_without[o * rec_len] : nullptr);
    });
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
        const int rec_len = BFI_PARTIAL_LEN(nx), split_len = BFI_SPLIT_LEN(d);
        std::vector<int> rec_first, rec_second, split_first, split_second;
        record_fields(nx, &rec_first, &rec_second);
        for (int j = 0; j < d; ++j) {
            split_first.push_back(1 + j);
            split_second.push_back(1 + d + j);
        }

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
        L.rec.resize(L.size() * rec_len);
        L.split.resize(L.size() * split_len);
        L.base.resize(L.size() * rec_len);
        BFI_TRY(eval_list(&ev, *lat, seed, init, cfg->split_samples,
                          [&](size_t w, const double *with, const double *sp, const double *plain) {
                              combine_parts(&L.rec[w * rec_len], with, plain, rec_len, rec_first,
                                            rec_second);
                              copy_or_zero(&L.base[w * rec_len], with, rec_len);
                              copy_or_zero(&L.split[w * split_len], sp, split_len);
                          }));

        bfi_status status = BFI_OK;
        const double min_ess = cfg->min_ess > 0 ? cfg->min_ess : 100.0;
        int rounds = 0, checks = 0;
        bool holdout_used = false;
        uint64_t holdout_seed = 0;
        double holdout_err = 0.0;
        double run_target = cfg->target_rel_err;  // tightened by failed holdout checks
        bfi_result res{};
        std::vector<LeafAnalysis> an;
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
            BFI_TRY(analyse(nx, d, L.size(), L.lo.data(), L.hi.data(), L.rec.data(), &an, &res,
                            L.vol.data()));
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
                        BFI_TRY(ev.without.stage(L.size()));
                        parallel_range(L.size(), kGrain, [&](size_t s) {
                            ev.without.set(s, L.id[s], 0, L.n[s], &L.lo[s * d], &L.hi[s * d]);
                        });
                        double hms = 0.0;
                        BFI_TRY(ev.without.run(hseed, hrec.data(), nullptr, &hms));
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
            if (rounds >= cfg->max_rounds) {
                status = BFI_EBUDGET;
                break;
            }
            phase.next("adaptive: decide and plan");
            const SplitStats st{d, rec_len, L.split.data(), L.base.data()};
            action.resize(L.size());
            std::optional<TraceRange> sub(std::in_place, "adaptive: rank and decide");
            Ranking order(an, L.id.data());
            const size_t examined =
                decide(an, st, L.id.data(), L.n.data(), *cfg, action.data(), order);
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
            // planned count of a leaf with action `act` and n samples at factor f
            auto target_of = [&](int32_t act, uint64_t n, uint64_t f) {
                const uint64_t base =
                    act == 0 ? 2 * n : std::min(std::max(n, cfg->n_min), cfg->n_max);
                const uint64_t cap = std::max(cfg->n_max, base);
                return base > cap / f ? cap : std::max(base, std::min(base * f, cap));
            };
            auto cost_of = [](int32_t act, uint64_t n, uint64_t t) {
                return act == 0 ? t - n : 2 * t;
            };
            // whether the count would still grow at 2f
            auto grows_of = [&](int32_t act, uint64_t n, uint64_t f, uint64_t t) {
                return f <= std::numeric_limits<uint64_t>::max() / 2 &&
                       target_of(act, n, 2 * f) > t;
            };
            uint64_t f = 1, planned = 0;
            size_t growable = 0;
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
                        const uint64_t t = target_of(action[s], L.n[s], f);
                        target[s] = t;
                        p += cost_of(action[s], L.n[s], t);
                        g += grows_of(action[s], L.n[s], f, t);
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
            struct Candidate {
                size_t leaf;
                int32_t act;
                uint64_t n;
            };
            std::vector<Candidate> batch;
            size_t batch_lo = 0;
            auto candidate = [&](size_t rank) {
                if (rank < batch_lo || rank >= batch_lo + batch.size()) {
                    // a leaf adds at most 2 n_max samples (counts stay within n_max):
                    // the round needs at least this many more leaves
                    const uint64_t left = cfg->round_evals - planned;
                    const uint64_t need = cfg->n_max <= std::numeric_limits<uint64_t>::max() / 2
                                              ? left / (2 * cfg->n_max) + 1
                                              : 1;
                    const size_t len = static_cast<size_t>(std::min<uint64_t>(
                        order.size() - rank, std::max<uint64_t>(4096, need)));
                    for (size_t k = 0; k < len; ++k)
                        (void)order[rank + k];  // gather the ranks first (serial)
                    batch.resize(len);
                    batch_lo = rank;
                    parallel_range(len, size_t(1) << 9, [&](size_t k) {
                        const size_t s = order[rank + k];
                        batch[k] = Candidate{
                            s,
                            action[s] == -1 ? leaf_action(an, st, s, L.id[s], L.n[s], *cfg)
                                            : kHasAction,
                            L.n[s]};
                    });
                }
                return batch[rank - batch_lo];
            };
            while (cfg->round_evals > 0 && planned < cfg->round_evals) {
                if (growable > 0) {
                    f *= 2;
                    plan_all();
                    continue;
                }
                // only the leaf taken up here gets an action in this loop, so a
                // batch's view of which leaves have one stays current
                Candidate c{0, kHasAction, 0};
                while (next_leaf < order.size() && (c = candidate(next_leaf)).act == kHasAction)
                    ++next_leaf;
                if (next_leaf == order.size())
                    break;
                ++next_leaf;
                const size_t s = c.leaf;
                if (c.act < 0) {
                    action[s] = -2;  // neither split nor doubling possible: skip it
                    continue;
                }
                action[s] = c.act;
                refined.push_back(s);
                const uint64_t t = target_of(c.act, c.n, f);
                target[s] = t;
                planned += cost_of(c.act, c.n, t);
                growable += grows_of(c.act, c.n, f, t);
            }
            for (size_t i = 0; i < order.sorted(); ++i)
                if (action[order[i]] == -2)
                    action[order[i]] = -1;
            sub.reset();
            sub.emplace("adaptive: budget trim");
            // trim to the evaluation budget in priority order (every refined leaf
            // lies in the part of the ranking read so far)
            uint64_t cost = 0;
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
            size_t grown = L.size();
            for (size_t w = 0; w < origin.size(); ++w)
                dst[w] = origin[w].kind == 2 ? grown++ : origin[w].leaf;
            L.id.resize(grown);
            L.n.resize(grown);
            L.lo.resize(grown * d);
            L.hi.resize(grown * d);
            L.rec.resize(grown * rec_len);
            L.split.resize(grown * split_len);
            L.base.resize(grown * rec_len);
            L.vol.resize(grown);
            grow_range.reset();
            phase.next("adaptive: evaluate and fold");
            // the results go into the leaf set in place as each entry's records
            // are read; every entry has its own destination
            BFI_TRY(eval_list(
                &ev, *lat, seed, work, cfg->split_samples,
                [&](size_t w, const double *with, const double *sp, const double *plain) {
                    const size_t s = dst[w];
                    if (origin[w].kind == 0) {
                        double R[BFI_PARTIAL_LEN(BFI_MAX_NX)];
                        combine_parts(R, with, plain, rec_len, rec_first, rec_second);
                        merge_shifted(&L.rec[s * rec_len], R, 1, rec_first, rec_second, 0);
                        if (with && with[0] > 0) {
                            // the continuation still lies below split_samples
                            merge_shifted(&L.split[s * split_len], sp, 0, split_first,
                                          split_second, -1);
                            merge_shifted(&L.base[s * rec_len], with, 1, rec_first, rec_second,
                                          0);
                        }
                        L.n[s] = target[s];
                        return;
                    }
                    L.id[s] = work.id[w];
                    L.n[s] = work.n[w];
                    std::copy(&work.lo[w * d], &work.lo[w * d] + d, &L.lo[s * d]);
                    std::copy(&work.hi[w * d], &work.hi[w * d] + d, &L.hi[s * d]);
                    L.vol[s] = box_volume(&L.lo[s * d], &L.hi[s * d], d);
                    combine_parts(&L.rec[s * rec_len], with, plain, rec_len, rec_first,
                                  rec_second);
                    copy_or_zero(&L.split[s * split_len], sp, split_len);
                    copy_or_zero(&L.base[s * rec_len], with, rec_len);
                }));
            evals += cost;
            ++rounds;
        }

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
        const size_t m = std::min(cap, L.size());
        for (size_t s = 0; s < m; ++s) {
            if (leaf_id)
                leaf_id[s] = L.id[s];
            if (leaf_n)
                leaf_n[s] = L.n[s];
            if (leaf_offset)
                leaf_offset[s] = 0;
            if (leaf_lo)
                std::memcpy(leaf_lo + s * d, &L.lo[s * d], d * sizeof(double));
            if (leaf_hi)
                std::memcpy(leaf_hi + s * d, &L.hi[s * d], d * sizeof(double));
        }
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
        std::vector<LeafAnalysis> an;
        bfi_result res;
        BFI_TRY(analyse(lat->nx, d, leaves->count, leaves->lo, leaves->hi, partials, &an, &res));
        const SplitStats st{d, BFI_PARTIAL_LEN(lat->nx), split, split_base ? split_base : partials};
        Ranking order(an, leaves->id);
        decide(an, st, leaves->id, leaves->n, *cfg, action, order);
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
