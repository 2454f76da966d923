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
#include <cstring>
#include <limits>
#include <numeric>

#include "runtime.h"

using namespace bfi;

namespace {

constexpr double kSplitGain = 0.9;

struct LeafAnalysis {
    double e = 0.0;        // contribution to the variance of C
    int best_dim = 0;      // j*
    double gain = 1.0;     // (sigma_L + sigma_U)(j*) / (2 sigma)
};

// Scale factors that move every record to the smallest shift of the list.
std::vector<double> common_shift_factors(size_t count, const double *partials, int rec_len)
{
    double sig = std::numeric_limits<double>::infinity();
    for (size_t s = 0; s < count; ++s)
        sig = std::min(sig, partials[s * rec_len + 1]);
    std::vector<double> f(count);
    for (size_t s = 0; s < count; ++s)
        f[s] = std::exp(sig - partials[s * rec_len + 1]);
    return f;
}

// Contribution of every leaf to the variance of C, and the estimate itself.
bfi_status analyse(int nx, int d, size_t count, const double *lo, const double *hi,
                   const double *partials, std::vector<LeafAnalysis> *out, bfi_result *res)
{
    const int rec_len = BFI_PARTIAL_LEN(nx);
    BFI_TRY(finalize_records(nx, d, count, lo, hi, partials, res));
    const std::vector<double> f = common_shift_factors(count, partials, rec_len);
    // Z in the common shift
    double z = 0.0;
    std::vector<double> V(count);
    for (size_t s = 0; s < count; ++s) {
        double vol = 1.0;
        for (int k = 0; k < d; ++k)
            vol *= hi[s * d + k] - lo[s * d + k];
        V[s] = vol;
        z += vol * f[s] * partials[s * rec_len + 2] / partials[s * rec_len];
    }
    out->assign(count, LeafAnalysis{});
    for (size_t s = 0; s < count; ++s) {
        const double *rec = partials + s * rec_len;
        const double n = rec[0], nn = n * (n - 1.0), v2 = V[s] * V[s];
        const double a = f[s], a2 = a * a;
        const double sw = a * rec[2], sw2 = a2 * rec[3];
        const double var_z = v2 * (sw2 - sw * sw / n) / nn;
        double e = 0.0;
        for (int r = 0; r < nx; ++r) {
            const double C = res->C[r];
            const double spw = a * rec[4 + r], spw2 = a2 * rec[4 + nx + r],
                         spww = a2 * rec[4 + 2 * nx + r];
            const double var_n = v2 * (spw2 - spw * spw / n) / nn;
            const double cov = v2 * (spww - spw * sw / n) / nn;
            e += var_n - 2.0 * C * cov + C * C * var_z;
        }
        (*out)[s].e = z > 0 ? std::max(e, 0.0) / (z * z) : 0.0;
    }
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

// Decide actions: -1 keep, 0 double, 1 + j split along j.
// Decide actions: -1 keep, 0 double, 1 + j split along j.  *order gets the
// leaves in ranking order (descending e, ties by lower id).
void decide(std::vector<LeafAnalysis> &an, const SplitStats &st, const uint64_t *ids,
            const uint64_t *n, const bfi_adaptive_config &cfg, int32_t *action,
            std::vector<size_t> *order)
{
    const size_t count = an.size();
    order->resize(count);
    std::iota(order->begin(), order->end(), 0);
    std::sort(order->begin(), order->end(), [&](size_t x, size_t y) {
        if (an[x].e != an[y].e)
            return an[x].e > an[y].e;
        return ids[x] < ids[y];
    });
    double total = 0.0;
    for (const auto &a : an)
        total += a.e;
    std::fill(action, action + count, -1);
    double taken = 0.0;
    for (size_t i = 0; i < count; ++i) {
        const size_t s = (*order)[i];
        if (i > 0 && taken >= cfg.refine_fraction * total)
            break;
        if (an[s].e <= 0.0 && i > 0)
            break;
        taken += an[s].e;
        action[s] = leaf_action(an, st, s, ids[s], n[s], cfg);
    }
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

struct LeafSet {
    int d = 0, nx = 0;
    std::vector<uint64_t> id, n;
    // rec: all samples; split and base: split statistics and the record of the
    // samples they cover (the first split_samples of the leaf's stream)
    std::vector<double> lo, hi, rec, split, base;
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

// Evaluate a work list on the device.  The samples below index `split_samples`
// of each stream (all of them when 0) go through the kernel variant with split
// statistics, the rest through the plain kernel.  Per entry: rec covers all its
// samples, base and split the ones with statistics (count 0 and zeros if none).
bfi_status eval_list(bfi_context *ctx, const bfi_lattice &lat, int prec, uint64_t seed,
                     const SubList &work, uint64_t split_samples, const bfi_launch *launch,
                     std::vector<double> *rec, std::vector<double> *split,
                     std::vector<double> *base)
{
    const int d = lat.nx * lat.nt, rec_len = BFI_PARTIAL_LEN(lat.nx), split_len = BFI_SPLIT_LEN(d);
    const size_t count = work.size();
    rec->assign(count * rec_len, 0.0);
    split->assign(count * split_len, 0.0);
    base->assign(count * rec_len, 0.0);
    // the two lists: entry w's covered part [offset, min(end, P)) and the rest
    SubList with, without;
    with.d = without.d = d;
    std::vector<size_t> with_of, without_of;
    for (size_t w = 0; w < count; ++w) {
        const uint64_t off = work.offset[w], end = off + work.n[w];
        const uint64_t cut = split_samples == 0 ? end : std::min(std::max(split_samples, off), end);
        const uint64_t parts[2][2] = {{off, cut}, {cut, end}};
        for (int k = 0; k < 2; ++k) {
            if (parts[k][1] <= parts[k][0])
                continue;
            SubList &dst = k == 0 ? with : without;
            (k == 0 ? with_of : without_of).push_back(w);
            dst.id.push_back(work.id[w]);
            dst.offset.push_back(parts[k][0]);
            dst.n.push_back(parts[k][1] - parts[k][0]);
            dst.lo.insert(dst.lo.end(), &work.lo[w * d], &work.lo[w * d] + d);
            dst.hi.insert(dst.hi.end(), &work.hi[w * d], &work.hi[w * d] + d);
        }
    }
    std::vector<int> first, second;
    record_fields(lat.nx, &first, &second);
    if (with.size() > 0) {
        TraceRange tr("adaptive: samples with split statistics");
        std::vector<double> r(with.size() * rec_len), sp(with.size() * split_len);
        bfi_subvolumes v = with.view();
        BFI_TRY(bfi_eval(ctx, &lat, static_cast<bfi_precision>(prec), seed, &v, launch, r.data(),
                         sp.data()));
        for (size_t i = 0; i < with.size(); ++i) {
            const size_t w = with_of[i];
            std::copy(&r[i * rec_len], &r[i * rec_len] + rec_len, &(*base)[w * rec_len]);
            std::copy(&r[i * rec_len], &r[i * rec_len] + rec_len, &(*rec)[w * rec_len]);
            std::copy(&sp[i * split_len], &sp[i * split_len] + split_len, &(*split)[w * split_len]);
        }
    }
    if (without.size() > 0) {
        TraceRange tr("adaptive: samples through the plain kernel");
        std::vector<double> r(without.size() * rec_len);
        bfi_subvolumes v = without.view();
        BFI_TRY(bfi_eval(ctx, &lat, static_cast<bfi_precision>(prec), seed, &v, launch, r.data(),
                         nullptr));
        for (size_t i = 0; i < without.size(); ++i)
            merge_record(&(*rec)[without_of[i] * rec_len], &r[i * rec_len], rec_len, first, second);
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
        L.id = init.id;
        L.n = init.n;
        L.lo = init.lo;
        L.hi = init.hi;
        BFI_TRY(eval_list(ctx, *lat, prec, seed, init, cfg->split_samples, launch, &L.rec,
                          &L.split, &L.base));

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
        for (;;) {
            TracePhases phase("adaptive: analyse");
            BFI_TRY(analyse(nx, d, L.size(), L.lo.data(), L.hi.data(), L.rec.data(), &an, &res));
            report(rel_err(res));
            // stop check; with holdout, a failed check tightens the running target
            // and is retried on the same leaves only while the running estimate
            // still meets it
            bool stop = false;
            while (!stop && rel_err(res) <= run_target && res.ess >= min_ess) {
                if (!cfg->holdout) {
                    stop = true;
                    break;
                }
                phase.next("adaptive: holdout pass");
                // holdout check: the same leaves, samples drawn afresh under a
                // seed of their own, so no refinement decision has seen them
                uint64_t cost = 0;
                for (uint64_t n : L.n)
                    cost += n;
                if (cost > cfg->max_evals - evals) {
                    status = BFI_EBUDGET;
                    stop = true;
                    break;
                }
                ++checks;
                const uint64_t hseed = seed + static_cast<uint64_t>(checks) * 0x9E3779B97F4A7C15ull;
                SubList fresh;
                fresh.d = d;
                fresh.id = L.id;
                fresh.n = L.n;
                fresh.offset.assign(L.size(), 0);
                fresh.lo = L.lo;
                fresh.hi = L.hi;
                std::vector<double> hrec(L.size() * rec_len);
                bfi_subvolumes v = fresh.view();
                BFI_TRY(bfi_eval(ctx, lat, prec, hseed, &v, launch, hrec.data(), nullptr));
                evals += cost;
                bfi_result hres{};
                BFI_TRY(finalize_records(nx, d, L.size(), L.lo.data(), L.hi.data(), hrec.data(),
                                         &hres));
                const double herr = rel_err(hres);
                holdout_err = herr;
                report(rel_err(res));
                if (herr <= cfg->target_rel_err && hres.ess >= min_ess) {
                    res = hres;
                    holdout_used = true;
                    holdout_seed = hseed;
                    stop = true;
                    break;
                }
                // the running estimate was optimistic: ask more of it
                run_target *= std::min(0.5, cfg->target_rel_err / herr);
            }
            if (stop)
                break;
            if (rounds >= cfg->max_rounds) {
                status = BFI_EBUDGET;
                break;
            }
            phase.next("adaptive: decide and plan");
            const SplitStats st{d, rec_len, L.split.data(), L.base.data()};
            std::vector<int32_t> action(L.size());
            std::vector<size_t> order;
            decide(an, st, L.id.data(), L.n.data(), *cfg, action.data(), &order);

            // planned sample counts: children clamp(n, n_min, n_max) each, doubled
            // leaves 2n; scaled by a power of two up to the round's work floor
            // planned count of a refined leaf at scale factor f (within n_max):
            // children clamp(n, n_min, n_max) each, doubled leaves 2n, times f
            std::vector<uint64_t> target(L.size(), 0);  // new per-leaf (or per-child) count
            auto leaf_target = [&](size_t s, uint64_t f) {
                const uint64_t base = action[s] == 0 ? 2 * L.n[s]
                                                      : std::min(std::max(L.n[s], cfg->n_min),
                                                                 cfg->n_max);
                const uint64_t cap = std::max(cfg->n_max, base);
                return base > cap / f ? cap : std::max(base, std::min(base * f, cap));
            };
            auto leaf_cost = [&](size_t s) {
                return action[s] == 0 ? target[s] - L.n[s] : 2 * target[s];
            };
            // refined leaves whose count would still grow at 2f
            auto grows = [&](size_t s, uint64_t f) {
                return f <= std::numeric_limits<uint64_t>::max() / 2 &&
                       leaf_target(s, 2 * f) > target[s];
            };
            uint64_t f = 1, planned = 0;
            size_t growable = 0;
            auto plan_all = [&]() {
                planned = 0;
                growable = 0;
                for (size_t s = 0; s < L.size(); ++s) {
                    if (action[s] < 0)
                        continue;
                    target[s] = leaf_target(s, f);
                    planned += leaf_cost(s);
                    growable += grows(s, f);
                }
            };
            plan_all();
            // work floor: scale the refined leaves by powers of two; once n_max caps
            // them all, refine further leaves in variance order (each at the current
            // factor; the next pass doubles again if one of them can still grow)
            size_t next_leaf = 0;
            while (cfg->round_evals > 0 && planned < cfg->round_evals) {
                if (growable > 0) {
                    f *= 2;
                    plan_all();
                    continue;
                }
                while (next_leaf < order.size() && action[order[next_leaf]] != -1)
                    ++next_leaf;
                if (next_leaf == order.size())
                    break;
                const size_t s = order[next_leaf];
                action[s] = leaf_action(an, st, s, L.id[s], L.n[s], *cfg);
                if (action[s] < 0) {
                    action[s] = -2;  // neither split nor doubling possible: skip it
                    continue;
                }
                target[s] = leaf_target(s, f);
                planned += leaf_cost(s);
                growable += grows(s, f);
            }
            for (auto &a : action)
                if (a == -2)
                    a = -1;
            // trim to the evaluation budget in priority order
            uint64_t cost = 0;
            for (size_t s : order) {
                if (action[s] < 0)
                    continue;
                const uint64_t c = action[s] == 0 ? target[s] - L.n[s] : 2 * target[s];
                if (evals + cost + c > cfg->max_evals)
                    action[s] = -1;
                else
                    cost += c;
            }
            if (cost == 0) {
                status = BFI_EBUDGET;
                break;
            }

            // work list: children (fresh streams) and continuations
            SubList work;
            work.d = d;
            struct Origin {
                size_t leaf;
                int kind;  // 0 continuation, 1 lower child, 2 upper child
            };
            std::vector<Origin> origin;
            for (size_t s = 0; s < L.size(); ++s) {
                if (action[s] < 0)
                    continue;
                const double *lo = &L.lo[s * d], *hi = &L.hi[s * d];
                if (action[s] == 0) {
                    work.id.push_back(L.id[s]);
                    work.n.push_back(target[s] - L.n[s]);
                    work.offset.push_back(L.n[s]);
                    work.lo.insert(work.lo.end(), lo, lo + d);
                    work.hi.insert(work.hi.end(), hi, hi + d);
                    origin.push_back({s, 0});
                    continue;
                }
                const int j = action[s] - 1;
                const double mid = 0.5 * (lo[j] + hi[j]);
                const uint64_t child_n = target[s];
                for (int half = 0; half < 2; ++half) {
                    work.id.push_back(2 * L.id[s] + half);
                    work.n.push_back(child_n);
                    work.offset.push_back(0);
                    work.lo.insert(work.lo.end(), lo, lo + d);
                    work.hi.insert(work.hi.end(), hi, hi + d);
                    if (half == 0)
                        work.hi[(work.id.size() - 1) * d + j] = mid;
                    else
                        work.lo[(work.id.size() - 1) * d + j] = mid;
                    origin.push_back({s, 1 + half});
                }
            }
            phase.next("adaptive: evaluate");
            std::vector<double> wrec, wsplit, wbase;
            BFI_TRY(eval_list(ctx, *lat, prec, seed, work, cfg->split_samples, launch, &wrec,
                              &wsplit, &wbase));
            evals += cost;

            phase.next("adaptive: fold");
            // fold the results into the leaf set in place: a doubled leaf merges
            // its continuation, a split leaf becomes its lower child and its upper
            // child is appended (work proportional to the round's work list)
            size_t uppers = 0;
            for (const Origin &o : origin)
                uppers += o.kind == 2;
            const size_t grown = L.size() + uppers;
            L.id.reserve(grown);
            L.n.reserve(grown);
            L.lo.reserve(grown * d);
            L.hi.reserve(grown * d);
            L.rec.reserve(grown * rec_len);
            L.split.reserve(grown * split_len);
            L.base.reserve(grown * rec_len);
            for (size_t w = 0; w < origin.size(); ++w) {
                const size_t s = origin[w].leaf;
                const double *wr = &wrec[w * rec_len], *ws = &wsplit[w * split_len],
                             *wb = &wbase[w * rec_len];
                if (origin[w].kind == 0) {
                    merge_shifted(&L.rec[s * rec_len], wr, 1, rec_first, rec_second, 0);
                    if (wb[0] > 0) {
                        // the continuation still lies below split_samples
                        merge_shifted(&L.split[s * split_len], ws, 0, split_first, split_second,
                                      -1);
                        merge_shifted(&L.base[s * rec_len], wb, 1, rec_first, rec_second, 0);
                    }
                    L.n[s] = target[s];
                } else if (origin[w].kind == 1) {
                    L.id[s] = work.id[w];
                    L.n[s] = work.n[w];
                    std::copy(&work.lo[w * d], &work.lo[w * d] + d, &L.lo[s * d]);
                    std::copy(&work.hi[w * d], &work.hi[w * d] + d, &L.hi[s * d]);
                    std::copy(wr, wr + rec_len, &L.rec[s * rec_len]);
                    std::copy(ws, ws + split_len, &L.split[s * split_len]);
                    std::copy(wb, wb + rec_len, &L.base[s * rec_len]);
                } else {
                    L.id.push_back(work.id[w]);
                    L.n.push_back(work.n[w]);
                    L.lo.insert(L.lo.end(), &work.lo[w * d], &work.lo[w * d] + d);
                    L.hi.insert(L.hi.end(), &work.hi[w * d], &work.hi[w * d] + d);
                    L.rec.insert(L.rec.end(), wr, wr + rec_len);
                    L.split.insert(L.split.end(), ws, ws + split_len);
                    L.base.insert(L.base.end(), wb, wb + rec_len);
                }
            }
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
        std::vector<size_t> order;
        decide(an, st, leaves->id, leaves->n, *cfg, action, &order);
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
