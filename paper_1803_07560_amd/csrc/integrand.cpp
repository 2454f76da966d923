// Single integrands on the paper's integrand protocol and the paper's own
// subdivision policy (section 3: each subvolume is evaluated twice, the second
// time with a factor more samples, and split along the integrand's suggested
// dimension until one of three convergence criteria holds; section 4 gives the
// ranges of the criteria).  Evaluation runs on the same plans and kernels as
// the rest of the library; this file only turns records into (result, error,
// split dimension) and drives the generations.
#include <algorithm>
#include <cmath>
#include <limits>
#include <vector>

#include "runtime.h"

using namespace bfi;

namespace {

bfi_status check_integrand(const bfi_integrand *f, int *d)
{
    if (!f)
        return fail(BFI_EINVAL, "integrand is NULL");
    switch (f->kind) {
    case BFI_INTEGRAND_NSPHERE:
        if (f->dim < 1 || f->dim > kMaxNsphereDim)
            return fail(BFI_EINVAL, "N-sphere dimension must be in [1, %d]", kMaxNsphereDim);
        *d = f->dim;
        return BFI_OK;
    case BFI_INTEGRAND_BURGERS_Z:
    case BFI_INTEGRAND_BURGERS_N:
        BFI_TRY(check_lattice(&f->lat));
        if (f->lat.antithetic)
            return fail(BFI_EUNSUPPORTED, "the integrand protocol uses single points");
        if (!known_precision(f->prec))
            return fail(BFI_EINVAL, "unknown precision");
        *d = f->lat.nx * f->lat.nt;
        if (*d > 32)
            return fail(BFI_EUNSUPPORTED, "split suggestions need d <= 32");
        if (f->kind == BFI_INTEGRAND_BURGERS_N && (f->distance < 0 || f->distance >= f->lat.nx))
            return fail(BFI_EINVAL, "distance must be in [0, nx)");
        return BFI_OK;
    default:
        return fail(BFI_EINVAL, "unknown integrand kind %d", f->kind);
    }
}

// Records and split statistics of a subvolume list for an integrand.
bfi_status eval_records(bfi_context *ctx, const bfi_integrand &f, int d, uint64_t seed,
                        const SubList &subs, const bfi_launch *launch, std::vector<double> *rec,
                        std::vector<double> *split, int *rec_len)
{
    if (f.kind == BFI_INTEGRAND_NSPHERE) {
        bfi_plan *p = nullptr;
        BFI_TRY(plan_build_nsphere(ctx, d, subs, launch, &p));
        p->launch.use_graph = 0;
        *rec_len = p->rec_len;
        rec->assign(subs.size() * p->rec_len, 0.0);
        split->assign(subs.size() * BFI_SPLIT_LEN(d), 0.0);
        bfi_status s = plan_enqueue(p, seed, nullptr, ctx->stream, false);
        p->last_stream = ctx->stream;
        if (s == BFI_OK)
            s = bfi_plan_partials(p, rec->data());
        if (s == BFI_OK) {
            hipError_t e = hipMemcpy(split->data(), p->d_sub_split, split->size() * sizeof(double),
                                     hipMemcpyDeviceToHost);
            if (e != hipSuccess)
                s = hip_fail(e, "hipMemcpy(split)");
        }
        plan_free(p);
        return s;
    }
    *rec_len = BFI_PARTIAL_LEN(f.lat.nx);
    rec->assign(subs.size() * *rec_len, 0.0);
    split->assign(subs.size() * BFI_SPLIT_LEN(d), 0.0);
    bfi_subvolumes v = subs.view();
    return bfi_eval(ctx, &f.lat, static_cast<bfi_precision>(f.prec), seed, &v, launch, rec->data(),
                    split->data());
}

struct Estimate {
    double result, abserr;
    int32_t split_dim;
};

// Result V mean(f), error V s / sqrt(n), and the dimension minimising the sum
// of the two halves' standard deviations (each half holds n/2 samples in
// expectation); ties go to the lower dimension.
Estimate estimate(const bfi_integrand &f, int d, const double *lo, const double *hi,
                  const double *rec, const double *spl)
{
    double vol = 1.0;
    for (int k = 0; k < d; ++k)
        vol *= hi[k] - lo[k];
    const double n = rec[0], sigma = rec[1];
    const double e1 = std::exp(-sigma), e2 = e1 * e1;
    double s1, s2;
    if (f.kind == BFI_INTEGRAND_BURGERS_N) {
        const int nx = f.lat.nx, r = f.distance;
        s1 = rec[4 + r];
        s2 = rec[4 + nx + r];
    } else {
        s1 = rec[2];
        s2 = rec[3];
    }
    Estimate out;
    out.result = vol * e1 * s1 / n;
    const double var = std::max(s2 - s1 * s1 / n, 0.0) / (n - 1.0);
    out.abserr = vol * std::sqrt(e2 * var / n);
    // split suggestion from the statistics of the weight (f itself for N-sphere)
    const double S = rec[2], Q = rec[3], half = 0.5 * n;
    double best = std::numeric_limits<double>::infinity();
    out.split_dim = 0;
    for (int j = 0; j < d; ++j) {
        const double su = spl[1 + j], qu = spl[1 + d + j];
        const double sl = S - su, ql = Q - qu;
        const double vu = std::max(qu / half - (su / half) * (su / half), 0.0);
        const double vl = std::max(ql / half - (sl / half) * (sl / half), 0.0);
        const double sj = std::sqrt(vu) + std::sqrt(vl);
        if (sj < best) {
            best = sj;
            out.split_dim = j;
        }
    }
    return out;
}

bool converged(double r1, double r2, const bfi_hdi_config &c)
{
    const double diff = std::fabs(r2 - r1), big = std::max(std::fabs(r1), std::fabs(r2));
    if (c.rel_diff > 0 && diff <= (c.rel_diff - 1.0) * big)
        return true;
    if (c.abs_diff > 0 && diff <= c.abs_diff)
        return true;
    if (c.max_abs > 0 && big <= c.max_abs)
        return true;
    return false;
}

}  // namespace

extern "C" {

bfi_status bfi_integrand_eval(bfi_context *ctx, const bfi_integrand *f, uint64_t seed,
                              const bfi_subvolumes *subs, const bfi_launch *launch,
                              double *result, double *abserr, int32_t *split_dim)
{
    return guarded([&]() -> bfi_status {
        if (!ctx || !subs)
            return fail(BFI_EINVAL, "arguments must be non-NULL");
        int d = 0;
        BFI_TRY(check_integrand(f, &d));
        if (subs->count == 0)
            return BFI_OK;
        if (!result || !abserr || !split_dim)
            return fail(BFI_EINVAL, "output arrays must be non-NULL");
        bfi_lattice shape = f->lat;
        if (f->kind == BFI_INTEGRAND_NSPHERE) {
            shape.nx = d;  // only for the box checks
            shape.nt = 1;
        }
        BFI_TRY(check_subvolumes(&shape, subs));
        BFI_HIP(hipSetDevice(ctx->device));
        const SubList list = SubList::copy_of(*subs, d);
        std::vector<double> rec, spl;
        int rec_len = 0;
        BFI_TRY(eval_records(ctx, *f, d, seed, list, launch, &rec, &spl, &rec_len));
        for (size_t s = 0; s < list.size(); ++s) {
            const Estimate e = estimate(*f, d, &list.lo[s * d], &list.hi[s * d], &rec[s * rec_len],
                                        &spl[s * BFI_SPLIT_LEN(d)]);
            result[s] = e.result;
            abserr[s] = e.abserr;
            split_dim[s] = e.split_dim;
        }
        return BFI_OK;
    });
}

bfi_status bfi_integrate_hdi(bfi_context *ctx, const bfi_integrand *f, uint64_t seed,
                             const double *box_lo, const double *box_hi,
                             const bfi_hdi_config *cfg, const bfi_launch *launch, double *result,
                             double *abserr, bfi_hdi_stats *stats)
{
    return guarded([&]() -> bfi_status {
        if (!ctx || !box_lo || !box_hi || !cfg || !result || !abserr)
            return fail(BFI_EINVAL, "arguments must be non-NULL");
        int d = 0;
        BFI_TRY(check_integrand(f, &d));
        if (cfg->n_initial < 2 || !(cfg->sample_factor >= 1.0) || !std::isfinite(cfg->sample_factor))
            return fail(BFI_EINVAL, "need n_initial >= 2 and sample_factor >= 1");
        if (cfg->split_log2 < 0 || cfg->split_log2 > 24 || cfg->max_depth < 0 || cfg->max_depth > 60)
            return fail(BFI_EINVAL, "split_log2 in [0, 24] and max_depth in [0, 60]");
        for (int k = 0; k < d; ++k)
            if (!std::isfinite(box_lo[k]) || !std::isfinite(box_hi[k]) || !(box_lo[k] < box_hi[k]))
                return fail(BFI_EINVAL, "box dim %d: need finite lo < hi", k);
        BFI_HIP(hipSetDevice(ctx->device));
        const uint64_t n1 = cfg->n_initial;
        const uint64_t n2 = std::max<uint64_t>(
            2, static_cast<uint64_t>(std::llround(cfg->sample_factor * static_cast<double>(n1))));
        const uint64_t per_sub = n1 + n2;

        SubList open = uniform_split(d, box_lo, box_hi, cfg->split_log2, 0);
        std::vector<int> depth(open.size(), 0);
        if (open.size() * per_sub > cfg->max_evals)
            return fail(BFI_EINVAL, "the initial partition alone exceeds max_evals");

        double sum = 0.0, comp = 0.0, var = 0.0;
        uint64_t evals = 0, accepted = 0, unconverged = 0;
        int generations = 0, deepest = 0;
        bool budget_hit = false;
        while (open.size() > 0) {
            // both evaluations of every open subvolume in one batch: samples
            // [0, n1) and then [n1, n1 + n2) of its stream
            SubList work;
            work.d = d;
            for (int pass = 0; pass < 2; ++pass)
                for (size_t s = 0; s < open.size(); ++s) {
                    work.id.push_back(open.id[s]);
                    work.n.push_back(pass == 0 ? n1 : n2);
                    work.offset.push_back(pass == 0 ? 0 : n1);
                    work.lo.insert(work.lo.end(), &open.lo[s * d], &open.lo[s * d] + d);
                    work.hi.insert(work.hi.end(), &open.hi[s * d], &open.hi[s * d] + d);
                }
            std::vector<double> rec, spl;
            int rec_len = 0;
            BFI_TRY(eval_records(ctx, *f, d, seed, work, launch, &rec, &spl, &rec_len));
            evals += open.size() * per_sub;
            ++generations;

            SubList next;
            next.d = d;
            std::vector<int> next_depth;
            uint64_t reserved = 0;
            for (size_t s = 0; s < open.size(); ++s) {
                const size_t a = s, b = open.size() + s;
                const Estimate e1 = estimate(*f, d, &open.lo[s * d], &open.hi[s * d], &rec[a * rec_len],
                                             &spl[a * BFI_SPLIT_LEN(d)]);
                const Estimate e2 = estimate(*f, d, &open.lo[s * d], &open.hi[s * d], &rec[b * rec_len],
                                             &spl[b * BFI_SPLIT_LEN(d)]);
                const bool ok = converged(e1.result, e2.result, *cfg);
                const bool deep = depth[s] >= cfg->max_depth || open.id[s] >= (uint64_t(1) << 62);
                const bool affordable = evals + reserved + 2 * per_sub <= cfg->max_evals;
                if (ok || deep || !affordable) {
                    const double t = sum + e2.result;
                    comp += std::fabs(sum) >= std::fabs(e2.result) ? (sum - t) + e2.result
                                                                    : (e2.result - t) + sum;
                    sum = t;
                    var += e2.abserr * e2.abserr;
                    ++accepted;
                    deepest = std::max(deepest, depth[s]);
                    if (!ok) {
                        ++unconverged;
                        budget_hit = budget_hit || !affordable;
                    }
                    continue;
                }
                reserved += 2 * per_sub;
                const int j = e2.split_dim;
                const double mid = 0.5 * (open.lo[s * d + j] + open.hi[s * d + j]);
                for (int half = 0; half < 2; ++half) {
                    next.id.push_back(2 * open.id[s] + half);
                    next.n.push_back(0);
                    next.offset.push_back(0);
                    next.lo.insert(next.lo.end(), &open.lo[s * d], &open.lo[s * d] + d);
                    next.hi.insert(next.hi.end(), &open.hi[s * d], &open.hi[s * d] + d);
                    if (half == 0)
                        next.hi[(next.id.size() - 1) * d + j] = mid;
                    else
                        next.lo[(next.id.size() - 1) * d + j] = mid;
                    next_depth.push_back(depth[s] + 1);
                }
            }
            open = std::move(next);
            depth = std::move(next_depth);
        }
        *result = sum + comp;
        *abserr = std::sqrt(var);
        if (stats) {
            stats->evals = evals;
            stats->accepted = accepted;
            stats->unconverged = unconverged;
            stats->generations = generations;
            stats->depth = deepest;
        }
        if (budget_hit)
            return fail(BFI_EBUDGET, "%llu subvolumes accepted unconverged at the evaluation budget",
                        static_cast<unsigned long long>(unconverged));
        return BFI_OK;
    });
}

}  // extern "C"
