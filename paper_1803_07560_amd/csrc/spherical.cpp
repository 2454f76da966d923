// Monte Carlo in spherical coordinates over the cube [-B, B]^d (the paper's
// discussion proposes switching from cartesian to spherical coordinates to
// concentrate resolution on the shell about the origin where the subdivision
// gathers): the cube is cut into radial shells, each shell is sampled
// uniformly in its volume by sph_kernels.hip, and a shell's integral is its
// volume pi^(d/2) / Gamma(d/2 + 1) (rho_hi^d - rho_lo^d) times the mean weight.
//
// Entry points: per-shell records (bfi_sph_eval), their finalize with shell
// volumes (bfi_sph_finalize), a two-stage integrator over equal-width shells
// out to the cube's corners (bfi_integrate_sph: a pilot pass, then the rest of
// the budget allocated to the shells in proportion to volume times the pilot's
// spread of the weight, Neyman's allocation, each shell continuing its own
// stream), and the test hook bfi_debug_sph_points.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "runtime.h"

using namespace bfi;

namespace {

struct DevMem {
    void *p = nullptr;
    ~DevMem()
    {
        if (p)
            (void)hipFree(p);
    }
};

bfi_status check_common(const bfi_lattice *lat, int prec, double box)
{
    BFI_TRY(check_lattice(lat));
    if (lat->antithetic)
        return fail(BFI_EUNSUPPORTED, "the spherical sampler draws single points");
    if (lat->nx * lat->nt > kSphMaxD)
        return fail(BFI_EUNSUPPORTED, "the spherical sampler is compiled for d <= %d", kSphMaxD);
    if (prec == BFI_FP64_SHIFTED)
        return fail(BFI_EUNSUPPORTED, "the spherical sampler has no shifted FP64 form");
    if (!known_precision(prec))
        return fail(BFI_EINVAL, "unknown precision %d", prec);
    if (!(box > 0.0) || !std::isfinite(box))
        return fail(BFI_EINVAL, "box must be positive and finite");
    return BFI_OK;
}

bfi_status check_shells(int d, const bfi_shells *sh)
{
    if (!sh)
        return fail(BFI_EINVAL, "shell list is NULL");
    if (sh->count == 0)
        return BFI_OK;
    if (sh->count > 0xFFFFFFFFull)
        return fail(BFI_EINVAL, "too many shells");
    if (!sh->id || !sh->rho_lo || !sh->rho_hi || !sh->n || !sh->offset)
        return fail(BFI_EINVAL, "shell arrays must be non-NULL");
    const unsigned blocks = static_cast<unsigned>((2 * ((d + 1) / 2) + 1 + 3) / 4);
    const unsigned __int128 index_end = (static_cast<unsigned __int128>(1) << 64) / blocks;
    for (size_t s = 0; s < sh->count; ++s) {
        const double lo = sh->rho_lo[s], hi = sh->rho_hi[s];
        if (!(lo >= 0.0) || !(hi > lo) || !std::isfinite(hi))
            return fail(BFI_EINVAL, "shell %zu: need 0 <= rho_lo < rho_hi, finite", s);
        if (sh->n[s] < 2)
            return fail(BFI_EINVAL, "shell %zu: n < 2", s);
        if (static_cast<unsigned __int128>(sh->offset[s]) + sh->n[s] > index_end)
            return fail(BFI_EINVAL, "shell %zu: sample indices overflow the Philox counter", s);
    }
    return BFI_OK;
}

// (rho_lo / rho_hi)^d, the shell's inner radius in the radius law
double inner_ratio(int d, double lo, double hi) { return std::pow(lo / hi, static_cast<double>(d)); }

double shell_volume(int d, double lo, double hi)
{
    // unit-ball volume pi^(d/2) / Gamma(d/2 + 1), taken through logarithms
    const double log_unit = 0.5 * d * std::log(M_PI) - std::lgamma(0.5 * d + 1.0);
    return std::exp(log_unit + d * std::log(hi)) * (1.0 - inner_ratio(d, lo, hi));
}

bfi_launch sph_launch(const bfi_launch *req)
{
    bfi_launch l{256, 256, 1, 0};
    if (req) {
        if (req->samples_per_thread > 0)
            l.samples_per_thread = req->samples_per_thread;
        if (req->block > 0)
            l.block = req->block;
        if (req->persistent >= 0)
            l.persistent = req->persistent != 0;
    }
    return l;
}

bfi_status sph_eval(bfi_context *ctx, const bfi_lattice &lat, int prec, uint64_t seed, double box,
                    const bfi_shells &sh, const bfi_launch *launch, double *partials)
{
    const int d = lat.nx * lat.nt, rec_len = BFI_PARTIAL_LEN(lat.nx);
    const size_t ns = sh.count;
    const bfi_launch l = sph_launch(launch);
    if (l.block != 64 && l.block != 128 && l.block != 256)
        return fail(BFI_EINVAL, "block must be 64, 128 or 256 (got %d)", l.block);
    if (l.samples_per_thread < 1 || l.samples_per_thread > (1 << 20))
        return fail(BFI_EINVAL, "samples_per_thread out of range");
    const uint64_t chunk = static_cast<uint64_t>(l.samples_per_thread) * l.block;
    std::vector<WorkItem> items;
    std::vector<uint32_t> first(ns + 1);
    for (size_t s = 0; s < ns; ++s) {
        first[s] = static_cast<uint32_t>(items.size());
        for (uint64_t start = 0; start < sh.n[s]; start += chunk) {
            items.push_back(WorkItem{nullptr, nullptr, start, static_cast<uint32_t>(s),
                                     static_cast<uint32_t>(std::min(chunk, sh.n[s] - start))});
            if (items.size() > 0x7FFFFFFFull)
                return fail(BFI_EINVAL, "more than 2^31 work items; raise samples_per_thread");
        }
    }
    first[ns] = static_cast<uint32_t>(items.size());
    std::vector<double> shell64(2 * ns);
    std::vector<float> shell32(2 * ns);
    for (size_t s = 0; s < ns; ++s) {
        shell64[2 * s] = sh.rho_hi[s];
        shell64[2 * s + 1] = inner_ratio(d, sh.rho_lo[s], sh.rho_hi[s]);
        shell32[2 * s] = static_cast<float>(shell64[2 * s]);
        shell32[2 * s + 1] = static_cast<float>(shell64[2 * s + 1]);
    }

    // one device block: parameters, ids, offsets, shells, items, records, head
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    size_t at = 0;
    auto take = [&](size_t bytes) {
        const size_t here = at;
        at = al(at + bytes);
        return here;
    };
    const size_t o_params = take(sizeof(EvalParams)), o_ids = take(ns * 8), o_off = take(ns * 8),
                 o_s64 = take(ns * 16), o_s32 = take(ns * 8),
                 o_items = take(items.size() * sizeof(WorkItem)), o_first = take((ns + 1) * 4),
                 o_irec = take(items.size() * rec_len * 8), o_srec = take(ns * rec_len * 8),
                 o_head = take(4);
    DevMem mem;
    BFI_HIP(hipMalloc(&mem.p, at));
    char *base = static_cast<char *>(mem.p);
    auto *params = reinterpret_cast<EvalParams *>(base + o_params);
    const EvalParams P{nullptr, nullptr, nullptr, nullptr,
                       reinterpret_cast<const uint64_t *>(base + o_ids),
                       reinterpret_cast<const uint64_t *>(base + o_off), make_coef(lat),
                       static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32)};
    for (size_t i = 0; i < items.size(); ++i) {
        items[i].params = params;
        items[i].rec = reinterpret_cast<double *>(base + o_irec) + i * rec_len;
    }
    hipStream_t st = ctx->stream;
    BFI_HIP(hipMemcpyAsync(params, &P, sizeof(P), hipMemcpyHostToDevice, st));
    BFI_HIP(hipMemcpyAsync(base + o_ids, sh.id, ns * 8, hipMemcpyHostToDevice, st));
    BFI_HIP(hipMemcpyAsync(base + o_off, sh.offset, ns * 8, hipMemcpyHostToDevice, st));
    BFI_HIP(hipMemcpyAsync(base + o_s64, shell64.data(), ns * 16, hipMemcpyHostToDevice, st));
    BFI_HIP(hipMemcpyAsync(base + o_s32, shell32.data(), ns * 8, hipMemcpyHostToDevice, st));
    BFI_HIP(hipMemcpyAsync(base + o_items, items.data(), items.size() * sizeof(WorkItem),
                           hipMemcpyHostToDevice, st));
    BFI_HIP(hipMemcpyAsync(base + o_first, first.data(), (ns + 1) * 4, hipMemcpyHostToDevice, st));

    LaunchSpec spec{prec, l.block, 0, l.persistent, 0, lat.observable, 0};
    auto *head = reinterpret_cast<uint32_t *>(base + o_head);
    if (l.persistent) {
        KernelInfo info{};
        BFI_HIP(sph_kernel_info(lat.nx, lat.nt, spec, &info));
        spec.grid = static_cast<uint32_t>(std::min<uint64_t>(
            static_cast<uint64_t>(std::max(info.blocks_per_cu, 1)) * std::max(ctx->cu_count, 1),
            items.size()));
        BFI_HIP(launch_reset_head(head, st));
    } else {
        spec.grid = static_cast<uint32_t>(items.size());
    }
    SphArgs a{};
    a.mc.items = reinterpret_cast<const WorkItem *>(base + o_items);
    a.mc.item_split = nullptr;
    a.mc.queue_head = l.persistent ? head : nullptr;
    a.mc.nitems = static_cast<uint32_t>(items.size());
    a.mc.samples_per_thread = static_cast<uint32_t>(l.samples_per_thread);
    a.shell64 = reinterpret_cast<const double *>(base + o_s64);
    a.shell32 = reinterpret_cast<const float *>(base + o_s32);
    a.box64 = box;
    a.box32 = static_cast<float>(box);
    BFI_HIP(launch_sph(lat.nx, lat.nt, spec, a, st));
    MergeArgs m{};
    m.item_rec = reinterpret_cast<const double *>(base + o_irec);
    m.sub_first = reinterpret_cast<const uint32_t *>(base + o_first);
    m.sub_rec = reinterpret_cast<double *>(base + o_srec);
    m.nsub = static_cast<uint32_t>(ns);
    m.nx = lat.nx;
    m.d = d;
    BFI_HIP(launch_merge(m, st));
    BFI_HIP(hipMemcpyAsync(partials, base + o_srec, ns * rec_len * 8, hipMemcpyDeviceToHost, st));
    BFI_HIP(hipStreamSynchronize(st));
    return BFI_OK;
}

bfi_status sph_finalize(const bfi_lattice &lat, const bfi_shells &sh, const double *partials,
                        bfi_result *out)
{
    const int d = lat.nx * lat.nt;
    std::vector<double> vol(sh.count);
    for (size_t s = 0; s < sh.count; ++s)
        vol[s] = shell_volume(d, sh.rho_lo[s], sh.rho_hi[s]);
    return finalize_records(lat.nx, d, sh.count, nullptr, nullptr, partials, out, 1, nullptr,
                            vol.data());
}

}  // namespace

extern "C" {

bfi_status bfi_sph_eval(bfi_context *ctx, const bfi_lattice *lat, bfi_precision prec,
                        uint64_t seed, double box, const bfi_shells *shells,
                        const bfi_launch *launch, double *partials)
{
    return guarded([&]() -> bfi_status {
        TraceRange trace("bfi_sph_eval");
        if (!ctx || !partials)
            return fail(BFI_EINVAL, "context and partials must be non-NULL");
        BFI_TRY(check_common(lat, prec, box));
        BFI_TRY(check_shells(lat->nx * lat->nt, shells));
        if (shells->count == 0)
            return BFI_OK;
        BFI_HIP(hipSetDevice(ctx->device));
        return sph_eval(ctx, *lat, prec, seed, box, *shells, launch, partials);
    });
}

bfi_status bfi_sph_finalize(const bfi_lattice *lat, const bfi_shells *shells,
                            const double *partials, bfi_result *out)
{
    return guarded([&]() -> bfi_status {
        if (!lat || !partials || !out)
            return fail(BFI_EINVAL, "arguments must be non-NULL");
        if (lat->nx < 1 || lat->nt < 1 || lat->nx > BFI_MAX_NX || lat->nx * lat->nt > BFI_MAX_D)
            return fail(BFI_EINVAL, "lattice out of range");
        BFI_TRY(check_shells(lat->nx * lat->nt, shells));
        if (shells->count == 0)
            return fail(BFI_EINVAL, "no shells");
        return sph_finalize(*lat, *shells, partials, out);
    });
}

bfi_status bfi_integrate_sph(bfi_context *ctx, const bfi_lattice *lat, bfi_precision prec,
                             uint64_t seed, double box, int32_t nshells, uint64_t budget,
                             double pilot_fraction, const bfi_launch *launch, bfi_result *out)
{
    return guarded([&]() -> bfi_status {
        TraceRange trace("bfi_integrate_sph");
        if (!ctx || !out)
            return fail(BFI_EINVAL, "arguments must be non-NULL");
        BFI_TRY(check_common(lat, prec, box));
        if (nshells < 1 || nshells > (1 << 20))
            return fail(BFI_EINVAL, "nshells must be in [1, 2^20]");
        if (!(pilot_fraction > 0.0) || pilot_fraction > 1.0)
            return fail(BFI_EINVAL, "pilot_fraction must be in (0, 1]");
        const uint64_t pilot = static_cast<uint64_t>(pilot_fraction * static_cast<double>(budget)) /
                               static_cast<uint64_t>(nshells);
        if (pilot < 2)
            return fail(BFI_EINVAL, "the pilot pass needs at least 2 samples per shell");
        BFI_HIP(hipSetDevice(ctx->device));
        const int d = lat->nx * lat->nt, rec_len = BFI_PARTIAL_LEN(lat->nx);
        const size_t ns = static_cast<size_t>(nshells);
        // equal-width shells from the centre out to the cube's corners
        const double rmax = box * std::sqrt(static_cast<double>(d));
        std::vector<uint64_t> id(ns), n(ns, pilot), offset(ns, 0);
        std::vector<double> lo(ns), hi(ns);
        for (size_t s = 0; s < ns; ++s) {
            id[s] = s + 1;
            lo[s] = rmax * static_cast<double>(s) / static_cast<double>(ns);
            hi[s] = rmax * static_cast<double>(s + 1) / static_cast<double>(ns);
        }
        bfi_shells sh{ns, id.data(), lo.data(), hi.data(), n.data(), offset.data()};
        std::vector<double> rec(ns * rec_len);
        BFI_TRY(sph_eval(ctx, *lat, prec, seed, box, sh, launch, rec.data()));
        // Neyman allocation of the rest: n_s proportional to V_s times the spread
        // of the pilot's weights, in the pilot's common shift
        const uint64_t used = pilot * ns;
        const uint64_t rest = budget > used ? budget - used : 0;
        double sig = INFINITY;
        for (size_t s = 0; s < ns; ++s)
            sig = std::min(sig, rec[s * rec_len + 1]);
        std::vector<double> share(ns, 0.0);
        double total = 0.0;
        for (size_t s = 0; s < ns; ++s) {
            const double *r = &rec[s * rec_len];
            const double f = std::exp(sig - r[1]), m = r[0];
            const double mean = f * r[2] / m, sq = f * f * r[3] / m;
            share[s] = shell_volume(d, lo[s], hi[s]) * std::sqrt(std::max(sq - mean * mean, 0.0));
            total += share[s];
        }
        std::vector<uint64_t> main_n(ns, 0);
        for (size_t s = 0; s < ns; ++s) {
            const double frac = total > 0.0 ? share[s] / total : 1.0 / static_cast<double>(ns);
            main_n[s] = static_cast<uint64_t>(frac * static_cast<double>(rest));
        }
        // the second pass continues each shell's stream after its pilot samples
        std::vector<uint64_t> id2, n2, off2;
        std::vector<double> lo2, hi2;
        std::vector<size_t> which;
        for (size_t s = 0; s < ns; ++s) {
            if (main_n[s] < 2)
                continue;
            which.push_back(s);
            id2.push_back(id[s]);
            n2.push_back(main_n[s]);
            off2.push_back(pilot);
            lo2.push_back(lo[s]);
            hi2.push_back(hi[s]);
        }
        if (!which.empty()) {
            bfi_shells sh2{which.size(), id2.data(), lo2.data(), hi2.data(), n2.data(), off2.data()};
            std::vector<double> rec2(which.size() * rec_len);
            BFI_TRY(sph_eval(ctx, *lat, prec, seed, box, sh2, launch, rec2.data()));
            std::vector<double> acc(which.size() * rec_len);
            for (size_t k = 0; k < which.size(); ++k)
                std::copy(&rec[which[k] * rec_len], &rec[which[k] * rec_len] + rec_len,
                          &acc[k * rec_len]);
            BFI_TRY(bfi_partials_merge(lat->nx, which.size(), acc.data(), rec2.data()));
            for (size_t k = 0; k < which.size(); ++k) {
                std::copy(&acc[k * rec_len], &acc[k * rec_len] + rec_len, &rec[which[k] * rec_len]);
                n[which[k]] += main_n[which[k]];
            }
        }
        return sph_finalize(*lat, sh, rec.data(), out);
    });
}

bfi_status bfi_debug_sph_points(bfi_context *ctx, const bfi_lattice *lat, bfi_precision prec,
                                uint64_t seed, uint64_t id, double rho_lo, double rho_hi,
                                uint64_t n, const uint64_t *index, double *out)
{
    return guarded([&]() -> bfi_status {
        if (!ctx || (n && (!index || !out)))
            return fail(BFI_EINVAL, "arguments must be non-NULL");
        BFI_TRY(check_common(lat, prec, 1.0));
        if (!(rho_lo >= 0.0) || !(rho_hi > rho_lo) || !std::isfinite(rho_hi))
            return fail(BFI_EINVAL, "need 0 <= rho_lo < rho_hi, finite");
        if (n == 0)
            return BFI_OK;
        const int d = lat->nx * lat->nt;
        BFI_HIP(hipSetDevice(ctx->device));
        DevMem mi, mo;
        BFI_HIP(hipMalloc(&mi.p, n * 8));
        BFI_HIP(hipMalloc(&mo.p, n * d * 8));
        BFI_HIP(hipMemcpy(mi.p, index, n * 8, hipMemcpyHostToDevice));
        SphDebugArgs a{static_cast<const uint64_t *>(mi.p), static_cast<double *>(mo.p), n, id,
                       rho_hi, inner_ratio(d, rho_lo, rho_hi), static_cast<uint32_t>(seed),
                       static_cast<uint32_t>(seed >> 32), prec};
        BFI_HIP(launch_sph_debug(lat->nx, lat->nt, a, ctx->stream));
        BFI_HIP(hipStreamSynchronize(ctx->stream));
        BFI_HIP(hipMemcpy(out, mo.p, n * d * 8, hipMemcpyDeviceToHost));
        return BFI_OK;
    });
}

}  // extern "C"
