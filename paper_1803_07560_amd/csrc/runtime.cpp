// Host runtime and C ABI: contexts, resident plans (descriptors, work items,
// persistent queue, captured graphs), finalize, the uniform-split entry, test
// hooks and the launch-shape autotuner.
#include "runtime.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <limits>
#include <sstream>
#include <thread>


namespace bfi {

namespace {
// fixed buffer: setting an error allocates nothing (the allocation-free entry
// point reports its errors through it too)
thread_local char g_last_error[512];
}

bfi_status fail(bfi_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    std::memcpy(g_last_error, buf, sizeof(buf));
    return s;
}

bfi_status hip_fail(hipError_t e, const char *what)
{
    return fail(e == hipErrorOutOfMemory ? BFI_ENOMEM : BFI_EDEVICE, "%s: %s", what,
                hipGetErrorString(e));
}

void clear_error() { g_last_error[0] = 0; }

bool shape_compiled(int nx, int nt)
{
#define BFI_SHAPE_MATCH(NX, NT) \
    if (nx == NX && nt == NT)   \
        return true;
    BFI_SHAPES(BFI_SHAPE_MATCH)
#undef BFI_SHAPE_MATCH
    return false;
}

hipError_t launch_mc(int nx, int nt, const LaunchSpec &spec, const McArgs &args, hipStream_t st)
{
#define BFI_SHAPE_LAUNCH(NX, NT)                             \
    if (nx == NX && nt == NT)                                \
        return launch_mc_shape<NX, NT>(spec, args, st);
    BFI_SHAPES(BFI_SHAPE_LAUNCH)
#undef BFI_SHAPE_LAUNCH
    return hipErrorNotSupported;
}

hipError_t kernel_info(int nx, int nt, const LaunchSpec &spec, KernelInfo *info)
{
#define BFI_SHAPE_INFO(NX, NT)                               \
    if (nx == NX && nt == NT)                                \
        return kernel_info_shape<NX, NT>(spec, info);
    BFI_SHAPES(BFI_SHAPE_INFO)
#undef BFI_SHAPE_INFO
    return hipErrorNotSupported;
}

hipError_t launch_is(int nx, int nt, const LaunchSpec &spec, const IsArgs &args, hipStream_t st)
{
#define BFI_IS_LAUNCH(NX, NT)                                \
    if (nx == NX && nt == NT)                                \
        return launch_is_shape<NX, NT>(spec, args, st);
    BFI_SHAPES(BFI_IS_LAUNCH)
#undef BFI_IS_LAUNCH
    return hipErrorNotSupported;
}

hipError_t is_kernel_info(int nx, int nt, const LaunchSpec &spec, KernelInfo *info)
{
#define BFI_IS_INFO(NX, NT)                                  \
    if (nx == NX && nt == NT)                                \
        return is_kernel_info_shape<NX, NT>(spec, info);
    BFI_SHAPES(BFI_IS_INFO)
#undef BFI_IS_INFO
    return hipErrorNotSupported;
}

hipError_t launch_sph(int nx, int nt, const LaunchSpec &spec, const SphArgs &args, hipStream_t st)
{
#define BFI_SPH_LAUNCH(NX, NT)                               \
    if (nx == NX && nt == NT)                                \
        return launch_sph_shape<NX, NT>(spec, args, st);
    BFI_SHAPES(BFI_SPH_LAUNCH)
#undef BFI_SPH_LAUNCH
    return hipErrorNotSupported;
}

hipError_t sph_kernel_info(int nx, int nt, const LaunchSpec &spec, KernelInfo *info)
{
#define BFI_SPH_INFO(NX, NT)                                 \
    if (nx == NX && nt == NT)                                \
        return sph_kernel_info_shape<NX, NT>(spec, info);
    BFI_SHAPES(BFI_SPH_INFO)
#undef BFI_SPH_INFO
    return hipErrorNotSupported;
}

hipError_t launch_sph_debug(int nx, int nt, const SphDebugArgs &args, hipStream_t st)
{
#define BFI_SPH_DEBUG(NX, NT)                                \
    if (nx == NX && nt == NT)                                \
        return launch_sph_debug_shape<NX, NT>(args, st);
    BFI_SHAPES(BFI_SPH_DEBUG)
#undef BFI_SPH_DEBUG
    return hipErrorNotSupported;
}

hipError_t launch_is_debug(int nx, int nt, const IsDebugArgs &args, hipStream_t st)
{
#define BFI_IS_DEBUG(NX, NT)                                 \
    if (nx == NX && nt == NT)                                \
        return launch_is_debug_shape<NX, NT>(args, st);
    BFI_SHAPES(BFI_IS_DEBUG)
#undef BFI_IS_DEBUG
    return hipErrorNotSupported;
}

namespace {

hipError_t launch_debug_action(int nx, int nt, const DebugActionArgs &args, hipStream_t st)
{
#define BFI_SHAPE_DBG(NX, NT)                                \
    if (nx == NX && nt == NT)                                \
        return launch_debug_action_shape<NX, NT>(args, st);
    BFI_SHAPES(BFI_SHAPE_DBG)
#undef BFI_SHAPE_DBG
    return hipErrorNotSupported;
}

template <class T>
T *dev_alloc(size_t count, hipError_t *err)
{
    void *p = nullptr;
    *err = count ? hipMalloc(&p, count * sizeof(T)) : hipSuccess;
    return static_cast<T *>(p);
}

// Device buffers freed on scope exit (for the one-shot test hooks).
struct DevBuf {
    void *p = nullptr;
    ~DevBuf()
    {
        if (p)
            (void)hipFree(p);
    }
};

}  // namespace

bfi_status check_lattice(const bfi_lattice *lat)
{
    if (!lat)
        return fail(BFI_EINVAL, "lattice is NULL");
    if (lat->nx < 1 || lat->nt < 1 || lat->nx > BFI_MAX_NX ||
        static_cast<int64_t>(lat->nx) * lat->nt > BFI_MAX_D)
        return fail(BFI_EINVAL, "lattice %dx%d out of range", lat->nx, lat->nt);
    const double v[] = {lat->nu, lat->D, lat->a, lat->tau, lat->g, lat->m2};
    for (double x : v)
        if (!std::isfinite(x))
            return fail(BFI_EINVAL, "lattice parameters must be finite");
    if (!(lat->D > 0) || !(lat->a > 0) || !(lat->tau > 0))
        return fail(BFI_EINVAL, "D, a and tau must be positive");
    if (lat->m2 < 0)
        return fail(BFI_EINVAL, "m2 must be >= 0");
    if (lat->observable != BFI_OBS_ANCHOR && lat->observable != BFI_OBS_AVERAGED)
        return fail(BFI_EINVAL, "unknown observable %d", lat->observable);
    if (lat->antithetic != 0 && lat->antithetic != 1)
        return fail(BFI_EINVAL, "antithetic must be 0 or 1 (got %d)", lat->antithetic);
    if (!shape_compiled(lat->nx, lat->nt))
        return fail(BFI_EUNSUPPORTED, "lattice %dx%d has no compiled kernel", lat->nx, lat->nt);
    if (lat->antithetic && lat->nx * lat->nt > kMaxPairD)
        return fail(BFI_EUNSUPPORTED, "antithetic pairs are compiled for d <= %d", kMaxPairD);
    return BFI_OK;
}

bfi_status check_subvolumes(const bfi_lattice *lat, const bfi_subvolumes *subs)
{
    if (!subs)
        return fail(BFI_EINVAL, "subvolume list is NULL");
    if (subs->count == 0)
        return BFI_OK;
    if (!subs->id || !subs->lo || !subs->hi || !subs->n || !subs->offset)
        return fail(BFI_EINVAL, "subvolume arrays must be non-NULL");
    const int d = lat->nx * lat->nt;
    // the Philox counter index * ceil(d/4) + j of the last sample must fit in
    // 64 bits: offset + n <= floor(2^64 / ceil(d/4))
    const unsigned __int128 index_end = (static_cast<unsigned __int128>(1) << 64) /
                                        static_cast<unsigned>((d + 3) / 4);
    for (size_t s = 0; s < subs->count; ++s) {
        if (subs->n[s] < 2)
            return fail(BFI_EINVAL, "subvolume %zu: n = %llu < 2", s,
                        static_cast<unsigned long long>(subs->n[s]));
        if (static_cast<unsigned __int128>(subs->offset[s]) + subs->n[s] > index_end)
            return fail(BFI_EINVAL, "subvolume %zu: sample indices overflow the Philox counter", s);
        for (int k = 0; k < d; ++k) {
            const double lo = subs->lo[s * d + k], hi = subs->hi[s * d + k];
            if (!std::isfinite(lo) || !std::isfinite(hi) || !(lo < hi))
                return fail(BFI_EINVAL, "subvolume %zu dim %d: need finite lo < hi", s, k);
        }
    }
    return BFI_OK;
}

ActionCoef make_coef(const bfi_lattice &lat)
{
    ActionCoef c;
    c.c_adv = lat.g * lat.tau / (2.0 * lat.a);
    c.c_visc = lat.nu * lat.tau / (lat.a * lat.a);
    c.k_diag = 2.0 * c.c_visc - 1.0;
    c.inv_2Dtau = 1.0 / (2.0 * lat.D * lat.tau);
    c.half_m2 = 0.5 * lat.m2;
    return c;
}

SubList SubList::copy_of(const bfi_subvolumes &s, int d)
{
    SubList out;
    out.d = d;
    out.id.assign(s.id, s.id + s.count);
    out.n.assign(s.n, s.n + s.count);
    out.offset.assign(s.offset, s.offset + s.count);
    out.lo.assign(s.lo, s.lo + s.count * d);
    out.hi.assign(s.hi, s.hi + s.count * d);
    return out;
}

SubList uniform_split(int d, const double *box_lo, const double *box_hi, int k, uint64_t budget)
{
    SubList out;
    out.d = d;
    const uint64_t count = uint64_t(1) << k;
    out.id.resize(count);
    out.n.resize(count);
    out.offset.assign(count, 0);
    out.lo.resize(count * d);
    out.hi.resize(count * d);
    const uint64_t base = budget / count, extra = budget % count;
    for (uint64_t b = 0; b < count; ++b) {
        out.id[b] = count + b;
        out.n[b] = base + (b < extra ? 1 : 0);
        double *lo = &out.lo[b * d], *hi = &out.hi[b * d];
        std::copy(box_lo, box_lo + d, lo);
        std::copy(box_hi, box_hi + d, hi);
        for (int t = 0; t < k; ++t) {
            const int dim = t % d;
            const double mid = 0.5 * (lo[dim] + hi[dim]);
            if ((b >> (k - 1 - t)) & 1)
                lo[dim] = mid;
            else
                hi[dim] = mid;
        }
    }
    return out;
}

bfi_launch resolve_launch(const bfi_context *ctx, const bfi_lattice &lat, int prec, bool split,
                          const bfi_launch *req)
{
    // defaults: 256-thread blocks, 64 samples per thread, persistent queue
    bfi_launch l{64, 256, 1, 0};
    if (ctx) {
        // the kernel variant's own entry (pairs, observable), else the entry of
        // the same sampler with the anchored product, else the single-point one
        // (the shifted FP64 form, untuned, takes the FP64 form's entries: the same
        // arithmetic and registers plus one shift)
        const int pairs = lat.antithetic ? 1 : 0;
        auto it = ctx->tuned.end();
        for (int p : {prec, prec == kFP64Shifted ? int(kFP64) : prec}) {
            if (it == ctx->tuned.end())
                it = ctx->tuned.find(TuneKey{lat.nx, lat.nt, p, pairs, lat.observable});
            if (it == ctx->tuned.end())
                it = ctx->tuned.find(TuneKey{lat.nx, lat.nt, p, pairs, 0});
            if (it == ctx->tuned.end())
                it = ctx->tuned.find(TuneKey{lat.nx, lat.nt, p, 0, 0});
        }
        if (it != ctx->tuned.end())
            l = it->second.launch;
    }
    if (req) {
        if (req->samples_per_thread > 0)
            l.samples_per_thread = req->samples_per_thread;
        if (req->block > 0)
            l.block = req->block;
        if (req->persistent >= 0)
            l.persistent = req->persistent != 0;
        l.use_graph = req->use_graph != 0;
    }
    l.use_graph = l.use_graph != 0;
    if (split)
        l.block = 256;
    return l;
}

namespace {

// Neumaier-compensated sum.
struct Nm {
    double s = 0, c = 0;
    void add(double x)
    {
        const double t = s + x;
        c += std::fabs(s) >= std::fabs(x) ? (s - t) + x : (x - t) + s;
        s = t;
    }
    void add(const Nm &o)
    {
        add(o.s);
        add(o.c);
    }
    double v() const { return s + c; }
};

constexpr size_t kFinalizeChunk = 8192;  // leaves per chunk of the per-leaf sums

}  // namespace

bfi_status finalize_records(int nx, int d, size_t nsub, const double *lo, const double *hi,
                            const double *partials, bfi_result *out, int evals_per_sample,
                            double *leaf_var, const double *volumes)
{
    if (!out)
        return fail(BFI_EINVAL, "result is NULL");
    std::memset(out, 0, sizeof(*out));
    out->nx = nx;
    if (nsub == 0)
        return fail(BFI_EINVAL, "no subvolumes");
    const int rec_len = BFI_PARTIAL_LEN(nx);
    const size_t nchunks = (nsub + kFinalizeChunk - 1) / kFinalizeChunk;
    // common shift: the smallest sigma of the subvolumes; and the first
    // subvolume with fewer than two samples, if any (per chunk, then in order)
    struct Scan {
        double sig;
        size_t bad;
    };
    std::vector<Scan> scan(nchunks);
    for_chunks(nchunks, [&](size_t c) {
        Scan sc{std::numeric_limits<double>::infinity(), nsub};
        const size_t s1 = std::min(nsub, (c + 1) * kFinalizeChunk);
        for (size_t s = c * kFinalizeChunk; s < s1; ++s) {
            sc.sig = std::min(sc.sig, partials[s * rec_len + 1]);
            if (!(partials[s * rec_len] >= 2.0) && sc.bad == nsub)
                sc.bad = s;
        }
        scan[c] = sc;
    });
    double sig = std::numeric_limits<double>::infinity();
    for (const Scan &sc : scan) {
        if (sc.bad < nsub)
            return fail(BFI_EINVAL, "subvolume %zu has n = %g < 2", sc.bad,
                        partials[sc.bad * rec_len]);
        sig = std::min(sig, sc.sig);
    }
    if (!std::isfinite(sig))
        return fail(BFI_EINVAL, "partial records carry no finite shift");

    // Two passes over the records, every distance r in the same pass; per-leaf
    // terms summed in fixed chunks of leaves, the chunk sums in chunk order.
    // per-subvolume volumes and shift factors; the buffers stay with the thread,
    // so repeated finalizes of large lists (adaptive rounds) reuse their pages
    // (plain pointers below: the chunks run on worker threads, where the names
    // would denote those threads' own, empty buffers)
    thread_local std::vector<double> V_buf, f1_buf;
    if (V_buf.size() < nsub) {
        V_buf.resize(nsub);
        f1_buf.resize(nsub);
    }
    double *const V = V_buf.data(), *const f1 = f1_buf.data();
    struct First {
        Nm Z, varZ, wsq, nev;
        std::vector<Nm> N;
    };
    std::vector<First> first(nchunks);
    for_chunks(nchunks, [&](size_t c) {
        First &acc = first[c];
        acc.N.assign(nx, Nm{});
        const size_t s1 = std::min(nsub, (c + 1) * kFinalizeChunk);
        for (size_t s = c * kFinalizeChunk; s < s1; ++s) {
            const double *rec = partials + s * rec_len;
            double vol = 1.0;
            if (volumes) {
                vol = volumes[s];
            } else {
                for (int k = 0; k < d; ++k)
                    vol *= hi[s * d + k] - lo[s * d + k];
            }
            V[s] = vol;
            const double n = rec[0];
            const double a = std::exp(sig - rec[1]);
            f1[s] = a;
            const double sw = a * rec[2], sw2 = a * a * rec[3];
            acc.Z.add(vol * sw / n);
            acc.varZ.add(vol * vol * (sw2 - sw * sw / n) / (n * (n - 1.0)));
            acc.wsq.add((vol / n) * (vol / n) * sw2);
            acc.nev.add(n);
            for (int r = 0; r < nx; ++r)
                acc.N[r].add(vol * a * rec[4 + r] / n);
        }
    });
    Nm Z, varZ, wsq, nev;
    std::vector<Nm> N(nx);
    for (const First &acc : first) {
        Z.add(acc.Z);
        varZ.add(acc.varZ);
        wsq.add(acc.wsq);
        nev.add(acc.nev);
        for (int r = 0; r < nx; ++r)
            N[r].add(acc.N[r]);
    }
    const double z = Z.v();  // Z exp(sigma)
    out->log_Z = std::log(z) - sig;
    out->Z = std::exp(out->log_Z);
    out->Z_err = std::sqrt(std::max(varZ.v(), 0.0)) * std::exp(-sig);
    out->ess = wsq.v() > 0 ? z * z / wsq.v() : 0.0;
    out->n_evals = nev.v() * evals_per_sample;
    std::vector<double> C(nx);
    for (int r = 0; r < nx; ++r)
        C[r] = N[r].v() / z;

    // delta method: per leaf Var N - 2 C Cov + C^2 Var Z for every r
    std::vector<std::vector<Nm>> second(nchunks);
    const double inv_z2 = z > 0 ? 1.0 / (z * z) : 0.0;
    for_chunks(nchunks, [&](size_t c) {
        std::vector<Nm> &var = second[c];
        var.assign(nx, Nm{});
        const size_t s1 = std::min(nsub, (c + 1) * kFinalizeChunk);
        for (size_t s = c * kFinalizeChunk; s < s1; ++s) {
            const double *rec = partials + s * rec_len;
            const double n = rec[0], v2 = V[s] * V[s], nn = n * (n - 1.0);
            const double a = f1[s], a2 = a * a;
            const double sw = a * rec[2], sw2 = a2 * rec[3];
            const double var_z = v2 * (sw2 - sw * sw / n) / nn;
            double e = 0.0;
            for (int r = 0; r < nx; ++r) {
                const double spw = a * rec[4 + r], spw2 = a2 * rec[4 + nx + r],
                             spww = a2 * rec[4 + 2 * nx + r];
                const double var_n = v2 * (spw2 - spw * spw / n) / nn;
                const double cov = v2 * (spww - spw * sw / n) / nn;
                const double t = var_n - 2.0 * C[r] * cov + C[r] * C[r] * var_z;
                var[r].add(t);
                e += t;
            }
            if (leaf_var)
                leaf_var[s] = std::max(e, 0.0) * inv_z2;
        }
    });
    for (int r = 0; r < nx; ++r) {
        Nm var;
        for (const auto &chunk : second)
            var.add(chunk[r]);
        out->C[r] = C[r];
        out->C_err[r] = std::sqrt(std::max(var.v(), 0.0)) / std::fabs(z);
    }
    return BFI_OK;
}

bfi_status plan_free(bfi_plan *p)
{
    if (!p)
        return BFI_OK;
    for (const bfi_plan::Replay &r : p->replays) {
        (void)hipGraphExecDestroy(r.exec);
        (void)hipGraphDestroy(r.def);
    }
    if (p->ev_start)
        (void)hipEventDestroy(p->ev_start);
    if (p->ev_stop)
        (void)hipEventDestroy(p->ev_stop);
    void *bufs[] = {p->d_base64, p->d_scale64, p->d_base32, p->d_scale32, p->d_ids,
                    p->d_offsets, p->d_params, p->d_items, p->d_item_rec, p->d_item_split, p->d_sub_first,
                    p->d_sub_rec, p->d_sub_split, p->d_head, p->d_is_table};
    for (void *b : bufs)
        if (b)
            (void)hipFree(b);
    delete p;
    return BFI_OK;
}

namespace {

bfi_status plan_build_core(bfi_context *ctx, int kind, const bfi_lattice &lat, int d, int nx,
                           int prec, const SubList &subs, const bfi_launch *launch, bool split,
                           bfi_plan **out);

}  // namespace

bfi_status plan_build(bfi_context *ctx, const bfi_lattice &lat, int prec, const SubList &subs,
                      const bfi_launch *launch, bool split, bfi_plan **out)
{
    return plan_build_core(ctx, 0, lat, lat.nx * lat.nt, lat.nx, prec, subs, launch, split, out);
}

bfi_status plan_build_nsphere(bfi_context *ctx, int dim, const SubList &subs,
                              const bfi_launch *launch, bfi_plan **out)
{
    if (dim < 1 || dim > kMaxNsphereDim)
        return fail(BFI_EINVAL, "N-sphere dimension must be in [1, %d]", kMaxNsphereDim);
    bfi_lattice none{};
    none.nx = 0;
    none.nt = 1;
    return plan_build_core(ctx, 1, none, dim, 0, kFP64, subs, launch, true, out);
}

bfi_status plan_build_is(bfi_context *ctx, const bfi_lattice &lat, int prec,
                         const SubList &streams, const IsTable &table, const bfi_launch *launch,
                         bfi_plan **out)
{
    if (lat.nx * lat.nt > kIsMaxD)
        return fail(BFI_EUNSUPPORTED, "the Gaussian-proposal sampler is compiled for d <= %d",
                    kIsMaxD);
    bfi_plan *p = nullptr;
    BFI_TRY(plan_build_core(ctx, 2, lat, lat.nx * lat.nt, lat.nx, prec, streams, launch, false,
                            &p));
    hipError_t e = hipMalloc(reinterpret_cast<void **>(&p->d_is_table), sizeof(IsTable));
    if (e == hipSuccess)
        e = hipMemcpy(p->d_is_table, &table, sizeof(IsTable), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        plan_free(p);
        return hip_fail(e, "sampler table upload");
    }
    *out = p;
    return BFI_OK;
}

namespace {

bfi_status plan_build_core(bfi_context *ctx, int kind, const bfi_lattice &lat, int d, int nx,
                           int prec, const SubList &subs, const bfi_launch *launch, bool split,
                           bfi_plan **out)
{
    if (kind == 0 && split && d > 32)
        return fail(BFI_EUNSUPPORTED, "split statistics need d <= 32 (d = %d)", d);
    if (subs.size() == 0)
        return fail(BFI_EINVAL, "empty subvolume list");
    if (subs.size() > 0xFFFFFFFFull)
        return fail(BFI_EINVAL, "too many subvolumes");
    // the tuned table holds mc_kernel shapes; the Gaussian-proposal sampler's
    // kernel (more work per sample) keeps 256 samples per thread and 256-thread
    // persistent blocks unless the caller asks otherwise
    bfi_launch l;
    if (kind == 0) {
        l = resolve_launch(ctx, lat, prec, split, launch);
    } else if (kind == 2) {
        const bfi_launch dflt{256, 256, 1, 0};
        bfi_launch want = dflt;
        if (launch) {
            if (launch->samples_per_thread > 0)
                want.samples_per_thread = launch->samples_per_thread;
            if (launch->block > 0)
                want.block = launch->block;
            if (launch->persistent >= 0)
                want.persistent = launch->persistent != 0;
            want.use_graph = launch->use_graph != 0;
        }
        l = resolve_launch(nullptr, lat, prec, split, &want);
    } else {
        l = resolve_launch(nullptr, lat, prec, true, launch);
    }
    if (!mc_block_ok(l.block))
        return fail(BFI_EINVAL, "block must be 64, 128, 256, 512 or 1024 (got %d)", l.block);
    if (kind == 2 && l.block > 256)
        return fail(BFI_EINVAL, "the Gaussian-proposal sampler takes blocks of 64, 128 or 256 "
                                "threads (got %d)", l.block);
    if (l.samples_per_thread < 1 || l.samples_per_thread > (1 << 20))
        return fail(BFI_EINVAL, "samples_per_thread out of range");
    const uint64_t chunk = static_cast<uint64_t>(l.samples_per_thread) * l.block;
    if (chunk > 0x7FFFFFFFull)
        return fail(BFI_EINVAL, "samples per work item exceed 2^31");

    // work items: ceil(n / chunk) per subvolume, subvolumes in list order
    std::vector<WorkItem> items;
    std::vector<uint32_t> first(subs.size() + 1, 0);
    uint64_t total_items = 0, n_evals = 0;
    for (size_t s = 0; s < subs.size(); ++s) {
        // checked per subvolume, so the running count cannot wrap
        total_items += subs.n[s] / chunk + (subs.n[s] % chunk != 0);
        if (total_items > 0x7FFFFFFFull)
            return fail(BFI_EINVAL, "more than 2^31 work items; raise samples_per_thread");
    }
    items.reserve(total_items);
    for (size_t s = 0; s < subs.size(); ++s) {
        first[s] = static_cast<uint32_t>(items.size());
        for (uint64_t start = 0; start < subs.n[s]; start += chunk) {
            const uint64_t cnt = std::min<uint64_t>(chunk, subs.n[s] - start);
            items.push_back(WorkItem{nullptr, nullptr, start, static_cast<uint32_t>(s),
                                     static_cast<uint32_t>(cnt)});
        }
        n_evals += subs.n[s];
    }
    if (lat.antithetic)
        n_evals *= 2;  // two points per sample index
    first[subs.size()] = static_cast<uint32_t>(items.size());

    // point map descriptors: scale = (hi - lo) 2^-32, base = lo + scale/2
    const size_t nd = subs.size() * d;
    std::vector<double> base64(nd), scale64(nd);
    std::vector<float> base32(nd), scale32(nd);
    for (size_t i = 0; i < nd; ++i) {
        scale64[i] = (subs.hi[i] - subs.lo[i]) * 0x1p-32;
        base64[i] = subs.lo[i] + 0.5 * scale64[i];
        scale32[i] = static_cast<float>(scale64[i]);
        base32[i] = static_cast<float>(base64[i]);
    }

    auto *p = new bfi_plan();
    p->ctx = ctx;
    p->kind = kind;
    p->lat = lat;
    p->prec = prec;
    p->d = d;
    p->nx = nx;
    p->rec_len = BFI_PARTIAL_LEN(nx);
    p->split = split;
    p->subs = subs;
    p->launch = l;
    p->nitems = static_cast<uint32_t>(items.size());
    p->n_evals = n_evals;

    hipError_t e = hipSuccess;
    auto cleanup_fail = [&](const char *what) {
        bfi_status st = hip_fail(e, what);
        plan_free(p);
        return st;
    };
#define BFI_ALLOC(field, T, count)                                  \
    do {                                                            \
        p->field = dev_alloc<T>((count), &e);                       \
        if (e != hipSuccess)                                        \
            return cleanup_fail("hipMalloc(" #field ")");           \
    } while (0)
    BFI_ALLOC(d_base64, double, nd);
    BFI_ALLOC(d_scale64, double, nd);
    BFI_ALLOC(d_base32, float, nd);
    BFI_ALLOC(d_scale32, float, nd);
    BFI_ALLOC(d_ids, uint64_t, subs.size());
    BFI_ALLOC(d_offsets, uint64_t, subs.size());
    BFI_ALLOC(d_params, EvalParams, 1);
    BFI_ALLOC(d_items, WorkItem, items.size());
    BFI_ALLOC(d_item_rec, double, items.size() * p->rec_len);
    BFI_ALLOC(d_sub_first, uint32_t, first.size());
    BFI_ALLOC(d_sub_rec, double, subs.size() * p->rec_len);
    BFI_ALLOC(d_head, uint32_t, 1);
    if (split) {
        BFI_ALLOC(d_item_split, double, items.size() * 2 * d);
        BFI_ALLOC(d_sub_split, double, subs.size() * BFI_SPLIT_LEN(d));
    }
#undef BFI_ALLOC
    for (size_t i = 0; i < items.size(); ++i) {
        items[i].params = p->d_params;
        items[i].rec = p->d_item_rec + i * p->rec_len;
    }
    p->params = EvalParams{p->d_base64, p->d_scale64, p->d_base32, p->d_scale32, p->d_ids,
                           p->d_offsets, kind != 1 ? make_coef(lat) : ActionCoef{}, 0u, 0u};
    struct Up {
        void *dst;
        const void *src;
        size_t bytes;
    } ups[] = {{p->d_base64, base64.data(), nd * 8}, {p->d_scale64, scale64.data(), nd * 8},
               {p->d_base32, base32.data(), nd * 4}, {p->d_scale32, scale32.data(), nd * 4},
               {p->d_ids, subs.id.data(), subs.size() * 8},
               {p->d_offsets, subs.offset.data(), subs.size() * 8},
               {p->d_items, items.data(), items.size() * sizeof(WorkItem)},
               {p->d_sub_first, first.data(), first.size() * 4},
               {p->d_params, &p->params, sizeof(EvalParams)}};
    for (const Up &u : ups) {
        e = hipMemcpy(u.dst, u.src, u.bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess)
            return cleanup_fail("hipMemcpy(plan upload)");
    }

    e = hipEventCreate(&p->ev_start);
    if (e == hipSuccess)
        e = hipEventCreate(&p->ev_stop);
    if (e != hipSuccess)
        return cleanup_fail("hipEventCreate");

    // persistent launches fill the chip once: resident blocks per CU x CUs
    if (l.persistent) {
        KernelInfo info{};
        if (kind == 0 || kind == 2) {
            LaunchSpec spec{prec, l.block, split ? 1 : 0, 1, 0, lat.observable,
                            lat.antithetic};
            e = kind == 0 ? kernel_info(lat.nx, lat.nt, spec, &info)
                          : is_kernel_info(lat.nx, lat.nt, spec, &info);
            if (e != hipSuccess)
                return cleanup_fail("kernel occupancy query");
        } else {
            info.blocks_per_cu = 4;  // 104 VGPRs: 4 waves per SIMD, one block per SIMD
        }
        const uint64_t resident = static_cast<uint64_t>(std::max(info.blocks_per_cu, 1)) *
                                  std::max(ctx->cu_count, 1);
        p->grid = static_cast<uint32_t>(std::min<uint64_t>(resident, items.size()));
    } else {
        p->grid = static_cast<uint32_t>(items.size());
    }
    *out = p;
    return BFI_OK;
}

}  // namespace

bfi_status plan_set_seed(bfi_plan *p, uint64_t seed)
{
    const uint32_t lo = static_cast<uint32_t>(seed), hi = static_cast<uint32_t>(seed >> 32);
    if (p->params.seed_lo == lo && p->params.seed_hi == hi)
        return BFI_OK;
    // kernels of earlier runs read the parameters from device memory
    if (p->last_stream)
        BFI_HIP(hipStreamSynchronize(p->last_stream));
    p->params.seed_lo = lo;
    p->params.seed_hi = hi;
    BFI_HIP(hipMemcpy(p->d_params, &p->params, sizeof(EvalParams), hipMemcpyHostToDevice));
    return BFI_OK;
}

bfi_status plan_enqueue(bfi_plan *p, uint64_t seed, double *dst, hipStream_t st, bool timed)
{
    BFI_TRY(plan_set_seed(p, seed));
    McArgs a{};
    a.items = p->d_items;
    a.item_split = p->d_item_split;
    a.queue_head = p->launch.persistent ? p->d_head : nullptr;
    a.nitems = p->nitems;
    a.samples_per_thread = static_cast<uint32_t>(p->launch.samples_per_thread);
    LaunchSpec spec{p->prec,  p->launch.block,    p->split ? 1 : 0, p->launch.persistent,
                    p->grid,  p->lat.observable, p->lat.antithetic};
    if (p->launch.persistent)
        BFI_HIP(launch_reset_head(p->d_head, st));
    if (timed)
        BFI_HIP(hipEventRecord(p->ev_start, st));
    if (p->kind == 1)
        BFI_HIP(launch_nsphere(NsphereArgs{a, p->d}, p->grid, st));
    else if (p->kind == 2)
        BFI_HIP(launch_is(p->lat.nx, p->lat.nt, spec, IsArgs{a, p->d_is_table}, st));
    else
        BFI_HIP(launch_mc(p->lat.nx, p->lat.nt, spec, a, st));
    if (timed)
        BFI_HIP(hipEventRecord(p->ev_stop, st));
    MergeArgs m{};
    m.item_rec = p->d_item_rec;
    m.item_split = p->d_item_split;
    m.sub_first = p->d_sub_first;
    m.sub_rec = p->d_sub_rec;
    m.sub_split = p->d_sub_split;
    m.nsub = static_cast<uint32_t>(p->subs.size());
    m.nx = p->nx;
    m.d = p->d;
    BFI_HIP(launch_merge(m, st));
    if (dst)
        BFI_HIP(hipMemcpyAsync(dst, p->d_sub_rec, p->subs.size() * p->rec_len * sizeof(double),
                               hipMemcpyDeviceToDevice, st));
    return BFI_OK;
}

}  // namespace bfi

using namespace bfi;

extern "C" {

const char *bfi_status_string(bfi_status s)
{
    // a C caller may pass any int: read it as one, not as the enumeration
    int32_t v = 0;
    std::memcpy(&v, &s, sizeof v < sizeof s ? sizeof v : sizeof s);
    switch (v) {
    case BFI_OK: return "ok";
    case BFI_EINVAL: return "invalid argument";
    case BFI_ENOMEM: return "out of memory";
    case BFI_EDEVICE: return "device error";
    case BFI_EUNSUPPORTED: return "unsupported";
    case BFI_EBUSY: return "busy";
    case BFI_ECANCELLED: return "cancelled";
    case BFI_EBUDGET: return "evaluation budget exhausted";
    case BFI_ENOTFOUND: return "unknown ticket";
    }
    return "unknown status";
}

const char *bfi_last_error(void) { return g_last_error; }

bfi_status bfi_shape_supported(int32_t nx, int32_t nt)
{
    return guarded([&]() -> bfi_status {
        return shape_compiled(nx, nt) ? BFI_OK : BFI_EUNSUPPORTED;
    });
}

bfi_status bfi_supported_shapes(int32_t *pairs, int32_t cap, int32_t *count)
{
    return guarded([&]() -> bfi_status {
        if (!count || (cap > 0 && !pairs))
            return fail(BFI_EINVAL, "bad arguments");
        int32_t n = 0;
    #define BFI_SHAPE_LIST(NX, NT)      \
        if (n < cap) {                  \
            pairs[2 * n] = NX;          \
            pairs[2 * n + 1] = NT;      \
        }                               \
        ++n;
        BFI_SHAPES(BFI_SHAPE_LIST)
    #undef BFI_SHAPE_LIST
        *count = n;
        return BFI_OK;
    });
}

bfi_status bfi_context_create(int32_t device, bfi_context **out)
{
    return guarded([&]() -> bfi_status {
        if (!out)
            return fail(BFI_EINVAL, "out is NULL");
        int ndev = 0;
        BFI_HIP(hipGetDeviceCount(&ndev));
        if (device < 0 || device >= ndev)
            return fail(BFI_EINVAL, "device %d out of range (%d devices)", device, ndev);
        BFI_HIP(hipSetDevice(device));
        hipDeviceProp_t prop;
        BFI_HIP(hipGetDeviceProperties(&prop, device));
        auto *ctx = new bfi_context();
        ctx->device = device;
        ctx->cu_count = prop.multiProcessorCount;
        ctx->arch = prop.gcnArchName;
        hipError_t e = hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete ctx;
            return hip_fail(e, "hipStreamCreateWithFlags");
        }
        // device address of the allocation-free entry point's scratch array
        const bfi_status st = noalloc_setup(device);
        if (st != BFI_OK) {
            (void)hipStreamDestroy(ctx->stream);
            delete ctx;
            return st;
        }
        *out = ctx;
        return BFI_OK;
    });
}

bfi_status bfi_context_destroy(bfi_context *ctx)
{
    return guarded([&]() -> bfi_status {
        if (!ctx)
            return BFI_OK;
        if (ctx->stream) {
            (void)hipStreamSynchronize(ctx->stream);
            (void)hipStreamDestroy(ctx->stream);
        }
        delete ctx;
        return BFI_OK;
    });
}

bfi_status bfi_plan_create(bfi_context *ctx, const bfi_lattice *lat, bfi_precision prec,
                           const bfi_subvolumes *subs, const bfi_launch *launch, bfi_plan **out)
{
    return guarded([&]() -> bfi_status {
        TraceRange trace("bfi_plan_create");
        if (!ctx || !out)
            return fail(BFI_EINVAL, "context and out must be non-NULL");
        if (!known_precision(prec))
            return fail(BFI_EINVAL, "unknown precision %d", static_cast<int>(prec));
        BFI_TRY(check_lattice(lat));
        BFI_TRY(check_subvolumes(lat, subs));
        BFI_HIP(hipSetDevice(ctx->device));
        return plan_build(ctx, *lat, prec, SubList::copy_of(*subs, lat->nx * lat->nt), launch, false,
                          out);
    });
}

bfi_status bfi_plan_run(bfi_plan *p, uint64_t seed, double *partials_dev, void *stream)
{
    return guarded([&]() -> bfi_status {
        TraceRange trace("bfi_plan_run");
        if (!p)
            return fail(BFI_EINVAL, "plan is NULL");
        BFI_HIP(hipSetDevice(p->ctx->device));
        hipStream_t st = stream ? static_cast<hipStream_t>(stream) : p->ctx->stream;
        if (p->launch.use_graph) {
            BFI_TRY(plan_set_seed(p, seed));
            // the replays are kept in order of last use: a hit moves to the back
            const bfi_plan::Replay *rp = nullptr;
            for (size_t i = 0; i < p->replays.size(); ++i) {
                if (p->replays[i].stream == st && p->replays[i].dst == partials_dev) {
                    const bfi_plan::Replay hit = p->replays[i];
                    p->replays.erase(p->replays.begin() + static_cast<std::ptrdiff_t>(i));
                    p->replays.push_back(hit);
                    rp = &p->replays.back();
                    break;
                }
            }
            if (!rp) {
                if (p->replays.size() >= bfi_plan::kMaxReplays) {
                    // drop the least recently used replay; the host waits for the
                    // plan's work on both streams before destroying it
                    if (p->last_stream)
                        BFI_HIP(hipStreamSynchronize(p->last_stream));
                    BFI_HIP(hipStreamSynchronize(p->replays.front().stream));
                    (void)hipGraphExecDestroy(p->replays.front().exec);
                    (void)hipGraphDestroy(p->replays.front().def);
                    p->replays.erase(p->replays.begin());
                }
                BFI_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
                bfi_status s = plan_enqueue(p, seed, partials_dev, st, false);
                hipGraph_t g = nullptr;
                hipError_t e = hipStreamEndCapture(st, &g);
                if (s != BFI_OK) {
                    if (g)
                        (void)hipGraphDestroy(g);
                    return s;
                }
                BFI_HIP(e);
                bfi_plan::Replay r;
                r.def = g;
                e = hipGraphInstantiate(&r.exec, g, nullptr, nullptr, 0);
                if (e != hipSuccess) {
                    (void)hipGraphDestroy(g);
                    return hip_fail(e, "hipGraphInstantiate");
                }
                r.stream = st;
                r.dst = partials_dev;
                p->replays.push_back(r);
                rp = &p->replays.back();
            }
            // a replay is timed as a whole: queue reset, kernel and merge
            BFI_HIP(hipEventRecord(p->ev_start, st));
            BFI_HIP(hipGraphLaunch(rp->exec, st));
            BFI_HIP(hipEventRecord(p->ev_stop, st));
        } else {
            BFI_TRY(plan_enqueue(p, seed, partials_dev, st, true));
        }
        p->last_stream = st;
        return BFI_OK;
    });
}

bfi_status bfi_plan_partials(bfi_plan *p, double *partials)
{
    return guarded([&]() -> bfi_status {
        if (!p || !partials)
            return fail(BFI_EINVAL, "plan and partials must be non-NULL");
        BFI_HIP(hipSetDevice(p->ctx->device));
        if (p->last_stream)
            BFI_HIP(hipStreamSynchronize(p->last_stream));
        BFI_HIP(hipMemcpy(partials, p->d_sub_rec, p->subs.size() * p->rec_len * sizeof(double),
                          hipMemcpyDeviceToHost));
        return BFI_OK;
    });
}

bfi_status bfi_plan_info(const bfi_plan *p, uint64_t *n_items, uint64_t *n_evals,
                         bfi_launch *resolved)
{
    return guarded([&]() -> bfi_status {
        if (!p)
            return fail(BFI_EINVAL, "plan is NULL");
        if (n_items)
            *n_items = p->nitems;
        if (n_evals)
            *n_evals = p->n_evals;
        if (resolved)
            *resolved = p->launch;
        return BFI_OK;
    });
}

bfi_status bfi_plan_kernel_ms(bfi_plan *p, double *ms)
{
    return guarded([&]() -> bfi_status {
        if (!p || !ms)
            return fail(BFI_EINVAL, "plan and ms must be non-NULL");
        if (!p->last_stream)
            return fail(BFI_EINVAL, "plan has not run");
        BFI_HIP(hipSetDevice(p->ctx->device));
        BFI_HIP(hipEventSynchronize(p->ev_stop));
        float f = 0.0f;
        BFI_HIP(hipEventElapsedTime(&f, p->ev_start, p->ev_stop));
        *ms = f;
        return BFI_OK;
    });
}

bfi_status bfi_plan_destroy(bfi_plan *p)
{
    return guarded([&]() -> bfi_status {
        if (p && p->ctx)
            (void)hipSetDevice(p->ctx->device);
        if (p && p->last_stream)
            (void)hipStreamSynchronize(p->last_stream);
        return plan_free(p);
    });
}

bfi_status bfi_eval(bfi_context *ctx, const bfi_lattice *lat, bfi_precision prec, uint64_t seed,
                    const bfi_subvolumes *subs, const bfi_launch *launch, double *partials,
                    double *split)
{
    return guarded([&]() -> bfi_status {
        TraceRange trace("bfi_eval");
        if (!ctx || !partials)
            return fail(BFI_EINVAL, "context and partials must be non-NULL");
        if (!known_precision(prec))
            return fail(BFI_EINVAL, "unknown precision %d", static_cast<int>(prec));
        BFI_TRY(check_lattice(lat));
        BFI_TRY(check_subvolumes(lat, subs));
        if (lat->antithetic && split)
            return fail(BFI_EUNSUPPORTED, "antithetic pairs have no split statistics");
        if (subs->count == 0)
            return BFI_OK;
        BFI_HIP(hipSetDevice(ctx->device));
        bfi_plan *p = nullptr;
        {
            TraceRange tb("bfi_eval: plan build and upload");
            BFI_TRY(plan_build(ctx, *lat, prec, SubList::copy_of(*subs, lat->nx * lat->nt), launch,
                               split != nullptr, &p));
        }
        bfi_launch l = p->launch;
        l.use_graph = 0;
        p->launch = l;
        bfi_status s = plan_enqueue(p, seed, nullptr, ctx->stream, true);
        p->last_stream = ctx->stream;
        if (s == BFI_OK)
            s = bfi_plan_partials(p, partials);
        if (s == BFI_OK && split) {
            hipError_t e = hipMemcpy(split, p->d_sub_split,
                                     subs->count * BFI_SPLIT_LEN(p->d) * sizeof(double),
                                     hipMemcpyDeviceToHost);
            if (e != hipSuccess)
                s = hip_fail(e, "hipMemcpy(split)");
        }
        plan_free(p);
        return s;
    });
}

bfi_status bfi_finalize(const bfi_lattice *lat, const bfi_subvolumes *subs,
                        const double *partials, bfi_result *out)
{
    return guarded([&]() -> bfi_status {
        if (!lat || !subs || !partials || !out)
            return fail(BFI_EINVAL, "arguments must be non-NULL");
        if (lat->nx < 1 || lat->nt < 1 || lat->nx > BFI_MAX_NX || lat->nx * lat->nt > BFI_MAX_D)
            return fail(BFI_EINVAL, "lattice out of range");
        if (subs->count && (!subs->lo || !subs->hi))
            return fail(BFI_EINVAL, "subvolume boxes must be non-NULL");
        if (lat->antithetic != 0 && lat->antithetic != 1)
            return fail(BFI_EINVAL, "antithetic must be 0 or 1 (got %d)", lat->antithetic);
        return finalize_records(lat->nx, lat->nx * lat->nt, subs->count, subs->lo, subs->hi,
                                partials, out, lat->antithetic ? 2 : 1);
    });
}

bfi_status bfi_integrate(bfi_context *ctx, const bfi_lattice *lat, bfi_precision prec,
                         uint64_t seed, const double *box_lo, const double *box_hi,
                         int32_t split_log2, uint64_t budget, const bfi_launch *launch,
                         bfi_result *out)
{
    return guarded([&]() -> bfi_status {
        TraceRange trace("bfi_integrate");
        if (!ctx || !box_lo || !box_hi || !out)
            return fail(BFI_EINVAL, "arguments must be non-NULL");
        BFI_TRY(check_lattice(lat));
        if (split_log2 < 0 || split_log2 > 24)
            return fail(BFI_EINVAL, "split_log2 must be in [0, 24]");
        const int d = lat->nx * lat->nt;
        for (int k = 0; k < d; ++k)
            if (!std::isfinite(box_lo[k]) || !std::isfinite(box_hi[k]) || !(box_lo[k] < box_hi[k]))
                return fail(BFI_EINVAL, "box dim %d: need finite lo < hi", k);
        // the budget counts integrand evaluations: two per antithetic pair
        const uint64_t per = lat->antithetic ? 2 : 1;
        if (budget / per < 2 * (uint64_t(1) << split_log2))
            return fail(BFI_EINVAL, "budget must give every subvolume at least 2 samples");
        SubList subs = uniform_split(d, box_lo, box_hi, split_log2, budget / per);
        std::vector<double> partials(subs.size() * BFI_PARTIAL_LEN(lat->nx));
        bfi_subvolumes v = subs.view();
        BFI_TRY(bfi_eval(ctx, lat, prec, seed, &v, launch, partials.data(), nullptr));
        return finalize_records(lat->nx, d, subs.size(), subs.lo.data(), subs.hi.data(),
                                partials.data(), out, static_cast<int>(per));
    });
}

bfi_status bfi_debug_points(bfi_context *ctx, int32_t d, bfi_precision prec, uint64_t seed,
                            uint64_t id, const double *lo, const double *hi,
                            const uint64_t *index, uint64_t n, double *out)
{
    return guarded([&]() -> bfi_status {
        if (!ctx || !lo || !hi || (n && (!index || !out)))
            return fail(BFI_EINVAL, "arguments must be non-NULL");
        if (d < 1 || d > BFI_MAX_D)
            return fail(BFI_EINVAL, "d out of range");
        if (!known_precision(prec))
            return fail(BFI_EINVAL, "unknown precision");
        for (int k = 0; k < d; ++k)
            if (!std::isfinite(lo[k]) || !std::isfinite(hi[k]) || !(lo[k] < hi[k]))
                return fail(BFI_EINVAL, "box dim %d: need finite lo < hi", k);
        if (n == 0)
            return BFI_OK;
        BFI_HIP(hipSetDevice(ctx->device));
        std::vector<double> b64(d), s64(d);
        std::vector<float> b32(d), s32(d);
        for (int k = 0; k < d; ++k) {
            s64[k] = (hi[k] - lo[k]) * 0x1p-32;
            b64[k] = lo[k] + 0.5 * s64[k];
            s32[k] = static_cast<float>(s64[k]);
            b32[k] = static_cast<float>(b64[k]);
        }
        DevBuf db64, ds64, db32, ds32, didx, dout;
        BFI_HIP(hipMalloc(&db64.p, d * 8));
        BFI_HIP(hipMalloc(&ds64.p, d * 8));
        BFI_HIP(hipMalloc(&db32.p, d * 4));
        BFI_HIP(hipMalloc(&ds32.p, d * 4));
        BFI_HIP(hipMalloc(&didx.p, n * 8));
        BFI_HIP(hipMalloc(&dout.p, n * d * 8));
        BFI_HIP(hipMemcpy(db64.p, b64.data(), d * 8, hipMemcpyHostToDevice));
        BFI_HIP(hipMemcpy(ds64.p, s64.data(), d * 8, hipMemcpyHostToDevice));
        BFI_HIP(hipMemcpy(db32.p, b32.data(), d * 4, hipMemcpyHostToDevice));
        BFI_HIP(hipMemcpy(ds32.p, s32.data(), d * 4, hipMemcpyHostToDevice));
        BFI_HIP(hipMemcpy(didx.p, index, n * 8, hipMemcpyHostToDevice));
        DebugPointArgs a{};
        a.base64 = static_cast<double *>(db64.p);
        a.scale64 = static_cast<double *>(ds64.p);
        a.base32 = static_cast<float *>(db32.p);
        a.scale32 = static_cast<float *>(ds32.p);
        a.index = static_cast<uint64_t *>(didx.p);
        a.out = static_cast<double *>(dout.p);
        a.id = id;
        a.n = n;
        a.seed_lo = static_cast<uint32_t>(seed);
        a.seed_hi = static_cast<uint32_t>(seed >> 32);
        a.d = d;
        a.prec = prec;
        BFI_HIP(launch_debug_points(a, ctx->stream));
        BFI_HIP(hipStreamSynchronize(ctx->stream));
        BFI_HIP(hipMemcpy(out, dout.p, n * d * 8, hipMemcpyDeviceToHost));
        return BFI_OK;
    });
}

bfi_status bfi_debug_action(bfi_context *ctx, const bfi_lattice *lat, bfi_precision prec,
                            uint64_t n, const double *points, double *out_S)
{
    return guarded([&]() -> bfi_status {
        if (!ctx || (n && (!points || !out_S)))
            return fail(BFI_EINVAL, "arguments must be non-NULL");
        if (!known_precision(prec))
            return fail(BFI_EINVAL, "unknown precision");
        BFI_TRY(check_lattice(lat));
        if (n == 0)
            return BFI_OK;
        BFI_HIP(hipSetDevice(ctx->device));
        const int d = lat->nx * lat->nt;
        DevBuf dp, ds;
        BFI_HIP(hipMalloc(&dp.p, n * d * 8));
        BFI_HIP(hipMalloc(&ds.p, n * 8));
        BFI_HIP(hipMemcpy(dp.p, points, n * d * 8, hipMemcpyHostToDevice));
        DebugActionArgs a{};
        a.points = static_cast<double *>(dp.p);
        a.out = static_cast<double *>(ds.p);
        a.n = n;
        a.coef = make_coef(*lat);
        a.prec = prec;
        BFI_HIP(launch_debug_action(lat->nx, lat->nt, a, ctx->stream));
        BFI_HIP(hipStreamSynchronize(ctx->stream));
        BFI_HIP(hipMemcpy(out_S, ds.p, n * 8, hipMemcpyDeviceToHost));
        return BFI_OK;
    });
}

}  // extern "C"
