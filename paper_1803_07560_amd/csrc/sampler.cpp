// Gaussian-proposal importance sampling of exp(-S) over a cube (host side).
//
// Dropping the nonlinear term of Eq. Gen2 leaves the quadratic form
// S0 = u.P.u / 2, P = A^T A / (D tau) + m2 I, A = (T - 1) - (nu tau / a^2) L,
// which the real Fourier basis of the lattice diagonalises; its eigenvalue for
// mode j = bt*nx + bx (frequencies kt, kx; second-difference eigenvalues
// mt = 2 cos(2 pi kt / nt) - 2, mx = 2 cos(2 pi kx / nx) - 2) is
//     lambda_j = (-mt - c mt mx + c^2 mx^2) / (D tau) + m2,  c = nu tau / a^2.
// The proposal draws a_j = scale_j z_j with z_j standard normal and
// scale_j = min(1/sqrt(lambda_j), R), except the constant mode, uniform over
// [-R, R] when lambda_0 R^2 < 4 (R = the largest |u| in the cube).  A fraction
// alpha of every budget comes from it and the rest from the cube's uniform
// density (Hesterberg's defensive mixture); every sample weighs
//     W = K exp(-S) / (alpha exp(-sum z^2/2) + (1 - alpha) K / V),
//     K = (2R if mode 0 is uniform) * prod_gaussian sqrt(2 pi) scale_j,
// bounded by V / (1 - alpha), with mean Z.  The device records hold W / K with
// their own shift; Z = sum W / N over all N samples, which finalize computes
// with stream "volumes" K n_s / N (each stream's mean weighted by its share).
#include <cmath>
#include <limits>
#include <vector>

#include "runtime.h"

using namespace bfi;

namespace {

struct Modes {
    std::vector<double> lambda, scale;
    bool uniform0 = false;
    double log_k = 0.0, R = 0.0;
};

void modes_of(const bfi_lattice &lat, double lo, double hi, Modes *m)
{
    const int nx = lat.nx, nt = lat.nt, d = nx * nt;
    const double two_pi = 6.283185307179586476925286766559;
    const double c = lat.nu * lat.tau / (lat.a * lat.a);
    const double R2 = d * std::max(lo * lo, hi * hi);
    m->R = std::sqrt(R2);
    m->lambda.assign(d, 0.0);
    m->scale.assign(d, 0.0);
    m->log_k = 0.0;
    for (int bt = 0; bt < nt; ++bt)
        for (int bx = 0; bx < nx; ++bx) {
            const int kt = (bt + 1) / 2, kx = (bx + 1) / 2;
            const double mt = 2.0 * std::cos(two_pi * kt / nt) - 2.0;
            const double mx = 2.0 * std::cos(two_pi * kx / nx) - 2.0;
            const int j = bt * nx + bx;
            const double lam = (-mt - c * mt * mx + c * c * mx * mx) / (lat.D * lat.tau) + lat.m2;
            m->lambda[j] = lam;
            if (j == 0 && lam * R2 < 4.0) {
                m->uniform0 = true;
                m->scale[j] = m->R;
                m->log_k += std::log(2.0 * m->R);
            } else {
                m->scale[j] = lam * R2 <= 1.0 ? m->R : 1.0 / std::sqrt(lam);
                m->log_k += 0.5 * std::log(two_pi) + std::log(m->scale[j]);
            }
        }
}

bfi_status check_args(const bfi_lattice *lat, int prec, double lo, double hi, double alpha)
{
    BFI_TRY(check_lattice(lat));
    if (lat->antithetic)
        return fail(BFI_EUNSUPPORTED, "the Gaussian-proposal sampler draws single points");
    if (lat->nx * lat->nt > kIsMaxD)
        return fail(BFI_EUNSUPPORTED, "the Gaussian-proposal sampler is compiled for d <= %d",
                    kIsMaxD);
    if (prec == BFI_FP64_SHIFTED)
        return fail(BFI_EUNSUPPORTED, "the Gaussian-proposal sampler has no shifted FP64 form");
    if (!known_precision(prec))
        return fail(BFI_EINVAL, "unknown precision %d", prec);
    if (!std::isfinite(lo) || !std::isfinite(hi) || !(lo < hi))
        return fail(BFI_EINVAL, "cube: need finite lo < hi");
    if (!(alpha >= 0.0 && alpha <= 1.0))
        return fail(BFI_EINVAL, "gaussian_fraction must be in [0, 1]");
    return BFI_OK;
}

IsTable make_table(const bfi_lattice &lat, double lo, double hi, double alpha, uint64_t seed,
                   Modes *modes)
{
    modes_of(lat, lo, hi, modes);
    const int d = lat.nx * lat.nt;
    IsTable t{};
    for (int j = 0; j < d; ++j) {
        t.scale64[j] = modes->scale[j];
        t.inv_scale64[j] = 1.0 / modes->scale[j];
        t.scale32[j] = static_cast<float>(t.scale64[j]);
        t.inv_scale32[j] = static_cast<float>(t.inv_scale64[j]);
    }
    t.lo64 = lo;
    t.hi64 = hi;
    t.map_scale64 = (hi - lo) * 0x1p-32;
    t.map_base64 = lo + 0.5 * t.map_scale64;
    t.lo32 = static_cast<float>(lo);
    t.hi32 = static_cast<float>(hi);
    t.map_scale32 = static_cast<float>(t.map_scale64);
    t.map_base32 = static_cast<float>(t.map_base64);
    const double ninf = -std::numeric_limits<double>::infinity();
    const double log_v = d * std::log(hi - lo);
    t.log_ga = alpha > 0.0 ? std::log(alpha) : ninf;
    t.log_un = alpha < 1.0 ? std::log1p(-alpha) + modes->log_k - log_v : ninf;
    t.uniform0 = modes->uniform0 ? 1 : 0;
    t.seed_lo = static_cast<uint32_t>(seed);
    t.seed_hi = static_cast<uint32_t>(seed >> 32);
    return t;
}

SubList stream_list(int d, double lo, double hi, size_t count, const uint64_t *id,
                    const uint64_t *n, const uint64_t *offset)
{
    SubList s;
    s.d = d;
    s.id.assign(id, id + count);
    s.n.assign(n, n + count);
    s.offset.assign(offset, offset + count);
    s.lo.assign(count * d, lo);
    s.hi.assign(count * d, hi);
    return s;
}

bfi_status run_streams(bfi_context *ctx, const bfi_lattice &lat, int prec, uint64_t seed,
                       double lo, double hi, double alpha, const SubList &streams,
                       const bfi_launch *launch, double *partials, Modes *modes)
{
    // the Philox counter index * blocks + j of the last sample must fit in 64
    // bits (Gaussian streams take ceil((2 ceil(d/2) + 1)/4) blocks per sample,
    // more than the uniform ones' ceil(d/4)): offset + n <= floor(2^64 / blocks)
    const int d = lat.nx * lat.nt;
    const unsigned __int128 index_end = (static_cast<unsigned __int128>(1) << 64) /
                                        static_cast<unsigned>((2 * ((d + 1) / 2) + 1 + 3) / 4);
    for (size_t s = 0; s < streams.size(); ++s) {
        if (streams.n[s] < 2)
            return fail(BFI_EINVAL, "stream %zu has n = %llu < 2", s,
                        static_cast<unsigned long long>(streams.n[s]));
        if (static_cast<unsigned __int128>(streams.offset[s]) + streams.n[s] > index_end)
            return fail(BFI_EINVAL, "stream %zu: sample indices overflow the Philox counter", s);
    }
    BFI_HIP(hipSetDevice(ctx->device));
    const IsTable table = make_table(lat, lo, hi, alpha, seed, modes);
    bfi_plan *p = nullptr;
    BFI_TRY(plan_build_is(ctx, lat, prec, streams, table, launch, &p));
    p->launch.use_graph = 0;
    bfi_status s = plan_enqueue(p, seed, nullptr, ctx->stream, true);
    p->last_stream = ctx->stream;
    if (s == BFI_OK)
        s = bfi_plan_partials(p, partials);
    plan_free(p);
    return s;
}

}  // namespace

extern "C" {

bfi_status bfi_is_modes(const bfi_lattice *lat, double box_lo, double box_hi, double *lambda,
                        int32_t *uniform, double *scale, double *log_k)
{
    return guarded([&]() -> bfi_status {
        BFI_TRY(check_args(lat, BFI_FP64, box_lo, box_hi, 0.5));
        if (!lambda || !uniform || !scale || !log_k)
            return fail(BFI_EINVAL, "outputs must be non-NULL");
        Modes m;
        modes_of(*lat, box_lo, box_hi, &m);
        const int d = lat->nx * lat->nt;
        for (int j = 0; j < d; ++j) {
            lambda[j] = m.lambda[j];
            scale[j] = m.scale[j];
            uniform[j] = (j == 0 && m.uniform0) ? 1 : 0;
        }
        *log_k = m.log_k;
        return BFI_OK;
    });
}

bfi_status bfi_is_eval(bfi_context *ctx, const bfi_lattice *lat, bfi_precision prec, uint64_t seed,
                       double box_lo, double box_hi, double gaussian_fraction, size_t count,
                       const uint64_t *stream_id, const uint64_t *n, const uint64_t *offset,
                       const bfi_launch *launch, double *partials)
{
    return guarded([&]() -> bfi_status {
        if (!ctx)
            return fail(BFI_EINVAL, "context is NULL");
        BFI_TRY(check_args(lat, prec, box_lo, box_hi, gaussian_fraction));
        if (count == 0)
            return BFI_OK;
        if (!stream_id || !n || !offset || !partials)
            return fail(BFI_EINVAL, "stream arrays and partials must be non-NULL");
        Modes m;
        const SubList streams =
            stream_list(lat->nx * lat->nt, box_lo, box_hi, count, stream_id, n, offset);
        return run_streams(ctx, *lat, prec, seed, box_lo, box_hi, gaussian_fraction, streams, launch,
                           partials, &m);
    });
}

bfi_status bfi_integrate_is(bfi_context *ctx, const bfi_lattice *lat, bfi_precision prec,
                            uint64_t seed, double box_lo, double box_hi, double gaussian_fraction,
                            uint32_t streams, uint64_t budget, const bfi_launch *launch,
                            bfi_result *out)
{
    return guarded([&]() -> bfi_status {
        if (!ctx || !out)
            return fail(BFI_EINVAL, "context and result must be non-NULL");
        BFI_TRY(check_args(lat, prec, box_lo, box_hi, gaussian_fraction));
        if (streams < 1)
            return fail(BFI_EINVAL, "need at least one stream");
        // round(alpha B) samples over Gaussian streams 1..S, the rest over uniform
        // streams 2^63 + 1..S; each share split floor(b/S) + (i < b mod S)
        const uint64_t n_g = static_cast<uint64_t>(
            std::llround(gaussian_fraction * static_cast<double>(budget)));
        std::vector<uint64_t> ids, ns, offs;
        const uint64_t shares[2] = {n_g, budget - n_g};
        for (int comp = 0; comp < 2; ++comp) {
            if (shares[comp] == 0)
                continue;
            const uint64_t base = comp == 0 ? 0 : kIsUniformStream;
            for (uint32_t i = 0; i < streams; ++i) {
                const uint64_t k = shares[comp] / streams + (i < shares[comp] % streams ? 1 : 0);
                if (k < 2)
                    return fail(BFI_EINVAL, "budget too small: every stream needs 2 samples");
                ids.push_back(base + 1 + i);
                ns.push_back(k);
                offs.push_back(0);
            }
        }
        const int d = lat->nx * lat->nt, nx = lat->nx;
        const SubList list = stream_list(d, box_lo, box_hi, ids.size(), ids.data(), ns.data(),
                                         offs.data());
        std::vector<double> rec(ids.size() * BFI_PARTIAL_LEN(nx));
        Modes m;
        BFI_TRY(run_streams(ctx, *lat, prec, seed, box_lo, box_hi, gaussian_fraction, list, launch,
                            rec.data(), &m));
        // stream "volume" K n_s / N folded into the record's shift
        const double log_total = std::log(static_cast<double>(budget));
        for (size_t s = 0; s < ids.size(); ++s)
            rec[s * BFI_PARTIAL_LEN(nx) + 1] -=
                m.log_k + std::log(static_cast<double>(ns[s])) - log_total;
        std::vector<double> unit_lo(ids.size() * d, 0.0), unit_hi(ids.size() * d, 1.0);
        return finalize_records(nx, d, ids.size(), unit_lo.data(), unit_hi.data(), rec.data(), out);
    });
}

bfi_status bfi_debug_is_points(bfi_context *ctx, const bfi_lattice *lat, bfi_precision prec,
                               uint64_t seed, double box_lo, double box_hi, uint64_t stream_id,
                               const uint64_t *index, uint64_t n, double *u_out,
                               double *half_z2_out)
{
    return guarded([&]() -> bfi_status {
        if (!ctx)
            return fail(BFI_EINVAL, "context is NULL");
        BFI_TRY(check_args(lat, prec, box_lo, box_hi, 0.5));
        if (n == 0)
            return BFI_OK;
        if (!index || !u_out || !half_z2_out)
            return fail(BFI_EINVAL, "index and outputs must be non-NULL");
        BFI_HIP(hipSetDevice(ctx->device));
        const int d = lat->nx * lat->nt;
        Modes m;
        const IsTable table = make_table(*lat, box_lo, box_hi, 0.5, seed, &m);
        struct Buf {
            void *p = nullptr;
            ~Buf()
            {
                if (p)
                    (void)hipFree(p);
            }
        } dt, di, du, dh;
        BFI_HIP(hipMalloc(&dt.p, sizeof(IsTable)));
        BFI_HIP(hipMalloc(&di.p, n * 8));
        BFI_HIP(hipMalloc(&du.p, n * d * 8));
        BFI_HIP(hipMalloc(&dh.p, n * 8));
        BFI_HIP(hipMemcpy(dt.p, &table, sizeof(IsTable), hipMemcpyHostToDevice));
        BFI_HIP(hipMemcpy(di.p, index, n * 8, hipMemcpyHostToDevice));
        IsDebugArgs a{};
        a.table = static_cast<const IsTable *>(dt.p);
        a.index = static_cast<const uint64_t *>(di.p);
        a.u_out = static_cast<double *>(du.p);
        a.hz_out = static_cast<double *>(dh.p);
        a.n = n;
        a.id = stream_id;
        a.prec = prec;
        BFI_HIP(launch_is_debug(lat->nx, lat->nt, a, ctx->stream));
        BFI_HIP(hipStreamSynchronize(ctx->stream));
        BFI_HIP(hipMemcpy(u_out, du.p, n * d * 8, hipMemcpyDeviceToHost));
        BFI_HIP(hipMemcpy(half_z2_out, dh.p, n * 8, hipMemcpyDeviceToHost));
        return BFI_OK;
    });
}

}  // extern "C"
