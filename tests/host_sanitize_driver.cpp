// Calls the host-only entry points of the C ABI (no GPU needed): status
// strings, shape table, finalize of shifted records, record merging, the
// adaptive refinement decision and their argument checks, so that a build of
// the host sources with AddressSanitizer and UndefinedBehaviorSanitizer can
// check them.  Exit status 0 and "ok" when every call behaves as declared.
#include <cmath>
#include <cstdio>
#include <vector>

#include "bfi.h"

#define EXPECT(c)                                                          \
    do {                                                                   \
        if (!(c)) {                                                        \
            std::fprintf(stderr, "%s:%d: %s\n", __FILE__, __LINE__, #c);   \
            return 1;                                                      \
        }                                                                  \
    } while (0)

static bfi_lattice lattice(int nx, int nt)
{
    bfi_lattice l{};
    l.nx = nx;
    l.nt = nt;
    l.nu = 0.7;
    l.D = l.a = l.tau = l.g = 1.0;
    return l;
}

int main()
{
    for (int s = 0; s >= -8; --s)
        EXPECT(bfi_status_string(static_cast<bfi_status>(s)) != nullptr);
    EXPECT(bfi_shape_supported(10, 2) == BFI_OK);
    EXPECT(bfi_shape_supported(7, 7) != BFI_OK);
    int32_t shapes[2 * 64];
    int32_t count = 0;
    EXPECT(bfi_supported_shapes(shapes, 64, &count) == BFI_OK && count > 0);

    for (int nx : {1, 3, 10}) {
        const int nt = 2, d = nx * nt, ns = 5, len = BFI_PARTIAL_LEN(nx);
        bfi_lattice lat = lattice(nx, nt);
        std::vector<uint64_t> id(ns), n(ns), off(ns, 0);
        std::vector<double> lo(ns * d), hi(ns * d), rec(ns * len), more(ns * len);
        std::vector<double> split(ns * BFI_SPLIT_LEN(d), 0.25);
        for (int s = 0; s < ns; ++s) {
            id[s] = 8 + s;
            n[s] = 100 + s;
            for (int k = 0; k < d; ++k) {
                lo[s * d + k] = -1.0 - 0.1 * s;
                hi[s * d + k] = 1.0 + 0.2 * k;
            }
            double *r = &rec[s * len];
            r[0] = static_cast<double>(n[s]);
            r[1] = -3.0 + s;  // shift
            r[2] = 40.0;
            r[3] = 30.0;
            for (int i = 0; i < nx; ++i) {
                r[4 + i] = 1.0 - 0.1 * i;
                r[4 + nx + i] = 2.0;
                r[4 + 2 * nx + i] = 0.5;
            }
            for (int i = 0; i < len; ++i)
                more[s * len + i] = r[i];
            more[s * len + 1] = 5.0 - s;
        }
        bfi_subvolumes sv{static_cast<size_t>(ns), id.data(), lo.data(), hi.data(), n.data(),
                          off.data()};
        bfi_result res{};
        EXPECT(bfi_finalize(&lat, &sv, rec.data(), &res) == BFI_OK);
        EXPECT(std::isfinite(res.log_Z) && res.nx == nx);
        lat.antithetic = 1;
        bfi_result res2{};
        EXPECT(bfi_finalize(&lat, &sv, rec.data(), &res2) == BFI_OK);
        EXPECT(res2.n_evals == 2 * res.n_evals);
        lat.antithetic = 0;
        EXPECT(bfi_partials_merge(nx, ns, rec.data(), more.data()) == BFI_OK);
        more[1] = NAN;
        EXPECT(bfi_partials_merge(nx, ns, rec.data(), more.data()) == BFI_EINVAL);
        EXPECT(bfi_partials_merge(0, ns, rec.data(), more.data()) == BFI_EINVAL);
        EXPECT(bfi_last_error() != nullptr);
        if (d <= 32) {
            bfi_adaptive_config cfg{};
            cfg.target_rel_err = 1e-3;
            cfg.max_evals = 1u << 20;
            cfg.n_min = 64;
            cfg.n_max = 1u << 16;
            cfg.split_log2 = 2;
            cfg.max_rounds = 8;
            cfg.refine_fraction = 0.5;
            std::vector<int32_t> action(ns, 7);
            EXPECT(bfi_adaptive_decide(&lat, &sv, rec.data(), split.data(), nullptr, &cfg,
                                       action.data()) == BFI_OK);
            for (int32_t a : action)
                EXPECT(a >= -1 && a <= d);
            std::vector<int32_t> again(ns, 7);
            EXPECT(bfi_adaptive_decide(&lat, &sv, rec.data(), split.data(), rec.data(), &cfg,
                                       again.data()) == BFI_OK);
            EXPECT(again == action);
            cfg.split_samples = 1;
            EXPECT(bfi_adaptive_decide(&lat, &sv, rec.data(), split.data(), nullptr, &cfg,
                                       action.data()) == BFI_EINVAL);
            cfg.split_samples = 0;
            cfg.refine_fraction = 2.0;
            EXPECT(bfi_adaptive_decide(&lat, &sv, rec.data(), split.data(), nullptr, &cfg,
                                       action.data()) == BFI_EINVAL);
        }
        rec[0] = 1.0;  // n < 2
        EXPECT(bfi_finalize(&lat, &sv, rec.data(), &res) == BFI_EINVAL);
    }
    std::printf("ok\n");
    return 0;
}
