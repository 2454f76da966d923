// Launch-shape autotuner and its JSON cache.
//
// Candidates: samples_per_thread K in {16, 32, ..., 1024} x block in
// {64, 128, ..., 1024} x {one block per item, persistent queue}.  Each candidate runs
// a resident plan over a uniform partition of [-4, 4]^d (1024 subvolumes, or
// fewer for tiny budgets) once to warm up and three times under HIP events on
// the context's stream; the fastest rate is kept for (nx, nt, precision, single
// points or antithetic pairs, observable).  A plan without an entry of its own
// takes its sampler's anchored-product entry, then the single-point one.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <fstream>
#include <sstream>

#include "runtime.h"

using namespace bfi;

namespace {

struct Events {
    hipEvent_t a = nullptr, b = nullptr;
    ~Events()
    {
        if (a)
            (void)hipEventDestroy(a);
        if (b)
            (void)hipEventDestroy(b);
    }
};

bfi_status time_candidate(bfi_context *ctx, const bfi_lattice &lat, int prec, const SubList &subs,
                          const bfi_launch &cand, double *rate)
{
    bfi_plan *p = nullptr;
    BFI_TRY(plan_build(ctx, lat, prec, subs, &cand, false, &p));
    Events ev;
    bfi_status s = BFI_OK;
    hipError_t e = hipEventCreate(&ev.a);
    if (e == hipSuccess)
        e = hipEventCreate(&ev.b);
    if (e != hipSuccess) {
        plan_free(p);
        return hip_fail(e, "hipEventCreate");
    }
    s = plan_enqueue(p, 1, nullptr, ctx->stream, false);
    if (s == BFI_OK && (e = hipEventRecord(ev.a, ctx->stream)) != hipSuccess)
        s = hip_fail(e, "hipEventRecord");
    for (int r = 0; r < 3 && s == BFI_OK; ++r)
        s = plan_enqueue(p, 2 + r, nullptr, ctx->stream, false);
    if (s == BFI_OK && (e = hipEventRecord(ev.b, ctx->stream)) != hipSuccess)
        s = hip_fail(e, "hipEventRecord");
    if (s == BFI_OK && (e = hipEventSynchronize(ev.b)) != hipSuccess)
        s = hip_fail(e, "hipEventSynchronize");
    float ms = 0.0f;
    if (s == BFI_OK && (e = hipEventElapsedTime(&ms, ev.a, ev.b)) != hipSuccess)
        s = hip_fail(e, "hipEventElapsedTime");
    if (s == BFI_OK)
        *rate = 3.0 * static_cast<double>(p->n_evals) / (ms * 1e-3);
    (void)hipStreamSynchronize(ctx->stream);
    plan_free(p);
    return s;
}

}  // namespace

extern "C" {

bfi_status bfi_autotune(bfi_context *ctx, const bfi_lattice *lat, bfi_precision prec,
                        uint64_t evals_per_trial, bfi_launch *best, double *best_evals_per_s)
{
    return guarded([&]() -> bfi_status {
        if (!ctx)
            return fail(BFI_EINVAL, "context is NULL");
        if (!known_precision(prec))
            return fail(BFI_EINVAL, "unknown precision");
        BFI_TRY(check_lattice(lat));
        if (evals_per_trial < (uint64_t(1) << 16))
            return fail(BFI_EINVAL, "evals_per_trial must be at least 2^16");
        BFI_HIP(hipSetDevice(ctx->device));
        const int d = lat->nx * lat->nt;
        const int k = static_cast<int>(std::min<uint64_t>(10, std::log2(evals_per_trial / 1024.0)));
        std::vector<double> lo(d, -4.0), hi(d, 4.0);
        // antithetic pairs: two evaluations per sample index
        SubList subs = uniform_split(d, lo.data(), hi.data(), std::max(k, 0),
                                     lat->antithetic ? evals_per_trial / 2 : evals_per_trial);

        const int Ks[] = {16, 32, 64, 128, 256, 512, 1024};
        const int blocks[] = {64, 128, 256, 512, 1024};
        bfi_launch top{};
        double top_rate = -1.0;
        for (int persistent = 0; persistent <= 1; ++persistent)
            for (int b : blocks)
                for (int K : Ks) {
                    bfi_launch cand{K, b, persistent, 0};
                    double rate = 0.0;
                    bfi_status s = time_candidate(ctx, *lat, prec, subs, cand, &rate);
                    if (s == BFI_EINVAL)
                        continue;  // e.g. too many work items for a small K
                    BFI_TRY(s);
                    if (rate > top_rate) {
                        top_rate = rate;
                        top = cand;
                    }
                }
        if (top_rate <= 0)
            return fail(BFI_EDEVICE, "no launch shape could be timed");
        ctx->tuned[TuneKey{lat->nx, lat->nt, prec, lat->antithetic ? 1 : 0, lat->observable}] =
            TuneEntry{top, top_rate};
        if (best)
            *best = top;
        if (best_evals_per_s)
            *best_evals_per_s = top_rate;
        return BFI_OK;
    });
}

bfi_status bfi_tune_save(const bfi_context *ctx, const char *path)
{
    return guarded([&]() -> bfi_status {
        if (!ctx || !path)
            return fail(BFI_EINVAL, "context and path must be non-NULL");
        std::ofstream f(path);
        if (!f)
            return fail(BFI_EINVAL, "cannot open %s for writing", path);
        f << "{\n  \"arch\": \"" << ctx->arch << "\",\n  \"entries\": [";
        bool firstEntry = true;
        for (const auto &kv : ctx->tuned) {
            f << (firstEntry ? "\n" : ",\n");
            firstEntry = false;
            char line[256];
            std::snprintf(line, sizeof(line),
                          "    {\"nx\": %d, \"nt\": %d, \"prec\": %d, \"pairs\": %d, "
                          "\"observable\": %d, \"samples_per_thread\": %d, \"block\": %d, "
                          "\"persistent\": %d, \"evals_per_s\": %.6e}",
                          kv.first.nx, kv.first.nt, kv.first.prec, kv.first.pairs, kv.first.obs,
                          kv.second.launch.samples_per_thread, kv.second.launch.block,
                          kv.second.launch.persistent, kv.second.evals_per_s);
            f << line;
        }
        f << "\n  ]\n}\n";
        return f ? BFI_OK : fail(BFI_EINVAL, "write to %s failed", path);
    });
}

bfi_status bfi_tune_load(bfi_context *ctx, const char *path)
{
    return guarded([&]() -> bfi_status {
        if (!ctx || !path)
            return fail(BFI_EINVAL, "context and path must be non-NULL");
        std::ifstream f(path);
        if (!f)
            return fail(BFI_EINVAL, "cannot open %s", path);
        std::stringstream ss;
        ss << f.rdbuf();
        const std::string txt = ss.str();
        // the file is the flat object bfi_tune_save writes: read "arch", then the
        // numeric fields of each {...} entry
        auto field = [](const std::string &obj, const char *key, double *v) {
            const std::string k = std::string("\"") + key + "\"";
            size_t p = obj.find(k);
            if (p == std::string::npos)
                return false;
            p = obj.find(':', p);
            if (p == std::string::npos)
                return false;
            char *end = nullptr;
            *v = std::strtod(obj.c_str() + p + 1, &end);
            return end != obj.c_str() + p + 1;
        };
        size_t a = txt.find("\"arch\"");
        if (a == std::string::npos)
            return fail(BFI_EINVAL, "%s: no arch", path);
        size_t q1 = txt.find('"', txt.find(':', a) + 1), q2 = txt.find('"', q1 + 1);
        if (q1 == std::string::npos || q2 == std::string::npos)
            return fail(BFI_EINVAL, "%s: bad arch", path);
        if (txt.substr(q1 + 1, q2 - q1 - 1) != ctx->arch)
            return BFI_OK;
        size_t pos = txt.find('[', q2);
        while (pos != std::string::npos) {
            size_t o = txt.find('{', pos), c = txt.find('}', o);
            if (o == std::string::npos || c == std::string::npos)
                break;
            const std::string obj = txt.substr(o, c - o + 1);
            double nx, nt, prec, K, block, pers, rate, pairs = 0, obs = 0;
            if (!field(obj, "pairs", &pairs))
                pairs = 0;  // entries written before pairs were tuned apart
            if (!field(obj, "observable", &obs))
                obs = 0;
            if (field(obj, "nx", &nx) && field(obj, "nt", &nt) && field(obj, "prec", &prec) &&
                field(obj, "samples_per_thread", &K) && field(obj, "block", &block) &&
                field(obj, "persistent", &pers) && field(obj, "evals_per_s", &rate)) {
                const int b = static_cast<int>(block);
                if (shape_compiled(static_cast<int>(nx), static_cast<int>(nt)) && K >= 1 &&
                    K <= (1 << 20) && (b == 64 || b == 128 || b == 256) &&
                    (prec == 0 || prec == 1 || prec == 2) && (pairs == 0 || pairs == 1) &&
                    (obs == 0 || obs == 1)) {
                    bfi_launch l{static_cast<int32_t>(K), b, pers != 0 ? 1 : 0, 0};
                    ctx->tuned[TuneKey{static_cast<int>(nx), static_cast<int>(nt),
                                       static_cast<int>(prec), static_cast<int>(pairs),
                                       static_cast<int>(obs)}] =
                        TuneEntry{l, rate};
                }
            }
            pos = c + 1;
        }
        return BFI_OK;
    });
}

}  // extern "C"
