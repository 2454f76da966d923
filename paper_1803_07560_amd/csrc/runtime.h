// Host runtime shared by the C ABI translation units (runtime.cpp, adaptive.cpp,
// server.cpp).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <exception>
#include <map>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "bfi.h"
#include "internal.h"
#include "is_internal.h"

namespace bfi {

bfi_status fail(bfi_status s, const char *fmt, ...);
bfi_status hip_fail(hipError_t e, const char *what);
void clear_error();

#define BFI_HIP(call)                                 \
    do {                                              \
        hipError_t bfi_e_ = (call);                   \
        if (bfi_e_ != hipSuccess)                     \
            return ::bfi::hip_fail(bfi_e_, #call);    \
    } while (0)

#define BFI_TRY(call)                                 \
    do {                                              \
        bfi_status bfi_s_ = (call);                   \
        if (bfi_s_ != BFI_OK)                         \
            return bfi_s_;                            \
    } while (0)

bool shape_compiled(int nx, int nt);
// BFI_FP64, BFI_FP32_SHIFTED or BFI_FP64_SHIFTED
inline bool known_precision(int prec)
{
    return prec == BFI_FP64 || prec == BFI_FP32_SHIFTED || prec == BFI_FP64_SHIFTED;
}
// Dispatch to the kernels compiled for lattice shape (nx, nt).
hipError_t launch_mc(int nx, int nt, const LaunchSpec &spec, const McArgs &args, hipStream_t st);
hipError_t kernel_info(int nx, int nt, const LaunchSpec &spec, KernelInfo *info);
// Gaussian-proposal sampler kernels of shape (nx, nt).
hipError_t launch_is(int nx, int nt, const LaunchSpec &spec, const IsArgs &args, hipStream_t st);
hipError_t is_kernel_info(int nx, int nt, const LaunchSpec &spec, KernelInfo *info);
hipError_t launch_is_debug(int nx, int nt, const IsDebugArgs &args, hipStream_t st);
bfi_status check_lattice(const bfi_lattice *lat);
bfi_status check_subvolumes(const bfi_lattice *lat, const bfi_subvolumes *subs);
ActionCoef make_coef(const bfi_lattice &lat);

// Owned copy of a subvolume list.
struct SubList {
    std::vector<uint64_t> id, n, offset;
    std::vector<double> lo, hi;  // count x d
    int d = 0;
    size_t size() const { return id.size(); }
    bfi_subvolumes view() const
    {
        return bfi_subvolumes{id.size(), id.data(), lo.data(), hi.data(), n.data(), offset.data()};
    }
    static SubList copy_of(const bfi_subvolumes &s, int d);
};

// Uniform bisection of a box: 2^k leaves, level t halves dim t mod d at
// 0.5 (lo + hi); heap ids 2^k + b; budget split floor(B/2^k) + (b < B mod 2^k).
SubList uniform_split(int d, const double *box_lo, const double *box_hi, int k, uint64_t budget);

struct TuneKey {
    int nx, nt, prec;
    int pairs = 0;  // antithetic pairs: a kernel of its own, tuned apart
    int obs = 0;    // observable (anchored or averaged), likewise
    bool operator<(const TuneKey &o) const
    {
        return std::tie(nx, nt, prec, pairs, obs) < std::tie(o.nx, o.nt, o.prec, o.pairs, o.obs);
    }
};
struct TuneEntry {
    bfi_launch launch;
    double evals_per_s;
};

// Runs the body of a C ABI entry point: C++ exceptions (host allocation
// failure above all) become status codes, so nothing unwinds into a C caller.
template <class F>
bfi_status guarded(F &&body) noexcept
{
    try {
        return body();
    } catch (const std::bad_alloc &) {
        return fail(BFI_ENOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        return fail(BFI_EINVAL, "%s", e.what());
    } catch (...) {
        return fail(BFI_EINVAL, "unexpected exception");
    }
}

// A named range of host work on the calling thread, visible to rocprofv3
// --marker-trace (roctx); without a tool attached the calls return at once.
struct TraceRange {
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};
// Consecutive phases of one loop body: next() closes the current range and
// opens the following one; leaving the scope closes the last.
struct TracePhases {
    explicit TracePhases(const char *first) { roctxRangePushA(first); }
    void next(const char *name)
    {
        roctxRangePop();
        roctxRangePushA(name);
    }
    ~TracePhases() { roctxRangePop(); }
    TracePhases(const TracePhases &) = delete;
    TracePhases &operator=(const TracePhases &) = delete;
};

// Resolve a requested launch (zeros = tuned or default) for a lattice.
bfi_launch resolve_launch(const bfi_context *ctx, const bfi_lattice &lat, int prec, bool split,
                          const bfi_launch *req);

// Host finalize of partial records (see bfi_finalize).
// evals_per_sample: integrand evaluations behind one record sample (2 for
// antithetic pairs), for n_evals.
bfi_status finalize_records(int nx, int d, size_t nsub, const double *lo, const double *hi,
                            const double *partials, bfi_result *out, int evals_per_sample = 1);

// Take the device address of the allocation-free entry point's scratch array on
// `device` (which must be current); once per device, later calls return at once.
bfi_status noalloc_setup(int device);

}  // namespace bfi

struct bfi_context {
    int device = 0;
    int cu_count = 0;
    hipStream_t stream = nullptr;
    std::string arch;
    std::map<bfi::TuneKey, bfi::TuneEntry> tuned;
};

// A resident evaluation: descriptors, work items and buffers on the device.
struct bfi_plan {
    bfi_context *ctx = nullptr;
    int kind = 0;  // 0: lattice action (mc_kernel), 1: N-sphere test integrand,
                   // 2: Gaussian-proposal sampler (is_kernel) over streams
    bfi_lattice lat{};
    int prec = 0;
    int d = 0, nx = 0, rec_len = 0;
    bool split = false;
    bfi::SubList subs;
    bfi_launch launch{};
    uint32_t nitems = 0;
    uint32_t grid = 0;
    uint64_t n_evals = 0;

    double *d_base64 = nullptr, *d_scale64 = nullptr;
    float *d_base32 = nullptr, *d_scale32 = nullptr;
    uint64_t *d_ids = nullptr, *d_offsets = nullptr;
    bfi::EvalParams *d_params = nullptr;
    bfi::EvalParams params{};  // host copy of *d_params
    bfi::WorkItem *d_items = nullptr;
    double *d_item_rec = nullptr, *d_item_split = nullptr;
    uint32_t *d_sub_first = nullptr;
    double *d_sub_rec = nullptr, *d_sub_split = nullptr;
    uint32_t *d_head = nullptr;
    bfi::IsTable *d_is_table = nullptr;  // kind 2

    // captured replays (queue reset, kernel, merge, copy to the destination), one
    // per (stream, destination) pair, the kMaxReplays used last kept (ordered by
    // last use): alternating output buffers replays without capturing again
    struct Replay {
        hipGraphExec_t exec = nullptr;
        hipGraph_t def = nullptr;
        hipStream_t stream = nullptr;
        double *dst = nullptr;
    };
    static constexpr size_t kMaxReplays = 4;
    std::vector<Replay> replays;
    hipStream_t last_stream = nullptr;
    // bracket the Monte Carlo kernel of every run (timing of the hot kernel)
    hipEvent_t ev_start = nullptr, ev_stop = nullptr;
};

namespace bfi {
bfi_status plan_build(bfi_context *ctx, const bfi_lattice &lat, int prec, const SubList &subs,
                      const bfi_launch *launch, bool split, bfi_plan **out);
// Plan for the Gaussian-proposal sampler: `streams` lists stream ids (bit 63:
// uniform component), sample counts and offsets; lo/hi rows are the cube.
bfi_status plan_build_is(bfi_context *ctx, const bfi_lattice &lat, int prec,
                         const SubList &streams, const IsTable &table, const bfi_launch *launch,
                         bfi_plan **out);
// Plan for the N-sphere integrand over `dim`-dimensional boxes (FP64, split
// statistics always on, 256-thread blocks); records have nx = 0.
bfi_status plan_build_nsphere(bfi_context *ctx, int dim, const SubList &subs,
                              const bfi_launch *launch, bfi_plan **out);
// timed: record the plan's events around the Monte Carlo kernel (not inside a
// graph capture, where recorded events carry no timestamps)
bfi_status plan_enqueue(bfi_plan *p, uint64_t seed, double *dst, hipStream_t stream, bool timed);
bfi_status plan_free(bfi_plan *p);
// Write the seed into the plan's device parameters (waits for earlier runs).
bfi_status plan_set_seed(bfi_plan *p, uint64_t seed);
}  // namespace bfi
