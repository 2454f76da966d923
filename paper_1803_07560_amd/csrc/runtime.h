// Host runtime shared by the C ABI translation units (runtime.cpp, adaptive.cpp,
// server.cpp).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstdint>
#include <exception>
#include <map>
#include <new>
#include <string>
#include <thread>
#include <tuple>
#include <type_traits>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "bfi.h"
#include "host_pool.h"
#include "internal.h"
#include "is_internal.h"
#include "sph_internal.h"

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
// Spherical-coordinate sampler kernels of shape (nx, nt).
hipError_t launch_sph(int nx, int nt, const LaunchSpec &spec, const SphArgs &args, hipStream_t st);
hipError_t sph_kernel_info(int nx, int nt, const LaunchSpec &spec, KernelInfo *info);
hipError_t launch_sph_debug(int nx, int nt, const SphDebugArgs &args, hipStream_t st);
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
// antithetic pairs), for n_evals.  leaf_var (nsub doubles, or NULL) gets each
// subvolume's contribution to the variance of C, sum_r [Var N_s - 2 C Cov_s +
// C^2 Var Z_s] / Z^2, clamped at 0.  Large lists are summed in parallel chunks
// whose sums combine in a fixed order (the result does not depend on threads).
// volumes (nsub doubles, or NULL): the products of the extents, when the caller
// keeps them (they must equal the product over dimensions in order).
bfi_status finalize_records(int nx, int d, size_t nsub, const double *lo, const double *hi,
                            const double *partials, bfi_result *out, int evals_per_sample = 1,
                            double *leaf_var = nullptr, const double *volumes = nullptr);

// Evaluates work lists that change from call to call (adaptive rounds) with
// resident buffers: entries are pushed into pinned staging, run() uploads them,
// builds items and point maps on the device, drains them with the persistent
// kernel, merges and downloads one record (and split statistics) per entry,
// all as one captured graph updated in place from call to call.  Buffers grow
// geometrically and are freed by the destructor.  Blocking on the context's
// stream; not thread-safe.
class ResidentEval {
public:
    ResidentEval() = default;
    ~ResidentEval();
    ResidentEval(const ResidentEval &) = delete;
    ResidentEval &operator=(const ResidentEval &) = delete;
    // split: accumulate split statistics (256-thread blocks, d <= 32)
    bfi_status init(bfi_context *ctx, const bfi_lattice &lat, int prec, bool split,
                    const bfi_launch *launch);
    bfi_status reserve(size_t count);
    // append one entry: samples [offset, offset + n) of stream `id` over [lo, hi)
    bfi_status push(uint64_t id, uint64_t offset, uint64_t n, const double *lo, const double *hi);
    // bulk form: stage(count) sizes the list, then set() fills entry i (entries
    // may be set from several threads)
    bfi_status stage(size_t count);
    void set(size_t i, uint64_t id, uint64_t offset, uint64_t n, const double *lo,
             const double *hi)
    {
        set_counts(i, id, offset, n);
        set_box(i, lo, hi);
    }
    // the two halves of set: prepare reads the counts; the boxes are read only
    // when the replay copies them to the device, so they may be written after
    // prepare and before launch
    void set_counts(size_t i, uint64_t id, uint64_t offset, uint64_t n)
    {
        h_id_[i] = id;
        h_off_[i] = offset;
        h_n_[i] = n;
    }
    void set_box(size_t i, const double *lo, const double *hi)
    {
        const size_t d = static_cast<size_t>(d_);
        std::copy(lo, lo + d, h_lo_ + i * d);
        std::copy(hi, hi + d, h_hi_ + i * d);
    }
    size_t size() const { return count_; }
    // evaluate the pushed entries (then cleared): rec_out gets count x
    // BFI_PARTIAL_LEN(nx) records, split_out count x BFI_SPLIT_LEN(d) (split
    // only); device_ms the replay's duration from events around it
    bfi_status run(uint64_t seed, double *rec_out, double *split_out, double *device_ms);
    // the same in three steps, so that several evaluators' replays can be queued
    // back to back on the context's stream (all prepared before any launch: a
    // capture never begins while one of them is in flight) and the host reads
    // one's records while the next runs: prepare captures (or updates) the
    // replay, launch queues it, finish waits for it and copies the records out
    bfi_status prepare(uint64_t seed);
    bfi_status launch();
    bfi_status finish(double *rec_out, double *split_out, double *device_ms);
    // the last finished list's records and split statistics in the pinned
    // buffers the replay copied them to (finish with NULL outputs skips the
    // copy), valid until the next prepare; with record copies on only
    const double *records() const { return h_rec_; }
    const double *split_records() const { return h_split_; }
    // whether a replay copies its records to the host (default yes), set
    // before prepare; without, they stay in device memory for a consumer queued
    // after the replay on the context's stream, valid until the next prepare
    void set_copy_records(bool on) { copy_records_ = on; }
    const double *device_records() const { return d_sub_rec_; }
    const double *device_split_records() const { return d_sub_split_; }
    int instantiations() const { return instantiations_; }
    int updates() const { return updates_; }

private:
    bfi_status enqueue(size_t nsub, uint64_t nitems, hipStream_t st);
    void release();

    bfi_context *ctx_ = nullptr;
    bfi_lattice lat_{};
    int prec_ = 0, d_ = 0, rec_len_ = 0, split_len_ = 0;
    bool split_ = false, copy_records_ = true;
    bfi_launch launch_{};
    uint64_t chunk_ = 0, resident_blocks_ = 0;
    size_t count_ = 0;
    // pinned staging
    uint64_t *h_id_ = nullptr, *h_n_ = nullptr, *h_off_ = nullptr;
    double *h_lo_ = nullptr, *h_hi_ = nullptr, *h_rec_ = nullptr, *h_split_ = nullptr;
    EvalParams *h_params_ = nullptr;
    size_t cap_h_sub_ = 0, cap_h_rec_ = 0, cap_h_split_ = 0, cap_params_ = 0;
    // device
    uint64_t *d_id_ = nullptr, *d_n_ = nullptr, *d_off_ = nullptr;
    double *d_lo_ = nullptr, *d_hi_ = nullptr, *d_base64_ = nullptr, *d_scale64_ = nullptr;
    float *d_base32_ = nullptr, *d_scale32_ = nullptr;
    EvalParams *d_params_ = nullptr;
    uint32_t *d_sub_first_ = nullptr, *d_head_ = nullptr;
    WorkItem *d_items_ = nullptr;
    double *d_item_rec_ = nullptr, *d_item_split_ = nullptr, *d_sub_rec_ = nullptr,
           *d_sub_split_ = nullptr;
    size_t cap_d_sub_[6] = {}, cap_d_map_[6] = {}, cap_d_items_[3] = {}, cap_dparams_ = 0,
           cap_head_ = 0;
    hipGraphExec_t exec_ = nullptr;
    hipEvent_t ev_start_ = nullptr, ev_stop_ = nullptr;
    int instantiations_ = 0, updates_ = 0;
    size_t prepared_ = 0;   // entries of the replay prepared and not yet finished
    bool launched_ = false;
};

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
