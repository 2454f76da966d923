// Resident evaluation of work lists that change from call to call (the rounds of
// adaptive refinement): device buffers and pinned host staging sized once and
// grown geometrically, the whole device sequence captured in a hipGraph.
//
// One call: the list staged in pinned memory is copied to the device, the
// point maps and work items are built there (launch_build_items), the queue
// head is reset, the persistent Monte Carlo kernel drains the items, the merge
// kernel folds them into per-entry records, and the records (and split
// statistics) are copied back to pinned memory.  That sequence is captured on
// the context's stream and applied to the executable graph of the previous
// call with hipGraphExecUpdate (same nodes, new sizes and arguments); only when
// the update is refused is the graph instantiated again.  No device allocation
// happens unless a list outgrows every list before it.
#include "runtime.h"

#include <algorithm>
#include <cstring>

namespace bfi {

namespace {

template <class T>
hipError_t grow_device(T **p, size_t *cap, size_t need)
{
    if (need <= *cap && *p)
        return hipSuccess;
    const size_t n = std::max<size_t>({need, 2 * *cap, 64});
    if (*p) {
        hipError_t e = hipFree(*p);
        if (e != hipSuccess)
            return e;
        *p = nullptr;
    }
    *cap = 0;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(p), n * sizeof(T));
    if (e == hipSuccess)
        *cap = n;
    return e;
}

// Pinned staging keeps its contents when it grows (entries are appended).
template <class T>
hipError_t grow_pinned(T **p, size_t *cap, size_t used, size_t need)
{
    if (need <= *cap && *p)
        return hipSuccess;
    const size_t n = std::max<size_t>({need, 2 * *cap, 64});
    T *q = nullptr;
    hipError_t e = hipHostMalloc(reinterpret_cast<void **>(&q), n * sizeof(T), hipHostMallocDefault);
    if (e != hipSuccess)
        return e;
    if (*p) {
        std::memcpy(q, *p, used * sizeof(T));
        (void)hipHostFree(*p);
    }
    *p = q;
    *cap = n;
    return hipSuccess;
}

}  // namespace

ResidentEval::~ResidentEval() { release(); }

void ResidentEval::release()
{
    // a replay may still be queued (an error between launch and finish): let it
    // end before its graph and buffers go
    if (ctx_)
        (void)hipStreamSynchronize(ctx_->stream);
    if (exec_)
        (void)hipGraphExecDestroy(exec_);
    exec_ = nullptr;
    prepared_ = 0;
    launched_ = false;
    void *dev[] = {d_id_, d_n_, d_off_, d_lo_, d_hi_, d_base64_, d_scale64_, d_base32_, d_scale32_,
                   d_params_, d_sub_first_, d_items_, d_item_rec_, d_item_split_, d_sub_rec_,
                   d_sub_split_, d_head_};
    for (void *p : dev)
        if (p)
            (void)hipFree(p);
    void *host[] = {h_id_, h_n_, h_off_, h_lo_, h_hi_, h_rec_, h_split_, h_params_};
    if (ev_start_)
        (void)hipEventDestroy(ev_start_);
    if (ev_stop_)
        (void)hipEventDestroy(ev_stop_);
    ev_start_ = ev_stop_ = nullptr;
    for (void *p : host)
        if (p)
            (void)hipHostFree(p);
    d_id_ = d_n_ = d_off_ = nullptr;
    d_lo_ = d_hi_ = d_base64_ = d_scale64_ = nullptr;
    d_base32_ = d_scale32_ = nullptr;
    d_params_ = nullptr;
    d_sub_first_ = nullptr;
    d_items_ = nullptr;
    d_item_rec_ = d_item_split_ = d_sub_rec_ = d_sub_split_ = nullptr;
    d_head_ = nullptr;
    h_id_ = h_n_ = h_off_ = nullptr;
    h_lo_ = h_hi_ = h_rec_ = h_split_ = nullptr;
    h_params_ = nullptr;
}

bfi_status ResidentEval::init(bfi_context *ctx, const bfi_lattice &lat, int prec, bool split,
                              const bfi_launch *launch)
{
    ctx_ = ctx;
    lat_ = lat;
    prec_ = prec;
    split_ = split;
    d_ = lat.nx * lat.nt;
    rec_len_ = BFI_PARTIAL_LEN(lat.nx);
    split_len_ = BFI_SPLIT_LEN(d_);
    launch_ = resolve_launch(ctx, lat, prec, split, launch);
    launch_.use_graph = 1;
    if (!mc_block_ok(launch_.block))
        return fail(BFI_EINVAL, "block must be 64, 128, 256, 512 or 1024 (got %d)", launch_.block);
    if (launch_.samples_per_thread < 1 || launch_.samples_per_thread > (1 << 20))
        return fail(BFI_EINVAL, "samples_per_thread out of range");
    chunk_ = static_cast<uint64_t>(launch_.samples_per_thread) * launch_.block;
    if (chunk_ > 0x7FFFFFFFull)
        return fail(BFI_EINVAL, "samples per work item exceed 2^31");
    LaunchSpec spec{prec, launch_.block, split ? 1 : 0, 1, 0, lat.observable, lat.antithetic};
    KernelInfo info{};
    BFI_HIP(kernel_info(lat.nx, lat.nt, spec, &info));
    resident_blocks_ = static_cast<uint64_t>(std::max(info.blocks_per_cu, 1)) *
                       std::max(ctx->cu_count, 1);
    BFI_HIP(grow_pinned(&h_params_, &cap_params_, 0, 1));
    BFI_HIP(grow_device(&d_params_, &cap_dparams_, 1));
    BFI_HIP(grow_device(&d_head_, &cap_head_, 1));
    count_ = 0;
    return BFI_OK;
}

bfi_status ResidentEval::reserve(size_t count)
{
    if (count <= cap_h_sub_ && h_id_)
        return BFI_OK;
    const size_t n = std::max<size_t>({count, 2 * cap_h_sub_, 64});
    const size_t d = static_cast<size_t>(d_);
    size_t c = cap_h_sub_;
    BFI_HIP(grow_pinned(&h_id_, &c, count_, n));
    c = cap_h_sub_;
    BFI_HIP(grow_pinned(&h_n_, &c, count_, n));
    c = cap_h_sub_;
    BFI_HIP(grow_pinned(&h_off_, &c, count_, n));
    c = cap_h_sub_ * d;
    BFI_HIP(grow_pinned(&h_lo_, &c, count_ * d, n * d));
    c = cap_h_sub_ * d;
    BFI_HIP(grow_pinned(&h_hi_, &c, count_ * d, n * d));
    cap_h_sub_ = n;
    return BFI_OK;
}

bfi_status ResidentEval::stage(size_t count)
{
    count_ = 0;
    BFI_TRY(reserve(count));
    count_ = count;
    return BFI_OK;
}

bfi_status ResidentEval::push(uint64_t id, uint64_t offset, uint64_t n, const double *lo,
                              const double *hi)
{
    if (count_ + 1 > cap_h_sub_ || !h_id_)
        BFI_TRY(reserve(count_ + 1));
    const size_t d = static_cast<size_t>(d_);
    h_id_[count_] = id;
    h_off_[count_] = offset;
    h_n_[count_] = n;
    std::memcpy(h_lo_ + count_ * d, lo, d * sizeof(double));
    std::memcpy(h_hi_ + count_ * d, hi, d * sizeof(double));
    ++count_;
    return BFI_OK;
}

bfi_status ResidentEval::run(uint64_t seed, double *rec_out, double *split_out, double *device_ms)
{
    BFI_TRY(prepare(seed));
    BFI_TRY(launch());
    return finish(rec_out, split_out, device_ms);
}

bfi_status ResidentEval::prepare(uint64_t seed)
{
    prepared_ = 0;
    const size_t nsub = count_;
    if (nsub == 0)
        return BFI_OK;
    if (nsub >= 0xFFFFFFFFull)
        return fail(BFI_EINVAL, "too many entries in one list");
    const size_t d = static_cast<size_t>(d_);
    uint64_t nitems = 0;
    for (size_t s = 0; s < nsub; ++s) {
        nitems += h_n_[s] / chunk_ + (h_n_[s] % chunk_ != 0);
        if (nitems > 0x7FFFFFFFull)
            return fail(BFI_EINVAL, "more than 2^31 work items; raise samples_per_thread");
    }
    // device capacity (a buffer that moves is a new argument of its nodes, which
    // the graph update below takes like any other)
    BFI_HIP(grow_device(&d_id_, &cap_d_sub_[0], nsub));
    BFI_HIP(grow_device(&d_n_, &cap_d_sub_[1], nsub));
    BFI_HIP(grow_device(&d_off_, &cap_d_sub_[2], nsub));
    BFI_HIP(grow_device(&d_sub_first_, &cap_d_sub_[3], nsub + 1));
    BFI_HIP(grow_device(&d_lo_, &cap_d_map_[0], nsub * d));
    BFI_HIP(grow_device(&d_hi_, &cap_d_map_[1], nsub * d));
    BFI_HIP(grow_device(&d_base64_, &cap_d_map_[2], nsub * d));
    BFI_HIP(grow_device(&d_scale64_, &cap_d_map_[3], nsub * d));
    BFI_HIP(grow_device(&d_base32_, &cap_d_map_[4], nsub * d));
    BFI_HIP(grow_device(&d_scale32_, &cap_d_map_[5], nsub * d));
    BFI_HIP(grow_device(&d_items_, &cap_d_items_[0], nitems));
    BFI_HIP(grow_device(&d_item_rec_, &cap_d_items_[1], nitems * rec_len_));
    BFI_HIP(grow_device(&d_sub_rec_, &cap_d_sub_[4], nsub * rec_len_));
    // pinned room for the records only when they come back (at a million
    // leaves that is hundreds of megabytes, slow to pin)
    if (copy_records_)
        BFI_HIP(grow_pinned(&h_rec_, &cap_h_rec_, 0, nsub * rec_len_));
    if (split_) {
        BFI_HIP(grow_device(&d_item_split_, &cap_d_items_[2], nitems * 2 * d));
        BFI_HIP(grow_device(&d_sub_split_, &cap_d_sub_[5], nsub * split_len_));
        if (copy_records_)
            BFI_HIP(grow_pinned(&h_split_, &cap_h_split_, 0, nsub * split_len_));
    }
    *h_params_ = EvalParams{d_base64_, d_scale64_, d_base32_, d_scale32_, d_id_, d_off_,
                            make_coef(lat_), static_cast<uint32_t>(seed),
                            static_cast<uint32_t>(seed >> 32)};

    hipStream_t st = ctx_->stream;
    BFI_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    bfi_status s = enqueue(nsub, nitems, st);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(st, &g);
    if (s != BFI_OK) {
        if (g)
            (void)hipGraphDestroy(g);
        return s;
    }
    BFI_HIP(e);
    if (exec_) {
        hipGraphNode_t bad = nullptr;
        hipGraphExecUpdateResult why = hipGraphExecUpdateSuccess;
        e = hipGraphExecUpdate(exec_, g, &bad, &why);
        if (e != hipSuccess || why != hipGraphExecUpdateSuccess) {
            (void)hipGetLastError();  // a refused update is not an error of the call
            (void)hipGraphExecDestroy(exec_);
            exec_ = nullptr;
        } else {
            ++updates_;
        }
    }
    if (!exec_) {
        e = hipGraphInstantiate(&exec_, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            exec_ = nullptr;
            (void)hipGraphDestroy(g);
            return hip_fail(e, "hipGraphInstantiate");
        }
        ++instantiations_;
    }
    (void)hipGraphDestroy(g);
    if (!ev_start_) {
        BFI_HIP(hipEventCreate(&ev_start_));
        BFI_HIP(hipEventCreate(&ev_stop_));
    }
    prepared_ = nsub;
    return BFI_OK;
}

bfi_status ResidentEval::launch()
{
    if (prepared_ == 0)
        return BFI_OK;
    hipStream_t st = ctx_->stream;
    BFI_HIP(hipEventRecord(ev_start_, st));
    BFI_HIP(hipGraphLaunch(exec_, st));
    BFI_HIP(hipEventRecord(ev_stop_, st));
    launched_ = true;
    return BFI_OK;
}

bfi_status ResidentEval::finish(double *rec_out, double *split_out, double *device_ms)
{
    if (device_ms)
        *device_ms = 0.0;
    const size_t nsub = prepared_;
    if (nsub == 0) {
        count_ = 0;
        return BFI_OK;
    }
    if (!launched_)
        return fail(BFI_EINVAL, "finish before launch");
    launched_ = false;
    prepared_ = 0;
    BFI_HIP(hipEventSynchronize(ev_stop_));
    if (device_ms) {
        float ms = 0.0f;
        BFI_HIP(hipEventElapsedTime(&ms, ev_start_, ev_stop_));
        *device_ms = ms;
    }
    if (rec_out || split_out)
        if (!copy_records_)
            return fail(BFI_EINVAL, "records kept on the device");
    if (rec_out)
        std::memcpy(rec_out, h_rec_, nsub * rec_len_ * sizeof(double));
    if (split_ && split_out)
        std::memcpy(split_out, h_split_, nsub * split_len_ * sizeof(double));
    count_ = 0;
    return BFI_OK;
}

bfi_status ResidentEval::enqueue(size_t nsub, uint64_t nitems, hipStream_t st)
{
    const size_t d = static_cast<size_t>(d_);
    BFI_HIP(hipMemcpyAsync(d_id_, h_id_, nsub * 8, hipMemcpyHostToDevice, st));
    BFI_HIP(hipMemcpyAsync(d_n_, h_n_, nsub * 8, hipMemcpyHostToDevice, st));
    BFI_HIP(hipMemcpyAsync(d_off_, h_off_, nsub * 8, hipMemcpyHostToDevice, st));
    BFI_HIP(hipMemcpyAsync(d_lo_, h_lo_, nsub * d * 8, hipMemcpyHostToDevice, st));
    BFI_HIP(hipMemcpyAsync(d_hi_, h_hi_, nsub * d * 8, hipMemcpyHostToDevice, st));
    BFI_HIP(hipMemcpyAsync(d_params_, h_params_, sizeof(EvalParams), hipMemcpyHostToDevice, st));
    BuildArgs ba{d_lo_, d_hi_, d_n_, d_sub_first_, d_base64_, d_scale64_, d_base32_, d_scale32_,
                 d_items_, d_params_, d_item_rec_, chunk_, static_cast<uint32_t>(nsub), d_,
                 rec_len_};
    BFI_HIP(launch_build_items(ba, st));
    BFI_HIP(launch_reset_head(d_head_, st));
    LaunchSpec spec{prec_, launch_.block, split_ ? 1 : 0, 1,
                    static_cast<uint32_t>(std::min<uint64_t>(resident_blocks_, nitems)),
                    lat_.observable, lat_.antithetic};
    McArgs a{};
    a.items = d_items_;
    a.item_split = split_ ? d_item_split_ : nullptr;
    a.queue_head = d_head_;
    a.nitems = static_cast<uint32_t>(nitems);
    a.samples_per_thread = static_cast<uint32_t>(launch_.samples_per_thread);
    BFI_HIP(launch_mc(lat_.nx, lat_.nt, spec, a, st));
    MergeArgs m{};
    m.item_rec = d_item_rec_;
    m.item_split = split_ ? d_item_split_ : nullptr;
    m.sub_first = d_sub_first_;
    m.sub_rec = d_sub_rec_;
    m.sub_split = split_ ? d_sub_split_ : nullptr;
    m.nsub = static_cast<uint32_t>(nsub);
    m.nx = lat_.nx;
    m.d = d_;
    BFI_HIP(launch_merge(m, st));
    if (!copy_records_)
        return BFI_OK;
    BFI_HIP(hipMemcpyAsync(h_rec_, d_sub_rec_, nsub * rec_len_ * 8, hipMemcpyDeviceToHost, st));
    if (split_)
        BFI_HIP(hipMemcpyAsync(h_split_, d_sub_split_, nsub * split_len_ * 8,
                               hipMemcpyDeviceToHost, st));
    return BFI_OK;
}

}  // namespace bfi
