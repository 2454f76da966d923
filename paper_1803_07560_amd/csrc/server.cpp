// Continuous-batching request server.
//
// A request is one correlation estimate: lattice and parameters, precision,
// seed, a box [-B, B]^d split uniformly into 2^k subvolumes and a sample budget.
// At submission it is validated and cut into work items of a fixed size per
// (lattice shape, precision); its device state (point maps, ids, offsets,
// parameters and one partial record per item) is allocated when it is
// admitted, which happens in arrival order while the memory budget and the
// request slots allow.  A worker thread runs scheduling steps: every admitted
// request contributes an equal share of the step's evaluation target (at least
// `chunks_per_step` items) from its remaining items, the step's items are
// grouped by (shape, precision) and each group is drained by one persistent
// kernel through a device queue, the groups on separate streams so kernels of
// different shapes overlap on the chip; requests that finish are merged on
// the device, finalized on the host and released.  Because an item's record
// depends only on its own request (fixed item size and block reduction order),
// a request's result is bit-identical whether it runs alone or mixed with others.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "runtime.h"

using namespace bfi;

namespace {

using Clock = std::chrono::steady_clock;

enum class State { Pending, Admitted, Done, Cancelled, Failed };

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Request {
    uint64_t ticket = 0;
    bfi_request req{};
    int d = 0, nx = 0, rec_len = 0;
    SubList subs;
    std::vector<WorkItem> items;      // device pointers filled at admission
    std::vector<uint32_t> sub_first;  // nsub + 1 prefix of items per subvolume
    size_t next_item = 0, done_items = 0, inflight = 0;
    bfi_launch launch{};  // fixed per (shape, precision) for the server's lifetime
    uint32_t grid = 0;    // persistent grid for that launch
    // one device allocation, carved into the pieces below
    void *dmem = nullptr;
    size_t bytes = 0;
    EvalParams *d_params = nullptr;
    double *d_item_rec = nullptr, *d_sub_rec = nullptr;
    uint32_t *d_sub_first = nullptr;
    State state = State::Pending;
    bool cancel = false;
    bfi_status status = BFI_OK;
    std::string message;
    bfi_result result{};
    Clock::time_point t_submit, t_done;
};

// Byte layout of a request's device state: the parts uploaded at admission
// first (one contiguous image of `upload` bytes), then the records.
struct Layout {
    size_t params, base64, scale64, base32, scale32, ids, offsets, sub_first, upload, item_rec,
        sub_rec, total;
};

Layout layout_of(size_t nsub, int d, size_t nitems, int rec_len)
{
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    L.params = take(sizeof(EvalParams));
    L.base64 = take(nsub * d * 8);
    L.scale64 = take(nsub * d * 8);
    L.base32 = take(nsub * d * 4);
    L.scale32 = take(nsub * d * 4);
    L.ids = take(nsub * 8);
    L.offsets = take(nsub * 8);
    L.sub_first = take((nsub + 1) * 4);
    L.upload = o;
    L.item_rec = take(nitems * rec_len * 8);
    L.sub_rec = take(nsub * rec_len * 8);
    L.total = o;
    return L;
}

// Device blocks come in power-of-two sizes from 64 KiB: a finished request's
// block is kept for the next request of its size class instead of being freed,
// so admission rarely calls hipMalloc; memory is accounted by block size.
size_t block_size(size_t bytes)
{
    size_t c = size_t(64) << 10;
    while (c < bytes)
        c <<= 1;
    return c;
}

bool terminal(State s) { return s == State::Done || s == State::Cancelled || s == State::Failed; }

}  // namespace

struct bfi_server {
    bfi_context *ctx = nullptr;
    bfi_server_config cfg{};
    std::mutex mu;
    std::condition_variable work_cv, done_cv;
    std::thread worker;
    bool stop = false;
    uint64_t next_ticket = 1;
    std::deque<uint64_t> pending;
    std::vector<uint64_t> admitted;  // in admission order
    size_t rr = 0;                   // round-robin start of the next step
    std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
    uint64_t used_bytes = 0;
    bfi_server_stats stats{};
    static constexpr int kStreams = 4;
    hipStream_t stream = nullptr;              // copies, merges, first group
    hipStream_t group_streams[kStreams] = {};  // group g runs on group_streams[g % 4]
    hipEvent_t staged = nullptr;               // step items copied to the device
    // step buffer: kMaxGroups queue heads (zeros, copied with every step's
    // items, so no kernel resets them), then the step's work items
    static constexpr int kMaxGroups = 64;
    static constexpr size_t kHeadBytes = 256;
    char *d_step = nullptr, *h_step = nullptr;
    size_t step_cap = 0;  // work items
    std::map<TuneKey, std::pair<bfi_launch, uint32_t>> shapes;  // launch and grid
    // cached device blocks by size class, and their total
    std::map<size_t, std::vector<void *>> pool;
    size_t pool_bytes = 0;
    // pinned staging: admission images, and records of finished requests
    char *h_stage = nullptr, *h_done = nullptr;
    size_t stage_cap = 0, stage_used = 0, done_cap = 0;
};

namespace {

// Launch shape and persistent grid for (nx, nt, prec, observable, pairs); fixed
// for the server's lifetime so item sizes (and therefore results) never depend on
// the mix.
bfi_status shape_launch(bfi_server *srv, const bfi_lattice &lat, int prec, bfi_launch *l,
                        uint32_t *grid)
{
    const TuneKey key{lat.nx, lat.nt, prec, lat.antithetic, lat.observable};
    auto it = srv->shapes.find(key);
    if (it == srv->shapes.end()) {
        bfi_launch r = resolve_launch(srv->ctx, lat, prec, false, nullptr);
        const int cap = srv->cfg.max_samples_per_thread > 0 ? srv->cfg.max_samples_per_thread : 128;
        r.samples_per_thread = std::min(r.samples_per_thread, cap);
        r.persistent = 1;
        r.use_graph = 0;
        KernelInfo info{};
        LaunchSpec spec{prec, r.block, 0, 1, 0, lat.observable, lat.antithetic};
        BFI_HIP(kernel_info(lat.nx, lat.nt, spec, &info));
        const uint32_t g =
            static_cast<uint32_t>(std::max(info.blocks_per_cu, 1) * std::max(srv->ctx->cu_count, 1));
        it = srv->shapes.emplace(key, std::make_pair(r, g)).first;
    }
    *l = it->second.first;
    *grid = it->second.second;
    return BFI_OK;
}

void pool_release(bfi_server *srv, size_t keep)
{
    for (auto it = srv->pool.rbegin(); it != srv->pool.rend() && srv->pool_bytes > keep; ++it) {
        while (!it->second.empty() && srv->pool_bytes > keep) {
            (void)hipFree(it->second.back());
            it->second.pop_back();
            srv->pool_bytes -= it->first;
        }
    }
}

hipError_t pool_take(bfi_server *srv, size_t bytes, void **out)
{
    auto it = srv->pool.find(bytes);
    if (it != srv->pool.end() && !it->second.empty()) {
        *out = it->second.back();
        it->second.pop_back();
        srv->pool_bytes -= bytes;
        return hipSuccess;
    }
    hipError_t e = hipMalloc(out, bytes);
    if (e == hipErrorOutOfMemory && srv->pool_bytes > 0) {
        (void)hipGetLastError();
        pool_release(srv, 0);
        e = hipMalloc(out, bytes);
    }
    return e;
}

void free_device(bfi_server *srv, Request *r)
{
    if (r->dmem) {
        // no kernel of the request is in flight here (steps are waited for)
        srv->pool[r->bytes].push_back(r->dmem);
        srv->pool_bytes += r->bytes;
        r->dmem = nullptr;
        srv->used_bytes -= r->bytes;
        // the cache holds at most the budget's worth of blocks
        if (srv->pool_bytes > srv->cfg.memory_budget)
            pool_release(srv, srv->cfg.memory_budget / 2);
    }
}

// Pinned host buffer of at least `bytes`; its old contents are dropped.
hipError_t grow_pinned(char **p, size_t *cap, size_t bytes)
{
    if (*cap >= bytes && *p)
        return hipSuccess;
    if (*p)
        (void)hipHostFree(*p);
    *p = nullptr;
    *cap = 0;
    const size_t n = std::max(bytes, size_t(1) << 20);
    hipError_t e = hipHostMalloc(reinterpret_cast<void **>(p), n, hipHostMallocDefault);
    if (e == hipSuccess)
        *cap = n;
    return e;
}

void finish(bfi_server *srv, Request *r, State s, bfi_status st, const std::string &msg)
{
    free_device(srv, r);
    r->state = s;
    r->status = st;
    r->message = msg;
    r->t_done = Clock::now();
    if (s == State::Done)
        ++srv->stats.completed;
    srv->done_cv.notify_all();
}

// Allocate and upload a request's device state.  Called with the lock held.
// The uploaded parts are written into pinned staging as one image and copied
// asynchronously on the server stream, ahead of any step that uses them.
bfi_status admit_one(bfi_server *srv, Request *r)
{
    const size_t nsub = r->subs.size();
    const int d = r->d;
    const Layout L = layout_of(nsub, d, r->items.size(), r->rec_len);
    const size_t bytes = block_size(L.total);
    BFI_HIP(pool_take(srv, bytes, &r->dmem));
    r->bytes = bytes;
    srv->used_bytes += bytes;
    char *base = static_cast<char *>(r->dmem);
    if (srv->stage_used + L.upload > srv->stage_cap) {
        // earlier images may still be in flight: wait for them before reusing
        BFI_HIP(hipStreamSynchronize(srv->stream));
        srv->stage_used = 0;
        BFI_HIP(grow_pinned(&srv->h_stage, &srv->stage_cap, L.upload));
    }
    char *img = srv->h_stage + srv->stage_used;
    srv->stage_used += align_up(L.upload);
    auto *b64 = reinterpret_cast<double *>(img + L.base64);
    auto *s64 = reinterpret_cast<double *>(img + L.scale64);
    auto *b32 = reinterpret_cast<float *>(img + L.base32);
    auto *s32 = reinterpret_cast<float *>(img + L.scale32);
    for (size_t i = 0; i < nsub * d; ++i) {
        s64[i] = (r->subs.hi[i] - r->subs.lo[i]) * 0x1p-32;
        b64[i] = r->subs.lo[i] + 0.5 * s64[i];
        s32[i] = static_cast<float>(s64[i]);
        b32[i] = static_cast<float>(b64[i]);
    }
    const EvalParams P{reinterpret_cast<double *>(base + L.base64),
                       reinterpret_cast<double *>(base + L.scale64),
                       reinterpret_cast<float *>(base + L.base32),
                       reinterpret_cast<float *>(base + L.scale32),
                       reinterpret_cast<uint64_t *>(base + L.ids),
                       reinterpret_cast<uint64_t *>(base + L.offsets),
                       make_coef(r->req.lat),
                       static_cast<uint32_t>(r->req.seed),
                       static_cast<uint32_t>(r->req.seed >> 32)};
    std::memcpy(img + L.params, &P, sizeof(P));
    std::memcpy(img + L.ids, r->subs.id.data(), nsub * 8);
    std::memcpy(img + L.offsets, r->subs.offset.data(), nsub * 8);
    std::memcpy(img + L.sub_first, r->sub_first.data(), (nsub + 1) * 4);
    BFI_HIP(hipMemcpyAsync(base, img, L.upload, hipMemcpyHostToDevice, srv->stream));
    r->d_params = reinterpret_cast<EvalParams *>(base + L.params);
    r->d_item_rec = reinterpret_cast<double *>(base + L.item_rec);
    r->d_sub_first = reinterpret_cast<uint32_t *>(base + L.sub_first);
    r->d_sub_rec = reinterpret_cast<double *>(base + L.sub_rec);
    for (size_t i = 0; i < r->items.size(); ++i) {
        r->items[i].params = r->d_params;
        r->items[i].rec = r->d_item_rec + i * r->rec_len;
    }
    r->state = State::Admitted;
    return BFI_OK;
}

void admit(bfi_server *srv)
{
    while (!srv->pending.empty() &&
           static_cast<int32_t>(srv->admitted.size()) < srv->cfg.max_requests) {
        Request *r = srv->reqs.at(srv->pending.front()).get();
        const Layout L = layout_of(r->subs.size(), r->d, r->items.size(), r->rec_len);
        if (srv->used_bytes + block_size(L.total) > srv->cfg.memory_budget)
            break;  // first come, first served: wait for memory to free up
        srv->pending.pop_front();
        bfi_status s = admit_one(srv, r);
        if (s != BFI_OK) {
            finish(srv, r, State::Failed, s, bfi_last_error());
            continue;
        }
        srv->admitted.push_back(r->ticket);
    }
}

// Merge and finalize requests whose items are all done; release cancelled ones.
// Every finished request's merge and record copy is enqueued first, then one
// wait covers them all.
void complete(bfi_server *srv)
{
    std::vector<uint64_t> keep;
    std::vector<Request *> ready;
    size_t bytes = 0;
    for (uint64_t t : srv->admitted) {
        Request *r = srv->reqs.at(t).get();
        if (r->cancel && r->inflight == 0) {
            finish(srv, r, State::Cancelled, BFI_ECANCELLED, "cancelled");
            continue;
        }
        if (r->cancel || r->done_items < r->items.size()) {
            keep.push_back(t);
            continue;
        }
        ready.push_back(r);
        bytes += r->subs.size() * r->rec_len * sizeof(double);
    }
    srv->admitted.swap(keep);
    if (ready.empty())
        return;
    TraceRange trace("server: merge and finalize finished requests");
    hipError_t e = grow_pinned(&srv->h_done, &srv->done_cap, bytes);
    std::vector<double *> host(ready.size());
    size_t at = 0;
    for (size_t i = 0; i < ready.size() && e == hipSuccess; ++i) {
        Request *r = ready[i];
        MergeArgs m{};
        m.item_rec = r->d_item_rec;
        m.sub_first = r->d_sub_first;
        m.sub_rec = r->d_sub_rec;
        m.nsub = static_cast<uint32_t>(r->subs.size());
        m.nx = r->nx;
        m.d = r->d;
        host[i] = reinterpret_cast<double *>(srv->h_done + at);
        const size_t n = r->subs.size() * r->rec_len * sizeof(double);
        at += n;
        e = launch_merge(m, srv->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(host[i], r->d_sub_rec, n, hipMemcpyDeviceToHost, srv->stream);
    }
    if (e == hipSuccess)
        e = hipStreamSynchronize(srv->stream);
    if (e != hipSuccess) {
        for (Request *r : ready)
            finish(srv, r, State::Failed, BFI_EDEVICE, hipGetErrorString(e));
        return;
    }
    for (size_t i = 0; i < ready.size(); ++i) {
        Request *r = ready[i];
        const double *sub = host[i];
        const size_t len = r->subs.size() * r->rec_len;
        // records that overflowed (an action beyond the range of the precision:
        // every subvolume has samples, so even the shift is finite in a sound
        // record) fail this request only
        bool finite = true;
        for (size_t k = 0; k < len && finite; ++k)
            finite = std::isfinite(sub[k]);
        if (!finite) {
            finish(srv, r, State::Failed, BFI_EDEVICE, "non-finite sums");
            continue;
        }
        bfi_status s = finalize_records(r->nx, r->d, r->subs.size(), r->subs.lo.data(),
                                        r->subs.hi.data(), sub, &r->result,
                                        r->req.lat.antithetic ? 2 : 1);
        finite = std::isfinite(r->result.log_Z);
        for (int k = 0; k < r->nx; ++k)
            finite = finite && std::isfinite(r->result.C[k]);
        if (s != BFI_OK)
            finish(srv, r, State::Failed, s, bfi_last_error());
        else if (!finite)
            finish(srv, r, State::Failed, BFI_EDEVICE, "non-finite sums");
        else
            finish(srv, r, State::Done, BFI_OK, "");
    }
}

struct StepEntry {
    Request *r;
    size_t first, count;
};

// One scheduling step.  Called without the lock; entries were reserved under it.
bfi_status run_step(bfi_server *srv, const std::vector<StepEntry> &entries)
{
    struct Group {
        bfi_lattice lat;
        int prec;
        size_t off, count;
        bfi_launch launch;
        uint32_t grid;
    };
    std::vector<Group> groups;
    size_t total = 0;
    // group entries by (shape, precision, observable, pairs), keeping their order
    std::vector<bool> used(entries.size(), false);
    for (size_t i = 0; i < entries.size(); ++i) {
        if (used[i])
            continue;
        const bfi_request &q = entries[i].r->req;
        Group g{q.lat, q.prec, total, 0, entries[i].r->launch, entries[i].r->grid};
        for (size_t j = i; j < entries.size(); ++j) {
            const bfi_request &o = entries[j].r->req;
            if (used[j] || o.lat.nx != q.lat.nx || o.lat.nt != q.lat.nt || o.prec != q.prec ||
                o.lat.observable != q.lat.observable || o.lat.antithetic != q.lat.antithetic)
                continue;
            used[j] = true;
            const StepEntry &e = entries[j];
            std::memcpy(srv->h_step + bfi_server::kHeadBytes + total * sizeof(WorkItem),
                        e.r->items.data() + e.first, e.count * sizeof(WorkItem));
            total += e.count;
            g.count += e.count;
        }
        groups.push_back(g);
    }
    if (groups.size() > static_cast<size_t>(bfi_server::kMaxGroups))
        return fail(BFI_EDEVICE, "too many shape groups in one step");
    // the copy carries the zeroed queue heads and the items
    BFI_HIP(hipMemcpyAsync(srv->d_step, srv->h_step,
                           bfi_server::kHeadBytes + total * sizeof(WorkItem),
                           hipMemcpyHostToDevice, srv->stream));
    BFI_HIP(hipEventRecord(srv->staged, srv->stream));
    const int nstreams = static_cast<int>(std::min<size_t>(groups.size(), bfi_server::kStreams));
    for (int k = 1; k < nstreams; ++k)
        BFI_HIP(hipStreamWaitEvent(srv->group_streams[k], srv->staged, 0));
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        const Group &g = groups[gi];
        hipStream_t st = srv->group_streams[gi % bfi_server::kStreams];
        McArgs a{};
        a.items = reinterpret_cast<const WorkItem *>(srv->d_step + bfi_server::kHeadBytes) + g.off;
        a.item_split = nullptr;
        a.queue_head = reinterpret_cast<uint32_t *>(srv->d_step) + gi;
        a.nitems = static_cast<uint32_t>(g.count);
        a.samples_per_thread = static_cast<uint32_t>(g.launch.samples_per_thread);
        LaunchSpec spec{g.prec, g.launch.block, 0, 1,
                        static_cast<uint32_t>(std::min<size_t>(g.grid, g.count)),
                        g.lat.observable, g.lat.antithetic};
        BFI_HIP(launch_mc(g.lat.nx, g.lat.nt, spec, a, st));
    }
    for (int k = 0; k < nstreams; ++k)
        BFI_HIP(hipStreamSynchronize(srv->group_streams[k]));
    return BFI_OK;
}

void worker_loop(bfi_server *srv)
{
    (void)hipSetDevice(srv->ctx->device);
    roctxNameOsThread("bfi server worker");
    std::unique_lock<std::mutex> lk(srv->mu);
    for (;;) {
        admit(srv);
        complete(srv);
        std::vector<StepEntry> entries;
        const size_t na = srv->admitted.size();
        size_t budget = srv->step_cap;
        size_t active = 0;
        for (uint64_t t : srv->admitted) {
            const Request *r = srv->reqs.at(t).get();
            active += !r->cancel && r->next_item < r->items.size();
        }
        const uint64_t step_evals = srv->cfg.step_evals ? srv->cfg.step_evals : uint64_t(1) << 25;
        for (size_t k = 0; k < na && budget > 0; ++k) {
            Request *r = srv->reqs.at(srv->admitted[(srv->rr + k) % na]).get();
            if (r->cancel || r->next_item >= r->items.size())
                continue;
            // equal share of the step's evaluations, at least chunks_per_step items
            // (an item of antithetic pairs makes two evaluations per sample index)
            const uint64_t chunk = static_cast<uint64_t>(r->launch.samples_per_thread) *
                                   r->launch.block * (r->req.lat.antithetic ? 2 : 1);
            const uint64_t share = step_evals / std::max<size_t>(active, 1);
            const size_t quota = std::max<size_t>(static_cast<size_t>(srv->cfg.chunks_per_step),
                                                  static_cast<size_t>((share + chunk - 1) / chunk));
            const size_t take = std::min({quota, r->items.size() - r->next_item, budget});
            entries.push_back({r, r->next_item, take});
            r->next_item += take;
            r->inflight += take;
            budget -= take;
        }
        if (na)
            srv->rr = (srv->rr + 1) % na;
        if (entries.empty()) {
            if (srv->stop)
                break;
            srv->work_cv.wait_for(lk, std::chrono::milliseconds(20));
            continue;
        }
        lk.unlock();
        const auto t0 = Clock::now();
        // a failed step (an exception included) fails its requests, not the server
        bfi_status s = guarded([&]() -> bfi_status {
            TraceRange trace("server: step");
            return run_step(srv, entries);
        });
        const auto t1 = Clock::now();
        std::string msg = s == BFI_OK ? "" : bfi_last_error();
        lk.lock();
        srv->stats.busy_seconds += std::chrono::duration<double>(t1 - t0).count();
        ++srv->stats.steps;
        for (const StepEntry &e : entries) {
            e.r->inflight -= e.count;
            if (s == BFI_OK) {
                e.r->done_items += e.count;
                for (size_t i = e.first; i < e.first + e.count; ++i)
                    srv->stats.evals +=
                        e.r->items[i].count * static_cast<uint64_t>(e.r->req.lat.antithetic ? 2 : 1);
            } else if (!terminal(e.r->state)) {
                e.r->cancel = true;  // released by complete(); reported as failed below
                e.r->status = s;
                e.r->message = msg;
            }
        }
        if (s != BFI_OK) {
            for (uint64_t t : srv->admitted) {
                Request *r = srv->reqs.at(t).get();
                if (r->cancel && r->status != BFI_OK && r->inflight == 0)
                    finish(srv, r, State::Failed, r->status, r->message);
            }
            std::vector<uint64_t> keep;
            for (uint64_t t : srv->admitted)
                if (!terminal(srv->reqs.at(t)->state))
                    keep.push_back(t);
            srv->admitted.swap(keep);
        }
    }
    // shutdown: release everything still resident
    for (uint64_t t : srv->admitted)
        free_device(srv, srv->reqs.at(t).get());
    srv->admitted.clear();
}

bfi_status take_result(bfi_server *srv, uint64_t ticket, bfi_result *out, int32_t *done,
                       double *latency_s)
{
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end())
        return fail(BFI_ENOTFOUND, "unknown ticket %llu", static_cast<unsigned long long>(ticket));
    Request *r = it->second.get();
    if (!terminal(r->state)) {
        *done = 0;
        return BFI_OK;
    }
    *done = 1;
    if (out)
        *out = r->result;
    if (latency_s)
        *latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
    const bfi_status s = r->status;
    const std::string msg = r->message;
    srv->reqs.erase(it);
    if (s != BFI_OK)
        return fail(s, "%s", msg.c_str());
    return BFI_OK;
}

}  // namespace

extern "C" {

bfi_status bfi_server_create(bfi_context *ctx, const bfi_server_config *cfg, bfi_server **out)
{
    return guarded([&]() -> bfi_status {
        if (!ctx || !cfg || !out)
            return fail(BFI_EINVAL, "arguments must be non-NULL");
        if (cfg->max_requests < 1 || cfg->chunks_per_step < 1 || cfg->max_pending < 0 ||
            cfg->memory_budget == 0 || cfg->max_samples_per_thread < 0 ||
            cfg->max_samples_per_thread > (1 << 20))
            return fail(BFI_EINVAL, "bad server configuration");
        BFI_HIP(hipSetDevice(ctx->device));
        auto srv = std::make_unique<bfi_server>();
        srv->ctx = ctx;
        srv->cfg = *cfg;
        // room for every admitted request's minimum share plus the step target in items
        srv->step_cap = static_cast<size_t>(cfg->max_requests) * cfg->chunks_per_step + 65536;
        BFI_HIP(hipStreamCreateWithFlags(&srv->stream, hipStreamNonBlocking));
        srv->group_streams[0] = srv->stream;
        for (int k = 1; k < bfi_server::kStreams; ++k)
            BFI_HIP(hipStreamCreateWithFlags(&srv->group_streams[k], hipStreamNonBlocking));
        BFI_HIP(hipEventCreateWithFlags(&srv->staged, hipEventDisableTiming));
        static_assert(bfi_server::kMaxGroups * sizeof(uint32_t) <= bfi_server::kHeadBytes,
                      "queue heads fit the step buffer's head area");
        const size_t step_bytes = bfi_server::kHeadBytes + srv->step_cap * sizeof(WorkItem);
        hipError_t e = hipMalloc(reinterpret_cast<void **>(&srv->d_step), step_bytes);
        if (e == hipSuccess)
            e = hipHostMalloc(reinterpret_cast<void **>(&srv->h_step), step_bytes,
                              hipHostMallocDefault);
        if (e == hipSuccess)
            std::memset(srv->h_step, 0, bfi_server::kHeadBytes);  // the heads stay zero
        if (e != hipSuccess) {
            if (srv->d_step)
                (void)hipFree(srv->d_step);
            if (srv->h_step)
                (void)hipHostFree(srv->h_step);
            for (int k = 0; k < bfi_server::kStreams; ++k)
                (void)hipStreamDestroy(srv->group_streams[k]);
            (void)hipEventDestroy(srv->staged);
            return hip_fail(e, "server buffers");
        }
        bfi_server *p = srv.release();
        p->worker = std::thread(worker_loop, p);
        *out = p;
        return BFI_OK;
    });
}

bfi_status bfi_server_submit(bfi_server *srv, const bfi_request *req, uint64_t *ticket)
{
    return guarded([&]() -> bfi_status {
        if (!srv || !req || !ticket)
            return fail(BFI_EINVAL, "arguments must be non-NULL");
        BFI_TRY(check_lattice(&req->lat));
        if (!known_precision(req->prec))
            return fail(BFI_EINVAL, "unknown precision");
        if (!(req->box > 0) || !std::isfinite(req->box))
            return fail(BFI_EINVAL, "box must be positive and finite");
        if (req->split_log2 < 0 || req->split_log2 > 20)
            return fail(BFI_EINVAL, "split_log2 must be in [0, 20]");
        // the budget counts integrand evaluations: two per antithetic pair
        const uint64_t per = req->lat.antithetic ? 2 : 1;
        if (req->budget / per < 2 * (uint64_t(1) << req->split_log2))
            return fail(BFI_EINVAL, "budget must give every subvolume at least 2 samples");

        auto r = std::make_unique<Request>();
        r->req = *req;
        r->nx = req->lat.nx;
        r->d = req->lat.nx * req->lat.nt;
        r->rec_len = BFI_PARTIAL_LEN(r->nx);
        std::vector<double> lo(r->d, -req->box), hi(r->d, req->box);
        r->subs = uniform_split(r->d, lo.data(), hi.data(), req->split_log2, req->budget / per);
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            BFI_TRY(shape_launch(srv, req->lat, req->prec, &r->launch, &r->grid));
        }
        const uint64_t chunk = static_cast<uint64_t>(r->launch.samples_per_thread) * r->launch.block;
        // size the request before building it: work items and device state
        uint64_t nitems = 0;
        for (size_t s = 0; s < r->subs.size(); ++s) {
            nitems += r->subs.n[s] / chunk + (r->subs.n[s] % chunk != 0);
            if (nitems > 0x7FFFFFFFull)
                return fail(BFI_EINVAL, "request needs more than 2^31 work items");
        }
        {
            const Layout need = layout_of(r->subs.size(), r->d, static_cast<size_t>(nitems),
                                          r->rec_len);
            std::lock_guard<std::mutex> lk(srv->mu);
            if (block_size(need.total) > srv->cfg.memory_budget) {
                ++srv->stats.rejected;
                return fail(BFI_EBUSY,
                            "request needs a %zu-byte block of device state, budget is %llu",
                            block_size(need.total),
                            static_cast<unsigned long long>(srv->cfg.memory_budget));
            }
        }
        r->items.reserve(static_cast<size_t>(nitems));
        r->sub_first.assign(r->subs.size() + 1, 0);
        for (size_t s = 0; s < r->subs.size(); ++s) {
            r->sub_first[s] = static_cast<uint32_t>(r->items.size());
            for (uint64_t start = 0; start < r->subs.n[s]; start += chunk)
                r->items.push_back(WorkItem{nullptr, nullptr, start, static_cast<uint32_t>(s),
                                            static_cast<uint32_t>(
                                                std::min<uint64_t>(chunk, r->subs.n[s] - start))});
        }
        r->sub_first[r->subs.size()] = static_cast<uint32_t>(r->items.size());

        std::lock_guard<std::mutex> lk(srv->mu);
        if (static_cast<int32_t>(srv->pending.size()) >= srv->cfg.max_pending) {
            ++srv->stats.rejected;
            return fail(BFI_EBUSY, "pending queue full (%d)", srv->cfg.max_pending);
        }
        r->ticket = srv->next_ticket++;
        r->t_submit = Clock::now();
        *ticket = r->ticket;
        srv->pending.push_back(r->ticket);
        srv->reqs.emplace(r->ticket, std::move(r));
        ++srv->stats.submitted;
        srv->work_cv.notify_one();
        return BFI_OK;
    });
}

bfi_status bfi_server_poll(bfi_server *srv, uint64_t ticket, bfi_result *out, int32_t *done,
                           double *latency_s)
{
    return guarded([&]() -> bfi_status {
        if (!srv || !done)
            return fail(BFI_EINVAL, "arguments must be non-NULL");
        std::lock_guard<std::mutex> lk(srv->mu);
        return take_result(srv, ticket, out, done, latency_s);
    });
}

bfi_status bfi_server_wait(bfi_server *srv, uint64_t ticket, double timeout_s, bfi_result *out,
                           int32_t *done, double *latency_s)
{
    return guarded([&]() -> bfi_status {
        if (!srv || !done)
            return fail(BFI_EINVAL, "arguments must be non-NULL");
        std::unique_lock<std::mutex> lk(srv->mu);
        const auto until = Clock::now() + std::chrono::duration_cast<Clock::duration>(
                                              std::chrono::duration<double>(std::max(timeout_s, 0.0)));
        srv->done_cv.wait_until(lk, until, [&] {
            auto it = srv->reqs.find(ticket);
            return it == srv->reqs.end() || terminal(it->second->state);
        });
        return take_result(srv, ticket, out, done, latency_s);
    });
}

bfi_status bfi_server_cancel(bfi_server *srv, uint64_t ticket)
{
    return guarded([&]() -> bfi_status {
        if (!srv)
            return fail(BFI_EINVAL, "server is NULL");
        std::lock_guard<std::mutex> lk(srv->mu);
        auto it = srv->reqs.find(ticket);
        if (it == srv->reqs.end())
            return fail(BFI_ENOTFOUND, "unknown ticket");
        Request *r = it->second.get();
        if (terminal(r->state))
            return BFI_OK;
        ++srv->stats.cancelled;
        if (r->state == State::Pending) {
            srv->pending.erase(std::find(srv->pending.begin(), srv->pending.end(), ticket));
            finish(srv, r, State::Cancelled, BFI_ECANCELLED, "cancelled");
            return BFI_OK;
        }
        r->cancel = true;  // the worker releases it once no step holds its items
        srv->work_cv.notify_one();
        return BFI_OK;
    });
}

bfi_status bfi_server_stats_get(bfi_server *srv, bfi_server_stats *out)
{
    return guarded([&]() -> bfi_status {
        if (!srv || !out)
            return fail(BFI_EINVAL, "arguments must be non-NULL");
        std::lock_guard<std::mutex> lk(srv->mu);
        *out = srv->stats;
        return BFI_OK;
    });
}

bfi_status bfi_server_destroy(bfi_server *srv)
{
    return guarded([&]() -> bfi_status {
        if (!srv)
            return BFI_OK;
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            srv->stop = true;
            for (uint64_t t : srv->admitted)
                srv->reqs.at(t)->cancel = true;
            srv->pending.clear();
        }
        srv->work_cv.notify_all();
        if (srv->worker.joinable())
            srv->worker.join();
        (void)hipSetDevice(srv->ctx->device);
        for (auto &kv : srv->reqs)
            free_device(srv, kv.second.get());
        pool_release(srv, 0);
        (void)hipFree(srv->d_step);
        (void)hipHostFree(srv->h_step);
        if (srv->h_stage)
            (void)hipHostFree(srv->h_stage);
        if (srv->h_done)
            (void)hipHostFree(srv->h_done);
        for (int k = 0; k < bfi_server::kStreams; ++k)
            (void)hipStreamDestroy(srv->group_streams[k]);
        (void)hipEventDestroy(srv->staged);
        delete srv;
        return BFI_OK;
    });
}

}  // extern "C"
