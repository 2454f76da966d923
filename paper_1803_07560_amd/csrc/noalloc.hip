// bfi_eval_noalloc: bfi_eval without any allocation, for callers that cannot
// allocate device memory (code under stream capture, tight serving loops,
// harnesses that forbid hipMalloc).
//
// Everything bfi_eval keeps in a plan's buffers -- the copied subvolume list,
// the point maps, the parameter block, the work items, the item and subvolume
// records and the queue head -- lives in one file-scope device array,
// `scratch`, of kScratchBytes per device.  Its device address is taken once per
// device with hipGetSymbolAddress when a context is created on that device
// (noalloc_setup) and only that address is passed to kernels and copies: in
// host code the array's name is a host-side stand-in, not device memory.
// Point maps and work items are built on the device from the copied list
// (launch_build_items), so the host needs no staging either.  The kernels that evaluate, reduce and
// merge are bfi_eval's own, so with the same launch shape the records are the
// same bits.
//
// Every call on a device shares that device's array and leaves its contents
// there; calls that overlap in time on one device (two threads, two contexts
// on the same device) race.  The queue head is reset by a kernel before each
// evaluation; every other region is fully written before it is read.
#include <mutex>

#include "runtime.h"

namespace bfi {

namespace {

constexpr size_t kScratchBytes = BFI_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mutex;
unsigned char *g_scratch_ptr[kMaxDevices] = {};

// Offsets of the regions inside the scratch array, each 256-byte aligned.
struct Layout {
    size_t id, n, offset, lo, hi, base64, scale64, base32, scale32, params, sub_first, items,
        item_rec, item_split, sub_rec, sub_split, head, total;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

Layout layout_for(size_t nsub, int d, int rec_len, uint64_t nitems, bool split)
{
    Layout L{};
    size_t at = 0;
    auto take = [&](size_t bytes) {
        const size_t here = at;
        at = align256(at + bytes);
        return here;
    };
    const size_t nd = nsub * static_cast<size_t>(d);
    L.id = take(nsub * 8);
    L.n = take(nsub * 8);
    L.offset = take(nsub * 8);
    L.lo = take(nd * 8);
    L.hi = take(nd * 8);
    L.base64 = take(nd * 8);
    L.scale64 = take(nd * 8);
    L.base32 = take(nd * 4);
    L.scale32 = take(nd * 4);
    L.params = take(sizeof(EvalParams));
    L.sub_first = take((nsub + 1) * 4);
    L.items = take(nitems * sizeof(WorkItem));
    L.item_rec = take(nitems * rec_len * 8);
    L.item_split = split ? take(nitems * 2 * d * 8) : 0;
    L.sub_rec = take(nsub * rec_len * 8);
    L.sub_split = split ? take(nsub * BFI_SPLIT_LEN(d) * 8) : 0;
    L.head = take(4);
    L.total = at;
    return L;
}

}  // namespace

bfi_status noalloc_setup(int device)
{
    if (device < 0 || device >= kMaxDevices)
        return fail(BFI_EUNSUPPORTED, "device %d beyond the %d the scratch table holds", device,
                    kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (g_scratch_ptr[device])
        return BFI_OK;
    void *ptr = nullptr;
    // the caller made `device` current: this is that device's copy of the array
    BFI_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr)
        return fail(BFI_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[device] = static_cast<unsigned char *>(ptr);
    return BFI_OK;
}

}  // namespace bfi

using namespace bfi;

extern "C" bfi_status bfi_eval_noalloc(bfi_context *ctx, const bfi_lattice *lat,
                                       bfi_precision prec, uint64_t seed,
                                       const bfi_subvolumes *subs, const bfi_launch *launch,
                                       double *partials, double *split)
{
    return guarded([&]() -> bfi_status {
        if (!ctx || !partials)
            return fail(BFI_EINVAL, "context and partials must be non-NULL");
        if (!known_precision(prec))
            return fail(BFI_EINVAL, "unknown precision %d", static_cast<int>(prec));
        BFI_TRY(check_lattice(lat));
        BFI_TRY(check_subvolumes(lat, subs));
        if (lat->antithetic && split)
            return fail(BFI_EUNSUPPORTED, "antithetic pairs have no split statistics");
        const int d = lat->nx * lat->nt;
        if (split && d > 32)
            return fail(BFI_EUNSUPPORTED, "split statistics need d <= 32 (d = %d)", d);
        if (subs->count == 0)
            return BFI_OK;
        if (subs->count >= 0xFFFFFFFFull)
            return fail(BFI_EINVAL, "too many subvolumes");
        unsigned char *base = nullptr;
        {
            std::lock_guard<std::mutex> lock(g_scratch_mutex);
            if (ctx->device >= 0 && ctx->device < kMaxDevices)
                base = g_scratch_ptr[ctx->device];
        }
        if (!base)
            return fail(BFI_EDEVICE, "no scratch address for device %d", ctx->device);

        const bfi_launch l = resolve_launch(ctx, *lat, prec, split != nullptr, launch);
        if (!mc_block_ok(l.block))
            return fail(BFI_EINVAL, "block must be 64, 128, 256, 512 or 1024 (got %d)", l.block);
        if (l.samples_per_thread < 1 || l.samples_per_thread > (1 << 20))
            return fail(BFI_EINVAL, "samples_per_thread out of range");
        const uint64_t chunk = static_cast<uint64_t>(l.samples_per_thread) * l.block;
        if (chunk > 0x7FFFFFFFull)
            return fail(BFI_EINVAL, "samples per work item exceed 2^31");
        uint64_t nitems = 0;
        for (size_t s = 0; s < subs->count; ++s) {
            nitems += subs->n[s] / chunk + (subs->n[s] % chunk != 0);
            if (nitems > 0x7FFFFFFFull)
                return fail(BFI_EINVAL, "more than 2^31 work items; raise samples_per_thread");
        }
        const size_t nsub = subs->count;
        const int rec_len = BFI_PARTIAL_LEN(lat->nx);
        const Layout L = layout_for(nsub, d, rec_len, nitems, split != nullptr);
        if (L.total > kScratchBytes)
            return fail(BFI_EINVAL,
                        "the evaluation needs %zu bytes of scratch (%zu subvolumes, %llu work "
                        "items); the allocation-free entry point holds at most %zu",
                        L.total, nsub, static_cast<unsigned long long>(nitems), kScratchBytes);

        BFI_HIP(hipSetDevice(ctx->device));
        hipStream_t st = ctx->stream;
        auto at = [&](size_t off) { return static_cast<void *>(base + off); };
        const size_t nd = nsub * static_cast<size_t>(d);
        BFI_HIP(hipMemcpyAsync(at(L.id), subs->id, nsub * 8, hipMemcpyHostToDevice, st));
        BFI_HIP(hipMemcpyAsync(at(L.n), subs->n, nsub * 8, hipMemcpyHostToDevice, st));
        BFI_HIP(hipMemcpyAsync(at(L.offset), subs->offset, nsub * 8, hipMemcpyHostToDevice, st));
        BFI_HIP(hipMemcpyAsync(at(L.lo), subs->lo, nd * 8, hipMemcpyHostToDevice, st));
        BFI_HIP(hipMemcpyAsync(at(L.hi), subs->hi, nd * 8, hipMemcpyHostToDevice, st));

        auto *base64 = static_cast<double *>(at(L.base64));
        auto *scale64 = static_cast<double *>(at(L.scale64));
        auto *base32 = static_cast<float *>(at(L.base32));
        auto *scale32 = static_cast<float *>(at(L.scale32));
        auto *params = static_cast<EvalParams *>(at(L.params));
        const EvalParams hp{base64, scale64, base32, scale32,
                            static_cast<const uint64_t *>(at(L.id)),
                            static_cast<const uint64_t *>(at(L.offset)), make_coef(*lat),
                            static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32)};
        BFI_HIP(hipMemcpyAsync(params, &hp, sizeof(hp), hipMemcpyHostToDevice, st));

        auto *sub_first = static_cast<uint32_t *>(at(L.sub_first));
        auto *items = static_cast<WorkItem *>(at(L.items));
        auto *item_rec = static_cast<double *>(at(L.item_rec));
        auto *item_split = split ? static_cast<double *>(at(L.item_split)) : nullptr;
        auto *sub_rec = static_cast<double *>(at(L.sub_rec));
        auto *sub_split = split ? static_cast<double *>(at(L.sub_split)) : nullptr;
        auto *head = static_cast<uint32_t *>(at(L.head));

        BuildArgs ba{static_cast<const double *>(at(L.lo)), static_cast<const double *>(at(L.hi)),
                     static_cast<const uint64_t *>(at(L.n)), sub_first, base64, scale64, base32,
                     scale32, items, params, item_rec, chunk, static_cast<uint32_t>(nsub), d,
                     rec_len};
        BFI_HIP(launch_build_items(ba, st));

        LaunchSpec spec{prec, l.block, split ? 1 : 0, l.persistent, 0, lat->observable,
                        lat->antithetic};
        if (l.persistent) {
            KernelInfo info{};
            BFI_HIP(kernel_info(lat->nx, lat->nt, spec, &info));
            const uint64_t resident = static_cast<uint64_t>(std::max(info.blocks_per_cu, 1)) *
                                      std::max(ctx->cu_count, 1);
            spec.grid = static_cast<uint32_t>(std::min<uint64_t>(resident, nitems));
            BFI_HIP(launch_reset_head(head, st));
        } else {
            spec.grid = static_cast<uint32_t>(nitems);
        }
        McArgs a{};
        a.items = items;
        a.item_split = item_split;
        a.queue_head = l.persistent ? head : nullptr;
        a.nitems = static_cast<uint32_t>(nitems);
        a.samples_per_thread = static_cast<uint32_t>(l.samples_per_thread);
        BFI_HIP(launch_mc(lat->nx, lat->nt, spec, a, st));

        MergeArgs m{};
        m.item_rec = item_rec;
        m.item_split = item_split;
        m.sub_first = sub_first;
        m.sub_rec = sub_rec;
        m.sub_split = sub_split;
        m.nsub = static_cast<uint32_t>(nsub);
        m.nx = lat->nx;
        m.d = d;
        BFI_HIP(launch_merge(m, st));
        BFI_HIP(hipMemcpyAsync(partials, sub_rec, nsub * rec_len * sizeof(double),
                               hipMemcpyDeviceToHost, st));
        if (split)
            BFI_HIP(hipMemcpyAsync(split, sub_split, nsub * BFI_SPLIT_LEN(d) * sizeof(double),
                                   hipMemcpyDeviceToHost, st));
        BFI_HIP(hipStreamSynchronize(st));
        return BFI_OK;
    });
}
