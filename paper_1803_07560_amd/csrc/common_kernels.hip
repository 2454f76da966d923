// Shape-independent kernels: work items and point maps built on the device, queue
// reset, the ordered per-subvolume merge of work-item records, and the
// point-emitting test hook.
#include "device.hpp"

namespace bfi {
namespace {

// First work item of every subvolume: an exclusive prefix sum of
// ceil(n_s / chunk) in tiles of the block, one block for the whole list.
constexpr int kScanBlock = 1024;
__global__ void __launch_bounds__(kScanBlock)
    first_items_kernel(const uint64_t *n, uint32_t nsub, uint64_t chunk, uint32_t *sub_first)
{
    __shared__ uint32_t tile[kScanBlock];
    uint32_t carry = 0;
    const uint32_t t = threadIdx.x;
    for (uint32_t base = 0; base < nsub; base += kScanBlock) {
        const uint32_t s = base + t;
        const uint32_t cnt =
            s < nsub ? static_cast<uint32_t>(n[s] / chunk + (n[s] % chunk != 0)) : 0u;
        tile[t] = cnt;
        __syncthreads();
        // inclusive Hillis-Steele scan of the tile
        for (uint32_t off = 1; off < kScanBlock; off <<= 1) {
            const uint32_t add = t >= off ? tile[t - off] : 0u;
            __syncthreads();
            tile[t] += add;
            __syncthreads();
        }
        if (s < nsub)
            sub_first[s] = carry + tile[t] - cnt;
        const uint32_t tile_total = tile[kScanBlock - 1];
        __syncthreads();  // every read of the tile done before the next one is written
        carry += tile_total;
    }
    if (t == 0)
        sub_first[nsub] = carry;
}

// Point maps (scale = (hi - lo) 2^-32, base = lo + scale/2, then the FP32
// copies) and work items of each subvolume: block b takes subvolumes b, b +
// grid, ...  The arithmetic is the host's in bfi_eval, operation for operation.

__global__ void __launch_bounds__(256) build_kernel(BuildArgs a)
{
    for (uint32_t s = blockIdx.x; s < a.nsub; s += gridDim.x) {
        const size_t row = static_cast<size_t>(s) * a.d;
        for (int k = threadIdx.x; k < a.d; k += blockDim.x) {
            const double scale = (a.hi[row + k] - a.lo[row + k]) * 0x1p-32;
            const double base = __dadd_rn(a.lo[row + k], 0.5 * scale);
            a.scale64[row + k] = scale;
            a.base64[row + k] = base;
            a.scale32[row + k] = static_cast<float>(scale);
            a.base32[row + k] = static_cast<float>(base);
        }
        const uint32_t i0 = a.sub_first[s], i1 = a.sub_first[s + 1];
        const uint64_t n = a.n[s];
        for (uint32_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
            const uint64_t start = static_cast<uint64_t>(i - i0) * a.chunk;
            const uint64_t cnt = n - start < a.chunk ? n - start : a.chunk;
            a.items[i] = WorkItem{a.params, a.item_rec + static_cast<size_t>(i) * a.rec_len, start,
                                  s, static_cast<uint32_t>(cnt)};
        }
    }
}

__global__ void reset_head_kernel(uint32_t *head)
{
    if (blockIdx.x == 0 && threadIdx.x == 0)
        *head = 0u;
}

// One block per subvolume; thread f merges field f over the subvolume's items
// in item order with Neumaier compensation, after moving every item to the
// smallest shift of the subvolume (factor exp(sigma_min - sigma_item) for
// first-order sums, its square for second-order sums; 1 in FP64 form).  Items
// are read kMergeBatch at a time, all loads of a batch issued before its
// arithmetic (the sums keep item order), so that a subvolume of many items
// is not one load latency per item.
constexpr uint32_t kMergeBatch = 8;

__global__ void __launch_bounds__(64) merge_kernel(MergeArgs m)
{
    const uint32_t s = blockIdx.x;
    if (s >= m.nsub)
        return;
    const int nx = m.nx, d = m.d;
    const int rec_len = 4 + 3 * nx;
    const int split_len = m.item_split ? 2 * d : 0;
    const uint32_t i0 = m.sub_first[s], i1 = m.sub_first[s + 1];

    double sigma = __builtin_inf();
    for (uint32_t i = i0; i < i1; i += kMergeBatch) {
        double sg[kMergeBatch];
#pragma unroll
        for (uint32_t j = 0; j < kMergeBatch; ++j)
            sg[j] = i + j < i1 ? m.item_rec[static_cast<size_t>(i + j) * rec_len + 1]
                               : __builtin_inf();
#pragma unroll
        for (uint32_t j = 0; j < kMergeBatch; ++j)
            sigma = fmin(sigma, sg[j]);
    }
    if (i0 == i1)
        sigma = 0.0;

    double *out = m.sub_rec + static_cast<size_t>(s) * rec_len;
    for (int f = threadIdx.x; f < rec_len + split_len; f += blockDim.x) {
        if (f == 1)
            continue;
        int order;
        if (f < rec_len)
            order = f == 0 ? 0 : f == 2 ? 1 : f == 3 ? 2 : f < 4 + nx ? 1 : 2;
        else
            order = (f - rec_len) < d ? 1 : 2;
        double sum = 0.0, comp = 0.0;
        for (uint32_t i = i0; i < i1; i += kMergeBatch) {
            double vb[kMergeBatch], sb[kMergeBatch];
#pragma unroll
            for (uint32_t j = 0; j < kMergeBatch; ++j) {
                if (i + j < i1) {
                    const double *rec = m.item_rec + static_cast<size_t>(i + j) * rec_len;
                    vb[j] = f < rec_len ? rec[f]
                                        : m.item_split[static_cast<size_t>(i + j) * (2 * d) +
                                                       (f - rec_len)];
                    sb[j] = rec[1];
                }
            }
#pragma unroll
            for (uint32_t j = 0; j < kMergeBatch; ++j) {
                if (i + j < i1) {
                    double v = vb[j];
                    if (order != 0) {
                        const double f1 = exp(sigma - sb[j]);
                        v *= order == 1 ? f1 : f1 * f1;
                    }
                    const double t = sum + v;
                    comp += fabs(sum) >= fabs(v) ? (sum - t) + v : (v - t) + sum;
                    sum = t;
                }
            }
        }
        if (f < rec_len)
            out[f] = sum + comp;
        else
            m.sub_split[static_cast<size_t>(s) * (1 + 2 * d) + 1 + (f - rec_len)] = sum + comp;
    }
    if (threadIdx.x == 0) {
        out[1] = sigma;
        if (m.sub_split)
            m.sub_split[static_cast<size_t>(s) * (1 + 2 * d)] = sigma;
    }
}

// The N-sphere integrand of the paper's examples (section 3, Listings 1 and 2):
// half the volume of the unit (dim+1)-ball as the integral of sqrt(1 - |x|^2).
// Same points as the lattice kernels (Philox words, fma map); FP64 sums of f and
// f^2, and of both over the upper half of the box along each dimension.
__global__ void __launch_bounds__(256) nsphere_kernel(NsphereArgs na)
{
    constexpr int kBlock = 256, kWaves = kBlock / 64, kF = 2 + 2 * kMaxNsphereDim;
    const McArgs &a = na.mc;
    const int dim = na.dim;
    const int nb = (dim + 3) / 4;
    __shared__ double red[kWaves][kF];
    __shared__ uint32_t next_item;
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;

    uint32_t it;
    if (a.queue_head) {
        if (tid == 0)
            next_item = atomicAdd(a.queue_head, 1u);
        __syncthreads();
        it = __builtin_amdgcn_readfirstlane(next_item);
    } else {
        it = blockIdx.x;
    }
    while (it < a.nitems) {
        const WorkItem wi = dev::load_uniform(a.items + it);
        const EvalParams P = dev::load_uniform(wi.params);
        const uint64_t id = P.ids[wi.sub];
        const uint64_t first_index = P.offsets[wi.sub] + wi.start;
        const double *base = P.base64 + static_cast<size_t>(wi.sub) * dim;
        const double *scale = P.scale64 + static_cast<size_t>(wi.sub) * dim;
        const uint32_t id_lo = static_cast<uint32_t>(id), id_hi = static_cast<uint32_t>(id >> 32);

        double acc[kF];
#pragma unroll
        for (int i = 0; i < kF; ++i)
            acc[i] = 0.0;
        for (uint32_t k = 0; k < a.samples_per_thread; ++k) {
            const uint32_t local = k * kBlock + tid;
            if (local >= wi.count)
                break;
            const uint64_t q0 = (first_index + local) * static_cast<uint64_t>(nb);
            double r2 = 0.0;
            uint32_t upper = 0;
            for (int j = 0; j < nb; ++j) {
                uint32_t blk[4];
                dev::philox_block(q0 + j, id_lo, id_hi, P.seed_lo, P.seed_hi, blk);
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int kk = 4 * j + t;
                    if (kk < dim) {
                        const double u = dev::map_word(blk[t], scale[kk], base[kk]);
                        r2 = __fma_rn(u, u, r2);
                        upper |= (blk[t] >> 31) << kk;
                    }
                }
            }
            const double f = r2 < 1.0 ? sqrt(1.0 - r2) : 0.0;
            const double f2 = f * f;
            acc[0] += f;
            acc[1] += f2;
#pragma unroll
            for (int kk = 0; kk < kMaxNsphereDim; ++kk) {
                const bool up = kk < dim && ((upper >> kk) & 1u);
                acc[2 + kk] += up ? f : 0.0;
                acc[2 + kMaxNsphereDim + kk] += up ? f2 : 0.0;
            }
        }
#pragma unroll
        for (int i = 0; i < kF; ++i) {
            const double v = dev::wave_sum(acc[i]);
            if (lane == 0)
                red[wave][i] = v;
        }
        __syncthreads();
        for (int i = tid; i < kF; i += kBlock) {
            double total = 0.0;
#pragma unroll
            for (int w = 0; w < kWaves; ++w)
                total += red[w][i];
            if (i < 2) {
                wi.rec[2 + i] = total;
            } else {
                const int g = i - 2;
                const int which = g / kMaxNsphereDim, kk = g % kMaxNsphereDim;
                if (kk < dim)
                    a.item_split[static_cast<size_t>(it) * (2 * dim) + which * dim + kk] = total;
            }
        }
        if (tid == 0) {
            wi.rec[0] = static_cast<double>(wi.count);
            wi.rec[1] = 0.0;
        }
        if (!a.queue_head)
            break;
        __syncthreads();
        if (tid == 0)
            next_item = atomicAdd(a.queue_head, 1u);
        __syncthreads();
        it = __builtin_amdgcn_readfirstlane(next_item);
    }
}

__global__ void __launch_bounds__(256) debug_points_kernel(DebugPointArgs a)
{
    const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= a.n)
        return;
    const int d = a.d;
    const int nb = (d + 3) / 4;
    const uint64_t q0 = a.index[i] * static_cast<uint64_t>(nb);
    const uint32_t id_lo = static_cast<uint32_t>(a.id), id_hi = static_cast<uint32_t>(a.id >> 32);
    for (int j = 0; j < nb; ++j) {
        uint32_t blk[4];
        dev::philox_block(q0 + j, id_lo, id_hi, a.seed_lo, a.seed_hi, blk);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int k = 4 * j + t;
            if (k >= d)
                break;
            a.out[i * d + k] =
                a.prec != kFP32Shifted
                    ? dev::map_word(blk[t], a.scale64[k], a.base64[k])
                    : static_cast<double>(dev::map_word(blk[t], a.scale32[k], a.base32[k]));
        }
    }
}

}  // namespace

hipError_t launch_build_items(const BuildArgs &args, hipStream_t stream)
{
    if (args.nsub == 0)
        return hipSuccess;
    hipLaunchKernelGGL(first_items_kernel, dim3(1), dim3(kScanBlock), 0, stream, args.n, args.nsub,
                       args.chunk, args.sub_first);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    const uint32_t grid = args.nsub < 4096 ? args.nsub : 4096u;
    hipLaunchKernelGGL(build_kernel, dim3(grid), dim3(256), 0, stream, args);
    return hipGetLastError();
}

hipError_t launch_reset_head(uint32_t *head, hipStream_t stream)
{
    hipLaunchKernelGGL(reset_head_kernel, dim3(1), dim3(64), 0, stream, head);
    return hipGetLastError();
}

hipError_t launch_nsphere(const NsphereArgs &args, uint32_t grid, hipStream_t stream)
{
    if (args.dim < 1 || args.dim > kMaxNsphereDim || !args.mc.item_split)
        return hipErrorInvalidValue;
    if (grid == 0)
        return hipSuccess;
    hipLaunchKernelGGL(nsphere_kernel, dim3(grid), dim3(256), 0, stream, args);
    return hipGetLastError();
}

hipError_t launch_merge(const MergeArgs &args, hipStream_t stream)
{
    if (args.nsub == 0)
        return hipSuccess;
    hipLaunchKernelGGL(merge_kernel, dim3(args.nsub), dim3(64), 0, stream, args);
    return hipGetLastError();
}

hipError_t launch_debug_points(const DebugPointArgs &args, hipStream_t stream)
{
    const unsigned grid = static_cast<unsigned>((args.n + 255) / 256);
    if (grid == 0)
        return hipSuccess;
    hipLaunchKernelGGL(debug_points_kernel, dim3(grid), dim3(256), 0, stream, args);
    return hipGetLastError();
}

}  // namespace bfi
