// Monte Carlo in spherical coordinates for one lattice shape (compiled once per
// shape with -DBFI_NX=<space sites> -DBFI_NT=<time slices>).
//
// A work item is `count` consecutive samples of one radial shell of the cube
// [-B, B]^d.  Per sample, in one thread's registers: 2 ceil(d/2) + 1 Philox
// words; d standard normals z (Box-Muller pairs of words 2p, 2p + 1: cosine for
// the even coordinate, sine for the odd one), the radius from the last word,
// v = (x + 1/2) 2^-32, rho = rho_hi (t + v (1 - t))^(1/d) (t = (rho_lo /
// rho_hi)^d), and u = rho z / |z|: uniform in the shell's volume.  Inside the
// cube the weight is exp(-S(u)) (Eq. Gen2), outside 0; the observables, FP64
// sums, wavefront/LDS reduction and record layout are the plain kernel's, so
// the finalize with shell volumes gives the integral.  FP64 form: library log,
// sqrt, sincospi and pow; FP32 form: the hardware transcendentals and a shifted
// weight, as in the plain kernel.
#include <type_traits>

#include "device.hpp"
#include "normals.hpp"
#include "sph_internal.h"

#ifndef BFI_NX
#error "compile with -DBFI_NX=<nx> -DBFI_NT=<nt>"
#endif

namespace bfi {
namespace {

constexpr float kShiftGap = 64.0f;
constexpr float kLog2e = 1.44269504088896340736f;

template <int D>
struct SphWords {
    static constexpr int kPairs = (D + 1) / 2;
    static constexpr int kRadiusWord = 2 * kPairs;
    static constexpr int kBlocks = (2 * kPairs + 1 + 3) / 4;
};

// The point of sample `index` of a shell.
template <class T, int D>
__device__ __forceinline__ void shell_point(uint64_t index, uint32_t id_lo, uint32_t id_hi,
                                            uint32_t key_lo, uint32_t key_hi, T rho_hi, T t,
                                            T (&u)[D])
{
    using W = SphWords<D>;
    const uint64_t q0 = index * W::kBlocks;
    uint32_t blk[4];
    T norm2 = T(0);
#pragma unroll
    for (int p = 0; p < W::kPairs; ++p) {
        if ((p & 1) == 0)
            dev::philox_block(q0 + (p >> 1), id_lo, id_hi, key_lo, key_hi, blk);
        T zc, zs;
        dev::box_muller(blk[2 * (p & 1)], blk[2 * (p & 1) + 1], zc, zs);
        u[2 * p] = zc;
        norm2 = dev::fma_t(zc, zc, norm2);
        if (2 * p + 1 < D) {
            u[2 * p + 1] = zs;
            norm2 = dev::fma_t(zs, zs, norm2);
        }
    }
    constexpr int w = W::kRadiusWord;
    if constexpr ((w >> 2) != ((w - 1) >> 2))
        dev::philox_block(q0 + (w >> 2), id_lo, id_hi, key_lo, key_hi, blk);
    const uint32_t xr = blk[w & 3];
    T f;
    if constexpr (std::is_same_v<T, double>) {
        const double v = __fma_rn(static_cast<double>(xr), 0x1p-32, 0x1p-33);
        const double rho = rho_hi * pow(__fma_rn(v, 1.0 - t, t), 1.0 / D);
        f = rho / sqrt(norm2);
    } else {
        const float v = __fmaf_rn(static_cast<float>(xr), 0x1p-32f, 0x1p-33f);
        const float y = __fmaf_rn(v, 1.0f - t, t);
        const float rho = rho_hi * __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(y) * (1.0f / D));
        f = rho * __builtin_amdgcn_rsqf(norm2);
    }
#pragma unroll
    for (int k = 0; k < D; ++k)
        u[k] *= f;
}

template <int NX, int NT, int PREC, int BLOCK, bool AVG>
__global__ void __launch_bounds__(BLOCK) sph_kernel(SphArgs sa)
{
    using T = std::conditional_t<PREC == kFP64, double, float>;
    constexpr int D = NX * NT;
    constexpr int NW = BLOCK / 64;
    constexpr int NR = AVG ? NX / 2 + 1 : NX;
    constexpr int NF = 2 + 3 * NR;
    constexpr bool kHalfPair = AVG && NX % 2 == 0 && NX > 1;
    constexpr int kRecord = 2 + 3 * NX;
    static_assert(D <= kSphMaxD, "spherical sampler: d <= 32");
    const McArgs &a = sa.mc;
    __shared__ double red[NW][NF];
    __shared__ float red_sigma[NW];
    __shared__ uint32_t next_item;
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    const T box = PREC == kFP64 ? static_cast<T>(sa.box64) : static_cast<T>(sa.box32);
    const T inv_sites = T(1) / T(D);
    using ExpFma = std::conditional_t<PREC == kFP32Shifted, dev::FmaSgprCoef, dev::FmaVgprCoef>;
    const ExpFma efma;

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
        const dev::Coef<T> coef(P.coef);
        const bool mass = P.coef.half_m2 != 0.0;
        const uint32_t s = wi.sub;
        const uint64_t id = P.ids[s];
        const uint64_t first_index = P.offsets[s] + wi.start;
        const uint32_t id_lo = static_cast<uint32_t>(id), id_hi = static_cast<uint32_t>(id >> 32);
        T rho_hi, t;
        if constexpr (PREC == kFP64) {
            rho_hi = dev::load_uniform(sa.shell64 + 2 * static_cast<size_t>(s));
            t = dev::load_uniform(sa.shell64 + 2 * static_cast<size_t>(s) + 1);
        } else {
            rho_hi = dev::load_uniform(sa.shell32 + 2 * static_cast<size_t>(s));
            t = dev::load_uniform(sa.shell32 + 2 * static_cast<size_t>(s) + 1);
        }

        double acc[NF];
#pragma unroll
        for (int i = 0; i < NF; ++i)
            acc[i] = 0.0;
        float sigma = __builtin_inff();
        auto rescale = [&](double f1) {
            const double f2 = f1 * f1;
#pragma unroll
            for (int i = 0; i < NF; ++i)
                acc[i] *= (i == 0 || (i >= 2 && i < 2 + NR)) ? f1 : f2;
        };

        for (uint32_t k = 0; k < a.samples_per_thread; ++k) {
            const uint32_t local = k * BLOCK + tid;
            if (local >= wi.count)
                break;
            T u[D];
            shell_point<T, D>(first_index + local, id_lo, id_hi, P.seed_lo, P.seed_hi, rho_hi, t,
                              u);
            // inside the cube: the largest |u_j| (three-operand max; a
            // short-circuit test per coordinate compiles to a chain of
            // divergent branches)
            T umax = fabs(u[0]);
#pragma unroll
            for (int j = 1; j < D; ++j)
                umax = fmax(umax, fabs(u[j]));
            const bool inside = umax <= box;
            auto gen = [&](int l, T(&out)[NX], T) {
#pragma unroll
                for (int m = 0; m < NX; ++m)
                    out[m] = u[l * NX + m];
            };
            T first[NX];
            const T S = dev::action<T, NX, NT>(gen, first, coef, mass);
            T pr[NR];
            T pr_scale;
            if constexpr (AVG) {
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    const int terms = kHalfPair && 2 * r == NX ? NX / 2 : NX;
                    T acc_r = T(0);
#pragma unroll
                    for (int l = 0; l < NT; ++l)
#pragma unroll
                        for (int m = 0; m < terms; ++m)
                            acc_r = dev::fma_t(u[l * NX + m], u[l * NX + (m + r) % NX], acc_r);
                    pr[r] = kHalfPair && 2 * r == NX ? T(2) * acc_r : acc_r;
                }
                pr_scale = inv_sites;
            } else {
#pragma unroll
                for (int r = 0; r < NR; ++r)
                    pr[r] = first[r];
                pr_scale = first[0];
            }
            double w;
            if constexpr (PREC == kFP64) {
                w = inside ? exp_weight<ExpFma>(-S, efma) : 0.0;
                const double tw = pr_scale * w;
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    const double v = tw * pr[r];
                    acc[2 + r] += v;
                    acc[2 + NR + r] = __fma_rn(v, v, acc[2 + NR + r]);
                    acc[2 + 2 * NR + r] = __fma_rn(v, w, acc[2 + 2 * NR + r]);
                }
            } else {
                if (inside && S < sigma - kShiftGap) {
                    rescale(exp(static_cast<double>(S) - static_cast<double>(sigma)));
                    sigma = S;
                }
                const float w32 = inside ? __builtin_amdgcn_exp2f((sigma - S) * kLog2e) : 0.0f;
                w = static_cast<double>(w32);
                const float t32 = pr_scale * w32;
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    const double v = static_cast<double>(t32 * pr[r]);
                    acc[2 + r] += v;
                    acc[2 + NR + r] = __fma_rn(v, v, acc[2 + NR + r]);
                    acc[2 + 2 * NR + r] = __fma_rn(v, w, acc[2 + 2 * NR + r]);
                }
            }
            acc[0] += w;
            acc[1] = __fma_rn(w, w, acc[1]);
        }

        // reduction: wavefront butterflies, then waves in order through LDS
        float wave_sigma = 0.0f;
        if constexpr (PREC != kFP64) {
            wave_sigma = dev::wave_min(sigma);
            rescale(sigma == __builtin_inff()
                        ? 0.0
                        : exp(static_cast<double>(wave_sigma) - static_cast<double>(sigma)));
        }
#pragma unroll
        for (int i = 0; i < NF; ++i) {
            const double v = dev::wave_sum(acc[i]);
            if (lane == 0)
                red[wave][i] = v;
        }
        if (lane == 0)
            red_sigma[wave] = wave_sigma;
        __syncthreads();
        float block_sigma = 0.0f;
        if constexpr (PREC != kFP64) {
            block_sigma = red_sigma[0];
#pragma unroll
            for (int w = 1; w < NW; ++w)
                block_sigma = fminf(block_sigma, red_sigma[w]);
        }
        double *rec = wi.rec;
        for (int i = tid; i < kRecord; i += BLOCK) {
            // record field i: [w, w^2, p_r w (NX), (p_r w)^2 (NX), p_r w^2 (NX)]
            int src = i;
            if (i >= 2) {
                const int which = (i - 2) / NX, r = (i - 2) % NX;
                src = 2 + which * NR + (AVG && r > NX / 2 ? NX - r : r);
            }
            const int order = (src == 0 || (src >= 2 && src < 2 + NR)) ? 1 : 2;
            double total = 0.0;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                double v = red[w][src];
                if constexpr (PREC != kFP64) {
                    const float ws = red_sigma[w];
                    const double f1 = ws == __builtin_inff()
                                          ? 0.0
                                          : exp(static_cast<double>(block_sigma) -
                                                static_cast<double>(ws));
                    v *= order == 1 ? f1 : f1 * f1;
                }
                total += v;
            }
            rec[2 + i] = total;
        }
        if (tid == 0) {
            rec[0] = static_cast<double>(wi.count);
            // an item whose points all fell outside the cube has only zero sums: a
            // shift far above any action gives it the factor 0 wherever it is
            // merged with records that have weight (and 1 among empty ones)
            rec[1] = block_sigma == __builtin_inff() ? 1e300 : static_cast<double>(block_sigma);
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

template <int D, int PREC>
__global__ void __launch_bounds__(256) sph_debug_kernel(SphDebugArgs a)
{
    using T = std::conditional_t<PREC == kFP64, double, float>;
    const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= a.n)
        return;
    T u[D];
    shell_point<T, D>(a.index[i], static_cast<uint32_t>(a.id), static_cast<uint32_t>(a.id >> 32),
                      a.seed_lo, a.seed_hi, static_cast<T>(a.rho_hi), static_cast<T>(a.t), u);
#pragma unroll
    for (int k = 0; k < D; ++k)
        a.out[i * D + k] = static_cast<double>(u[k]);
}

template <int NX, int NT, int PREC, int BLOCK, bool AVG>
hipError_t launch_one(const LaunchSpec &spec, const SphArgs &args, hipStream_t stream)
{
    hipLaunchKernelGGL((sph_kernel<NX, NT, PREC, BLOCK, AVG>), dim3(spec.grid), dim3(BLOCK), 0,
                       stream, args);
    return hipGetLastError();
}

template <int NX, int NT, int PREC, int BLOCK, bool AVG>
hipError_t info_one(KernelInfo *info)
{
    hipFuncAttributes attr;
    hipError_t e = hipFuncGetAttributes(
        &attr, reinterpret_cast<const void *>(&sph_kernel<NX, NT, PREC, BLOCK, AVG>));
    if (e != hipSuccess)
        return e;
    int blocks = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, sph_kernel<NX, NT, PREC, BLOCK, AVG>,
                                                     BLOCK, 0);
    if (e != hipSuccess)
        return e;
    info->vgprs = attr.numRegs;
    info->sgprs = 0;
    info->blocks_per_cu = blocks;
    return hipSuccess;
}

// Dispatch over (precision, block, observable): FP64 and the FP32 form,
// 64/128/256-thread blocks, both observables.
template <int NX, int NT, bool Info, class... Args>
hipError_t dispatch(const LaunchSpec &spec, Args &&...args)
{
    if constexpr (NX * NT > kSphMaxD) {
        return hipErrorNotSupported;
    } else {
        if (spec.split || spec.pair || (spec.obs != 0 && spec.obs != 1))
            return hipErrorInvalidValue;
        if (spec.prec != kFP64 && spec.prec != kFP32Shifted)
            return hipErrorNotSupported;
        auto go = [&](auto prec_tag, auto block_tag, auto avg_tag) -> hipError_t {
            constexpr int PREC = decltype(prec_tag)::value;
            constexpr int BLOCK = decltype(block_tag)::value;
            constexpr bool AVG = decltype(avg_tag)::value;
            if constexpr (Info)
                return info_one<NX, NT, PREC, BLOCK, AVG>(args...);
            else
                return launch_one<NX, NT, PREC, BLOCK, AVG>(spec, args...);
        };
        auto by_block = [&](auto prec_tag, auto avg_tag) -> hipError_t {
            switch (spec.block) {
            case 64:
                return go(prec_tag, std::integral_constant<int, 64>{}, avg_tag);
            case 128:
                return go(prec_tag, std::integral_constant<int, 128>{}, avg_tag);
            case 256:
                return go(prec_tag, std::integral_constant<int, 256>{}, avg_tag);
            default:
                return hipErrorInvalidValue;
            }
        };
        auto by_obs = [&](auto prec_tag) -> hipError_t {
            return spec.obs ? by_block(prec_tag, std::true_type{})
                            : by_block(prec_tag, std::false_type{});
        };
        return spec.prec == kFP64 ? by_obs(std::integral_constant<int, kFP64>{})
                                  : by_obs(std::integral_constant<int, kFP32Shifted>{});
    }
}

}  // namespace

template <int NX, int NT>
hipError_t launch_sph_shape(const LaunchSpec &spec, const SphArgs &args, hipStream_t stream)
{
    return dispatch<NX, NT, false>(spec, args, stream);
}

template <int NX, int NT>
hipError_t sph_kernel_info_shape(const LaunchSpec &spec, KernelInfo *info)
{
    return dispatch<NX, NT, true>(spec, info);
}

template <int NX, int NT>
hipError_t launch_sph_debug_shape(const SphDebugArgs &args, hipStream_t stream)
{
    constexpr int D = NX * NT;
    if constexpr (D > kSphMaxD) {
        return hipErrorNotSupported;
    } else {
        const unsigned grid = static_cast<unsigned>((args.n + 255) / 256);
        if (grid == 0)
            return hipSuccess;
        if (args.prec == kFP64)
            hipLaunchKernelGGL((sph_debug_kernel<D, kFP64>), dim3(grid), dim3(256), 0, stream,
                               args);
        else
            hipLaunchKernelGGL((sph_debug_kernel<D, kFP32Shifted>), dim3(grid), dim3(256), 0,
                               stream, args);
        return hipGetLastError();
    }
}

template hipError_t launch_sph_shape<BFI_NX, BFI_NT>(const LaunchSpec &, const SphArgs &,
                                                     hipStream_t);
template hipError_t sph_kernel_info_shape<BFI_NX, BFI_NT>(const LaunchSpec &, KernelInfo *);
template hipError_t launch_sph_debug_shape<BFI_NX, BFI_NT>(const SphDebugArgs &, hipStream_t);

}  // namespace bfi
