// Monte Carlo kernels for one lattice shape (compiled once per shape with
// -DBFI_NX=<space sites> -DBFI_NT=<time slices>).
//
// Work decomposition: a work item is `count` consecutive samples of one
// subvolume; a block of BLOCK threads takes one item, thread t takes samples
// t, t + BLOCK, t + 2 BLOCK, ... (samples_per_thread of them at most).  Each
// sample is one lattice configuration held in the thread's registers:
//   Philox words -> point in the subvolume -> action S (Eq. Gen2)
//   -> weight exp(-S) -> FP64 sums of w, w^2, p_r w, (p_r w)^2, p_r w^2
// with p_r = u_{0,0} u_{0,r} (anchored), or p_r averaged over every anchor
// (u_{l,m} u_{l,m+r} summed slice by slice as the slices are generated and
// divided by nx nt; only r = 0 .. nx/2 are accumulated, the rest are their
// mirror images r <-> nx - r).  Per-thread sums are reduced across the
// wavefront with butterfly shuffles and across the block through LDS in a
// fixed order, so the item's record is bitwise reproducible for a given launch
// shape.  Persistent launches take items from a device counter instead of
// blockIdx.x; the records are the same.
#include <type_traits>

#include "device.hpp"

#ifndef BFI_NX
#error "compile with -DBFI_NX=<nx> -DBFI_NT=<nt>"
#endif

namespace bfi {
namespace {

// Shifted forms: the per-thread shift sigma follows the smallest action seen,
// but is only moved when a new sample would weigh more than e^64 relative to it,
// so the weight exp(sigma - S) stays in (0, e^64] (FP32: within range; FP64:
// squares and their sums far from overflow) and rescales are rare.
constexpr float kShiftGap = 64.0f;
constexpr float kLog2e = 1.44269504088896340736f;
// Split statistics in the FP32 form are summed per thread in FP32 (they steer
// the choice of the split dimension and enter no estimate): sum of w, with w in
// (0, e^64], and sum of (2^-40 w)^2, so that 2^20 terms at the largest weight
// stay below FP32's maximum; weights below about e^-16 of the shift fall under
// FP32's normal range in the second sum, far below its other terms.
constexpr float kSplitWScale = 0x1p-40f;
constexpr double kSplitW2Unscale = 0x1p80;

template <int NX, int D, bool SPLIT, bool AVG>
struct Fields {
    // distinct products: every r for the anchored product, r = 0 .. NX/2 for
    // the averaged one (symmetric in r <-> NX - r)
    static constexpr int kR = AVG ? NX / 2 + 1 : NX;
    // accumulated fields: [w, w^2, p_r w (kR), (p_r w)^2 (kR), p_r w^2 (kR),
    //                      U w (D), U w^2 (D)]
    static constexpr int kMain = 2 + 3 * kR;
    static constexpr int kCount = kMain + (SPLIT ? 2 * D : 0);
    // written fields: the record's [w, w^2, p_r w (NX), (p_r w)^2 (NX),
    // p_r w^2 (NX)], then the split statistics
    static constexpr int kRecord = 2 + 3 * NX;
    static constexpr int kOut = kRecord + (SPLIT ? 2 * D : 0);
    // 1 for sums of first order in w, 2 for second order (scaled by the square
    // of a shift factor)
    __host__ __device__ static constexpr int order(int i)
    {
        return i == 0 ? 1
               : i == 1 ? 2
               : i < 2 + kR ? 1
               : i < kMain ? 2
               : i < kMain + D ? 1
                               : 2;
    }
    // accumulated field that written field f comes from
    __host__ __device__ static constexpr int source(int f)
    {
        if (f < 2)
            return f;
        if (f >= kRecord)
            return kMain + (f - kRecord);
        const int which = (f - 2) / NX, r = (f - 2) % NX;
        return 2 + which * kR + (AVG && r > NX / 2 ? NX - r : r);
    }
};

// Waves per SIMD the register allocation must leave room for: without a floor
// the compiler spends the whole register file of one wave on large lattices.
// FP32-form antithetic pairs (two points in registers) are held to three waves
// per SIMD, the occupancy of the single-point kernel.  The FP32 form with split
// statistics (2d more FP32 accumulators): three waves with the averaged
// observable (a spill of about 30 registers, measured 4-10 % faster than two
// waves without one), two with the anchored product (three spill twice as
// much: 24 % slower); the FP64 form spills too much at two.
template <int NX, int NT, int PREC, bool SPLIT, bool AVG, bool PAIR>
constexpr int kMinWaves = NX * NT > 32             ? 2
                          : PREC != kFP32Shifted   ? 1
                          : SPLIT                  ? (AVG ? 3 : 2)
                          : PAIR                   ? 3
                                                   : 1;

template <int NX, int NT, int PREC, int BLOCK, bool SPLIT, bool AVG, bool PAIR>
__global__ void __launch_bounds__(BLOCK)
    __attribute__((amdgpu_waves_per_eu(kMinWaves<NX, NT, PREC, SPLIT, AVG, PAIR>))) mc_kernel(McArgs a)
{
    using T = std::conditional_t<PREC == kFP32Shifted, float, double>;
    // the shift's type: FP32 in the FP32 form, FP64 in the shifted FP64 form
    using Sig = std::conditional_t<PREC == kFP64Shifted, double, float>;
    constexpr bool kShifted = PREC != kFP64;
    constexpr int D = NX * NT;
    constexpr int NB = (D + 3) / 4;
    constexpr int NW = BLOCK / 64;
    using F = Fields<NX, D, SPLIT, AVG>;
    constexpr int NF = F::kCount;
    constexpr int NR = F::kR;
    // at r = NX/2 (NX even) each pair u_m u_{m+r} appears twice in the sum over
    // m: accumulate half the terms and double (exactly) at the end
    constexpr bool kHalfPair = AVG && NX % 2 == 0 && NX > 1;
    const T inv_sites = T(1) / T(D);
    // register class of the exponential's polynomial coefficients (FP64 weights)
    using ExpFma = std::conditional_t<
        (D > 32 || PREC == kFP32Shifted), dev::FmaSgprCoef,
        std::conditional_t<PAIR, dev::FmaVgprConst, dev::FmaVgprCoef>>;
    const ExpFma efma;
    // j * kPhiloxMulA for the blocks j >= 1 of a sample (see block_same_hi)
    constexpr bool kFoldCounter = D <= 32 && !PAIR && !SPLIT;
    uint64_t blk_add[kFoldCounter ? NB : 1];
#pragma unroll
    for (int j = 1; j < (kFoldCounter ? NB : 1); ++j) {
        blk_add[j] = static_cast<uint64_t>(j) * dev::kPhiloxMulA;
        asm volatile("" : "+v"(blk_add[j]));
    }
    constexpr bool kSplit32 = SPLIT && PREC == kFP32Shifted;
    static_assert(!SPLIT || D <= 32, "split statistics keep one bit per dimension in 32 bits");
    static_assert(!PAIR || (!SPLIT && D <= kMaxPairD), "antithetic pairs: d <= 32, no split");

    // point map held in registers when 2d values take at most 80 VGPRs
    constexpr bool kHoist = 2 * D * sizeof(T) / 4 <= 80;
    // large FP64 lattices park time slice 0 (needed again only to close the
    // time period and for the observables) in LDS, one column per thread, so
    // that its registers are free while the other slices are processed
    constexpr bool kParkFirst = PREC != kFP32Shifted && D > 32;
    __shared__ double park_lds[kParkFirst ? NX : 1][kParkFirst ? BLOCK : 1];
    __shared__ double red[NW][NF];
    // (offset, scale) of each variable side by side: one LDS read with an
    // immediate offset fetches both
    struct alignas(2 * sizeof(T)) T2 {
        T x, y;  // offset, scale
    };
    __shared__ T2 map_lds[kHoist ? 1 : D];
    __shared__ Sig red_sigma[NW];
    __shared__ uint32_t next_item;

    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63u, wave = tid >> 6;

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
        // the item, its parameters and its point map are the same for the whole
        // block: keep them in scalar registers
        const WorkItem wi = dev::load_uniform(a.items + it);
        const EvalParams P = dev::load_uniform(wi.params);
        dev::Coef<T> coef(P.coef);
        // each site's fma(c_adv, difference, k_diag) may read one scalar
        // operand: keep k_diag in a vector register for the whole item rather
        // than copying it there once per sample
        if constexpr (D <= 32 && !PAIR)
            asm volatile("" : "+v"(coef.k_diag));
        // the mass term is chosen once per item (a uniform branch around the
        // sample loop), not per sample
        const bool has_mass = P.coef.half_m2 != 0.0;
        const uint32_t seed_lo = P.seed_lo, seed_hi = P.seed_hi;
        const uint32_t s = wi.sub;
        const uint64_t id = P.ids[s];
        const uint64_t first_index = P.offsets[s] + wi.start;
        const uint32_t id_lo = static_cast<uint32_t>(id), id_hi = static_cast<uint32_t>(id >> 32);
        const T *base_g;
        const T *scale_g;
        if constexpr (PREC != kFP32Shifted) {
            base_g = P.base64 + static_cast<size_t>(s) * D;
            scale_g = P.scale64 + static_cast<size_t>(s) * D;
        } else {
            base_g = P.base32 + static_cast<size_t>(s) * D;
            scale_g = P.scale32 + static_cast<size_t>(s) * D;
        }
        // the subvolume's point map stays in registers for the whole item when
        // it fits (2d values): offsets in scalar registers, scales in vector
        // registers, so each fma of the map reads one scalar operand (measured
        // faster than both in scalar registers, which spill); larger lattices
        // read the map from LDS (broadcast)
        T base_r[kHoist ? D : 1], scale_r[kHoist ? D : 1];
        if constexpr (kHoist) {
#pragma unroll
            for (int kk = 0; kk < D; ++kk) {
                base_r[kk] = dev::load_uniform(base_g + kk);
                scale_r[kk] = scale_g[kk];
            }
        } else {
            for (int kk = tid; kk < D; kk += BLOCK) {
                map_lds[kk] = T2{base_g[kk], scale_g[kk]};
            }
            __syncthreads();
        }
        // `row` points at the LDS-resident map, offset by a run-time zero that
        // carries the slice's dependency on the action so far: the compiler can
        // neither hoist the reads out of the sample loop (4d values live) nor
        // issue them before the slice is due; reads use immediate offsets
        using LdsRow = const __attribute__((address_space(3))) T2 *;
        auto map_of = [&](int kk, LdsRow row) -> T2 {
            if constexpr (kHoist)
                return T2{base_r[kk], scale_r[kk]};
            else
                return T2{row[kk].x, row[kk].y};  // merged into one LDS read
        };

        // FP64 accumulators, the split statistics' in FP32 in the FP32 form
        constexpr int NA = kSplit32 ? F::kMain : NF;
        double acc[NA];
#pragma unroll
        for (int i = 0; i < NA; ++i)
            acc[i] = 0.0;
        float sacc[kSplit32 ? 2 * D : 1];
#pragma unroll
        for (int i = 0; i < (kSplit32 ? 2 * D : 1); ++i)
            sacc[i] = 0.0f;
        // no sample yet: +inf (FP32 form), or the largest finite double (FP64
        // form), against which an infinite action still weighs exp(-inf) = 0
        Sig sigma = PREC == kFP64Shifted ? static_cast<Sig>(__DBL_MAX__)
                                         : static_cast<Sig>(__builtin_inff());

        auto rescale = [&](double f1) {
            const double f2 = f1 * f1;
#pragma unroll
            for (int i = 0; i < NA; ++i)
                acc[i] *= F::order(i) == 1 ? f1 : f2;
            if constexpr (kSplit32) {
                // in FP64: f2 can lie below FP32's range while the product does not
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    sacc[k] = static_cast<float>(static_cast<double>(sacc[k]) * f1);
                    sacc[D + k] = static_cast<float>(static_cast<double>(sacc[D + k]) * f2);
                }
            }
        };
        // accumulated field i as an FP64 value in the record's scale
        auto acc_value = [&](int i) -> double {
            if constexpr (kSplit32) {
                if (i >= F::kMain) {
                    const int k = i - F::kMain;
                    return k < D ? static_cast<double>(sacc[k])
                                 : static_cast<double>(sacc[k]) * kSplitW2Unscale;
                }
            }
            return acc[i];
        };

        // counters of the item: q = (index) NB + block.  When they all share
        // one upper word (every item short of a 2^32 boundary of q), part of
        // Philox is the item's and is computed once (PhiloxItem)
        const uint64_t q_first = first_index * NB;
        const uint64_t q_end = (first_index + wi.count) * NB;  // host: no wrap
        const bool same_hi = (q_first >> 32) == ((q_end - 1) >> 32);
        const dev::PhiloxItem pitem = dev::philox_item(static_cast<uint32_t>(q_first >> 32),
                                                       id_lo, id_hi, seed_lo, seed_hi);
        const uint32_t q_first_lo = static_cast<uint32_t>(q_first);
        // a sample's block j on the one-upper-word path: its counter's add
        // folded into the first multiply (addends j A held in VGPR pairs) where
        // registers allow (d <= 32, one configuration per thread, no split)
        auto block_same_hi = [&](uint32_t lo, int j, uint32_t out[4]) {
            if constexpr (kFoldCounter) {
                if (j == 0)
                    dev::philox_block_item(lo, pitem, out);
                else
                    dev::philox_block_item_at(lo, blk_add[j], pitem, out);
            } else {
                dev::philox_block_item(lo + static_cast<uint32_t>(j), pitem, out);
            }
        };

        auto samples = [&](auto same_hi_tag, auto mass_tag) {
        constexpr bool kSameHi = decltype(same_hi_tag)::value;
        const bool mass = static_cast<bool>(mass_tag);
        for (uint32_t k = 0; k < a.samples_per_thread; ++k) {
            const uint32_t local = k * BLOCK + tid;
            if (local >= wi.count)
                break;
            const uint64_t q0 = (first_index + local) * NB;
            const uint32_t q0_lo = q_first_lo + local * static_cast<uint32_t>(NB);
            if constexpr (PAIR) {
                // antithetic pair: the point of the words and the point of the
                // complemented words, i.e. its reflection through the centre of
                // the subvolume; the record sums the pair means
                T pbar_a[AVG ? NR : 1], pbar_b[AVG ? NR : 1];
#pragma unroll
                for (int r = 0; r < (AVG ? NR : 1); ++r)
                    pbar_a[r] = pbar_b[r] = T(0);
                uint32_t wb[4];
                const LdsRow row = (LdsRow)(&map_lds[0]);
                auto gen2 = [&](int l, T(&oa)[NX], T(&ob)[NX], T) {
#pragma unroll
                    for (int m = 0; m < NX; ++m) {
                        const int kk = l * NX + m;
                        if ((kk & 3) == 0) {
                            if constexpr (kSameHi)
                                block_same_hi(q0_lo, kk >> 2, wb);
                            else
                                dev::philox_block(q0 + (kk >> 2), id_lo, id_hi, seed_lo,
                                                  seed_hi, wb);
                        }
                        const uint32_t x = wb[kk & 3];
                        const T2 mp = map_of(kk, row);
                        oa[m] = dev::map_word(x, mp.y, mp.x);
                        ob[m] = dev::map_word(~x, mp.y, mp.x);
                    }
                    if constexpr (AVG) {
#pragma unroll
                        for (int r = 0; r < NR; ++r) {
                            const int terms = kHalfPair && 2 * r == NX ? NX / 2 : NX;
#pragma unroll
                            for (int m = 0; m < terms; ++m) {
                                pbar_a[r] = dev::fma_t(oa[m], oa[(m + r) % NX], pbar_a[r]);
                                pbar_b[r] = dev::fma_t(ob[m], ob[(m + r) % NX], pbar_b[r]);
                            }
                        }
                    }
                };
                T fa[NX], fb[NX], sa, sb;
                dev::action_pair<T, NX, NT>(gen2, fa, fb, coef, mass, sa, sb);
                T pra[NR], prb[NR], psa, psb;
                if constexpr (AVG) {
#pragma unroll
                    for (int r = 0; r < NR; ++r) {
                        const bool dbl = kHalfPair && 2 * r == NX;
                        pra[r] = dbl ? T(2) * pbar_a[r] : pbar_a[r];
                        prb[r] = dbl ? T(2) * pbar_b[r] : pbar_b[r];
                    }
                    psa = psb = inv_sites;
                } else {
#pragma unroll
                    for (int r = 0; r < NR; ++r) {
                        pra[r] = fa[r];
                        prb[r] = fb[r];
                    }
                    psa = fa[0];
                    psb = fb[0];
                }
                double w, v[NR];
                if constexpr (PREC != kFP32Shifted) {
                    double wa, wbt;
                    if constexpr (PREC == kFP64Shifted) {
                        const double smin = fmin(sa, sb);
                        if (smin < sigma - static_cast<double>(kShiftGap)) {
                            rescale(exp(smin - sigma));
                            sigma = smin;
                        }
                        wa = exp_weight<ExpFma>(sigma - sa, efma);
                        wbt = exp_weight<ExpFma>(sigma - sb, efma);
                    } else {
                        wa = exp_weight<ExpFma>(-sa, efma);
                        wbt = exp_weight<ExpFma>(-sb, efma);
                    }
                    w = 0.5 * (wa + wbt);
                    const double ta = psa * wa, tb = psb * wbt;
#pragma unroll
                    for (int r = 0; r < NR; ++r)
                        v[r] = 0.5 * __fma_rn(ta, pra[r], tb * prb[r]);
                } else {
                    const float smin = fminf(sa, sb);
                    if (smin < sigma - kShiftGap) {
                        rescale(exp(static_cast<double>(smin) - static_cast<double>(sigma)));
                        sigma = smin;
                    }
                    const float wa = __builtin_amdgcn_exp2f((sigma - sa) * kLog2e);
                    const float wbt = __builtin_amdgcn_exp2f((sigma - sb) * kLog2e);
                    w = static_cast<double>(0.5f * (wa + wbt));
                    const float ta = psa * wa, tb = psb * wbt;
#pragma unroll
                    for (int r = 0; r < NR; ++r)
                        v[r] = static_cast<double>(0.5f * __fmaf_rn(ta, pra[r], tb * prb[r]));
                }
                acc[0] += w;
                acc[1] = __fma_rn(w, w, acc[1]);
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    acc[2 + r] += v[r];
                    acc[2 + NR + r] = __fma_rn(v[r], v[r], acc[2 + NR + r]);
                    acc[2 + 2 * NR + r] = __fma_rn(v[r], w, acc[2 + 2 * NR + r]);
                }
                continue;
            }
            uint32_t blk[4];
            uint32_t upper = 0;
            T pbar[AVG ? NR : 1];
#pragma unroll
            for (int r = 0; r < (AVG ? NR : 1); ++r)
                pbar[r] = T(0);
            auto gen = [&](int l, T(&out)[NX], T token) {
                uint64_t qs = q0;
                uint32_t qs_lo = q0_lo;
                uint32_t zoff = 0;
                LdsRow row = (LdsRow)(&map_lds[0]);
                if constexpr (D > 32) {
                    // make this slice's counters and map reads depend on the
                    // action so far, so the compiler cannot generate every slice
                    // (and read the whole map) up front and keep 2d coordinates
                    // and 4d map values live
                    if constexpr (kSameHi)
                        asm volatile("" : "+v"(qs_lo) : "v"(token));
                    else
                        asm volatile("" : "+v"(qs) : "v"(token));
                    asm volatile("v_mov_b32 %0, 0" : "=v"(zoff) : "v"(token));
                    row += zoff;
                }
#pragma unroll
                for (int m = 0; m < NX; ++m) {
                    const int kk = l * NX + m;
                    if ((kk & 3) == 0) {
                        if constexpr (kSameHi)
                            block_same_hi(qs_lo, kk >> 2, blk);
                        else
                            dev::philox_block(qs + (kk >> 2), id_lo, id_hi, seed_lo, seed_hi,
                                              blk);
                    }
                    const uint32_t x = blk[kk & 3];
                    if constexpr (SPLIT)
                        upper |= (x >> 31) << kk;
                    const T2 mp = map_of(kk, row);
                    out[m] = dev::map_word(x, mp.y, mp.x);
                }
                if constexpr (AVG) {
#pragma unroll
                    for (int r = 0; r < NR; ++r) {
                        const int terms = kHalfPair && 2 * r == NX ? NX / 2 : NX;
#pragma unroll
                        for (int m = 0; m < terms; ++m)
                            pbar[r] = dev::fma_t(out[m], out[(m + r) % NX], pbar[r]);
                    }
                }
            };
            T first[NX];
            T S;
            if constexpr (kParkFirst) {
                // the action of dev::action, with slice 0 parked in LDS between
                // its first use and the closing of the period
                gen(0, first, T(0));
#pragma unroll
                for (int m = 0; m < NX; ++m)
                    park_lds[m][tid] = first[m];
                T cur[NX];
#pragma unroll
                for (int m = 0; m < NX; ++m)
                    cur[m] = first[m];
                T r2 = T(0), u2 = T(0);
#pragma unroll
                for (int l = 0; l < NT; ++l) {
                    T nxt[NX];
                    if (l + 1 < NT) {
                        gen(l + 1, nxt, r2);
                    } else {
                        // reload through an address offset by a run-time zero
                        // that depends on the action so far: the compiler can
                        // neither forward the stored registers nor load early
                        uint32_t zoff;
                        asm volatile("v_mov_b32 %0, 0" : "=v"(zoff) : "v"(r2));
                        using LdsD = const __attribute__((address_space(3))) double *;
                        LdsD col = (LdsD)(&park_lds[0][0]) + zoff + tid;
#pragma unroll
                        for (int m = 0; m < NX; ++m)
                            nxt[m] = col[m * BLOCK];
                    }
                    r2 = dev::slice_r2<T, NX>(cur, nxt, coef, r2);
                    if (mass)
                        u2 = dev::slice_u2<T, NX>(cur, u2);
#pragma unroll
                    for (int m = 0; m < NX; ++m)
                        cur[m] = nxt[m];
                }
#pragma unroll
                for (int m = 0; m < NX; ++m)
                    first[m] = cur[m];  // slice 0, reloaded
                S = r2 * coef.inv_2Dtau;
                if (mass)
                    S = dev::fma_t(coef.half_m2, u2, S);
            } else {
                S = dev::action<T, NX, NT>(gen, first, coef, mass);
            }
            // p_r = pr_scale * pr[r]
            T pr[NR];
            T pr_scale;
            if constexpr (AVG) {
#pragma unroll
                for (int r = 0; r < NR; ++r)
                    pr[r] = kHalfPair && 2 * r == NX ? T(2) * pbar[r] : pbar[r];
                pr_scale = inv_sites;
            } else {
#pragma unroll
                for (int r = 0; r < NR; ++r)
                    pr[r] = first[r];
                pr_scale = first[0];
            }

            double w;
            [[maybe_unused]] float w32 = 0.0f;
            if constexpr (PREC != kFP32Shifted) {
                if constexpr (PREC == kFP64Shifted) {
                    if (S < sigma - static_cast<double>(kShiftGap)) {
                        // first sample (sigma = inf) or a new action far below
                        // the shift: move the shift to S
                        rescale(exp(S - sigma));
                        sigma = S;
                    }
                    w = exp_weight<ExpFma>(sigma - S, efma);
                } else {
                    w = exp_weight<ExpFma>(-S, efma);
                }
                const double t = pr_scale * w;
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    const double v = t * pr[r];
                    acc[2 + r] += v;
                    acc[2 + NR + r] = __fma_rn(v, v, acc[2 + NR + r]);
                    acc[2 + 2 * NR + r] = __fma_rn(v, w, acc[2 + 2 * NR + r]);
                }
            } else {
                if (S < sigma - kShiftGap) {
                    // first sample (sigma = inf: factor 0 on zero sums) or a new
                    // action far below the shift: move the shift to S
                    rescale(exp(static_cast<double>(S) - static_cast<double>(sigma)));
                    sigma = S;
                }
                w32 = __builtin_amdgcn_exp2f((sigma - S) * kLog2e);
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
            if constexpr (kSplit32) {
                const float ws = w32 * kSplitWScale;
                const float w2s = ws * ws;
#pragma unroll
                for (int kk = 0; kk < D; ++kk) {
                    // the half as 0 or 1: one fused multiply-add adds w or
                    // exactly nothing (finite w), as a select and an add would
                    const float up = static_cast<float>((upper >> kk) & 1u);
                    sacc[kk] = __builtin_fmaf(up, w32, sacc[kk]);
                    sacc[D + kk] = __builtin_fmaf(up, w2s, sacc[D + kk]);
                }
            } else if constexpr (SPLIT) {
                const double w2 = w * w;
#pragma unroll
                for (int kk = 0; kk < D; ++kk) {
                    const double up = static_cast<double>((upper >> kk) & 1u);
                    acc[F::kMain + kk] = __fma_rn(up, w, acc[F::kMain + kk]);
                    acc[F::kMain + D + kk] = __fma_rn(up, w2, acc[F::kMain + D + kk]);
                }
            }
        }
        };
        // (pairs and lattices of more than 32 sites keep the run-time flag:
        // duplicated sample loops raised their register pressure)
        auto samples_mass = [&](auto same_hi_tag) {
            if constexpr (PAIR || D > 32) {
                samples(same_hi_tag, has_mass);
            } else {
                if (has_mass)
                    samples(same_hi_tag, std::true_type{});
                else
                    samples(same_hi_tag, std::false_type{});
            }
        };
        if (same_hi)
            samples_mass(std::true_type{});
        else
            samples_mass(std::false_type{});

        // ---- reduction: wavefront butterflies, then waves in order through LDS
        Sig wave_sigma = Sig(0);
        if constexpr (kShifted) {
            wave_sigma = dev::wave_min(sigma);
            // lanes that took no sample hold sigma = inf and zero sums
            rescale(sigma == static_cast<Sig>(__builtin_inff())
                        ? 0.0
                        : exp(static_cast<double>(wave_sigma) - static_cast<double>(sigma)));
        }
#pragma unroll
        for (int i = 0; i < NF; ++i) {
            const double v = dev::wave_sum(acc_value(i));
            if (lane == 0)
                red[wave][i] = v;
        }
        if (lane == 0)
            red_sigma[wave] = wave_sigma;
        __syncthreads();

        Sig block_sigma = Sig(0);
        if constexpr (kShifted) {
            block_sigma = red_sigma[0];
#pragma unroll
            for (int w = 1; w < NW; ++w)
                block_sigma = block_sigma < red_sigma[w] ? block_sigma : red_sigma[w];
        }
        double *rec = wi.rec;
        for (int i = tid; i < F::kOut; i += BLOCK) {
            const int src = F::source(i);
            double total = 0.0;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                double v = red[w][src];
                if constexpr (kShifted) {
                    const Sig ws = red_sigma[w];
                    const double f1 = ws == static_cast<Sig>(__builtin_inff())
                                          ? 0.0
                                          : exp(static_cast<double>(block_sigma) -
                                                static_cast<double>(ws));
                    v *= F::order(src) == 1 ? f1 : f1 * f1;
                }
                total += v;
            }
            if (i < F::kRecord)
                rec[2 + i] = total;
            else
                a.item_split[static_cast<size_t>(it) * (2 * D) + (i - F::kRecord)] = total;
        }
        if (tid == 0) {
            rec[0] = static_cast<double>(wi.count);
            rec[1] = static_cast<double>(block_sigma);
        }

        if (!a.queue_head)
            break;
        __syncthreads();  // LDS slots free again before the next item
        if (tid == 0)
            next_item = atomicAdd(a.queue_head, 1u);
        __syncthreads();
        it = __builtin_amdgcn_readfirstlane(next_item);
    }
}

template <int NX, int NT, int PREC>
__global__ void __launch_bounds__(256) debug_action_kernel(DebugActionArgs a)
{
    using T = std::conditional_t<PREC == kFP32Shifted, float, double>;
    constexpr int D = NX * NT;
    const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= a.n)
        return;
    const double *p = a.points + i * D;
    auto gen = [&](int l, T(&out)[NX], T) {
#pragma unroll
        for (int m = 0; m < NX; ++m)
            out[m] = static_cast<T>(p[l * NX + m]);
    };
    T first[NX];
    const dev::Coef<T> coef(a.coef);
    a.out[i] = static_cast<double>(dev::action<T, NX, NT>(gen, first, coef, a.coef.half_m2 != 0.0));
}

template <int NX, int NT, int PREC, int BLOCK, bool SPLIT, bool AVG, bool PAIR>
hipError_t launch_one(const LaunchSpec &spec, const McArgs &args, hipStream_t stream)
{
    hipLaunchKernelGGL((mc_kernel<NX, NT, PREC, BLOCK, SPLIT, AVG, PAIR>), dim3(spec.grid),
                       dim3(BLOCK), 0, stream, args);
    return hipGetLastError();
}

template <int NX, int NT, int PREC, int BLOCK, bool SPLIT, bool AVG, bool PAIR>
hipError_t info_one(KernelInfo *info)
{
    hipFuncAttributes attr;
    hipError_t e = hipFuncGetAttributes(
        &attr, reinterpret_cast<const void *>(&mc_kernel<NX, NT, PREC, BLOCK, SPLIT, AVG, PAIR>));
    if (e != hipSuccess)
        return e;
    int blocks = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &blocks, mc_kernel<NX, NT, PREC, BLOCK, SPLIT, AVG, PAIR>, BLOCK, 0);
    if (e != hipSuccess)
        return e;
    info->vgprs = attr.numRegs;
    info->sgprs = 0;
    info->blocks_per_cu = blocks;
    return hipSuccess;
}

template <int NX, int NT, int BLOCK, bool SPLIT, bool AVG, bool PAIR,
          template <int, int, int, int, bool, bool, bool> class Op, class... Args>
hipError_t by_prec(const LaunchSpec &spec, Args &&...args)
{
    switch (spec.prec) {
    case kFP64:
        return Op<NX, NT, kFP64, BLOCK, SPLIT, AVG, PAIR>::run(spec, args...);
    case kFP32Shifted:
        return Op<NX, NT, kFP32Shifted, BLOCK, SPLIT, AVG, PAIR>::run(spec, args...);
    case kFP64Shifted:
        return Op<NX, NT, kFP64Shifted, BLOCK, SPLIT, AVG, PAIR>::run(spec, args...);
    default:
        return hipErrorInvalidValue;
    }
}

// Dispatch over (precision, block, split) for this shape, observable and
// sampler.  Split statistics are compiled for 256-thread blocks and d <= 32
// only; antithetic pairs for d <= kMaxPairD and without split statistics.
template <int NX, int NT, bool AVG, bool PAIR, template <int, int, int, int, bool, bool, bool> class Op,
          class... Args>
hipError_t dispatch_obs(const LaunchSpec &spec, Args &&...args)
{
    constexpr int D = NX * NT;
    if (spec.split) {
        if constexpr (D <= 32 && !PAIR) {
            if (spec.block != 256)
                return hipErrorInvalidValue;
            return by_prec<NX, NT, 256, true, AVG, false, Op>(spec, args...);
        } else {
            return hipErrorNotSupported;
        }
    }
    if constexpr (PAIR && D > kMaxPairD) {
        return hipErrorNotSupported;
    } else {
        switch (spec.block) {
        case 64:
            return by_prec<NX, NT, 64, false, AVG, PAIR, Op>(spec, args...);
        case 128:
            return by_prec<NX, NT, 128, false, AVG, PAIR, Op>(spec, args...);
        case 256:
            return by_prec<NX, NT, 256, false, AVG, PAIR, Op>(spec, args...);
        case 512:
            return by_prec<NX, NT, 512, false, AVG, PAIR, Op>(spec, args...);
        case 1024:
            return by_prec<NX, NT, 1024, false, AVG, PAIR, Op>(spec, args...);
        default:
            return hipErrorInvalidValue;
        }
    }
}

template <int NX, int NT, template <int, int, int, int, bool, bool, bool> class Op,
          class... Args>
hipError_t dispatch(const LaunchSpec &spec, Args &&...args)
{
    if (spec.pair != 0 && spec.pair != 1)
        return hipErrorInvalidValue;
    switch (spec.obs) {
    case 0:
        return spec.pair ? dispatch_obs<NX, NT, false, true, Op>(spec, args...)
                         : dispatch_obs<NX, NT, false, false, Op>(spec, args...);
    case 1:
        return spec.pair ? dispatch_obs<NX, NT, true, true, Op>(spec, args...)
                         : dispatch_obs<NX, NT, true, false, Op>(spec, args...);
    default:
        return hipErrorInvalidValue;
    }
}

template <int NX, int NT, int PREC, int BLOCK, bool SPLIT, bool AVG, bool PAIR>
struct LaunchOp {
    static hipError_t run(const LaunchSpec &spec, const McArgs &args, hipStream_t stream)
    {
        return launch_one<NX, NT, PREC, BLOCK, SPLIT, AVG, PAIR>(spec, args, stream);
    }
};

template <int NX, int NT, int PREC, int BLOCK, bool SPLIT, bool AVG, bool PAIR>
struct InfoOp {
    static hipError_t run(const LaunchSpec &, KernelInfo *info)
    {
        return info_one<NX, NT, PREC, BLOCK, SPLIT, AVG, PAIR>(info);
    }
};

}  // namespace

template <int NX, int NT>
hipError_t launch_mc_shape(const LaunchSpec &spec, const McArgs &args, hipStream_t stream)
{
    return dispatch<NX, NT, LaunchOp>(spec, args, stream);
}

template <int NX, int NT>
hipError_t kernel_info_shape(const LaunchSpec &spec, KernelInfo *info)
{
    return dispatch<NX, NT, InfoOp>(spec, info);
}

template <int NX, int NT>
hipError_t launch_debug_action_shape(const DebugActionArgs &args, hipStream_t stream)
{
    const unsigned grid = static_cast<unsigned>((args.n + 255) / 256);
    if (grid == 0)
        return hipSuccess;
    if (args.prec != kFP32Shifted)
        hipLaunchKernelGGL((debug_action_kernel<NX, NT, kFP64>), dim3(grid), dim3(256), 0, stream,
                           args);
    else
        hipLaunchKernelGGL((debug_action_kernel<NX, NT, kFP32Shifted>), dim3(grid), dim3(256), 0,
                           stream, args);
    return hipGetLastError();
}

template hipError_t launch_mc_shape<BFI_NX, BFI_NT>(const LaunchSpec &, const McArgs &,
                                                    hipStream_t);
template hipError_t kernel_info_shape<BFI_NX, BFI_NT>(const LaunchSpec &, KernelInfo *);
template hipError_t launch_debug_action_shape<BFI_NX, BFI_NT>(const DebugActionArgs &,
                                                              hipStream_t);

}  // namespace bfi
