// Gaussian-proposal importance sampling of exp(-S) for one lattice shape
// (compiled once per shape with -DBFI_NX=<space sites> -DBFI_NT=<time slices>).
//
// Proposal: dropping the nonlinear term of Eq. Gen2 leaves the quadratic form
// S0 = u.P.u / 2, P = A^T A / (D tau) + m2 I, A = (T - 1) - (nu tau / a^2) L.
// P is a polynomial in the periodic shifts, so the real Fourier basis of the
// lattice diagonalises it: u = sum_j a_j e_j with a_j = scale_j z_j, z_j
// standard normal (Box-Muller from Philox words), scale_j the mode's width;
// the constant mode may instead be uniform over [-R, R].  A defensive mixture
// with the box's uniform density (streams whose id has bit 63 set) bounds the
// weights: every sample of either component weighs
//     W / K = 1_box(u) exp(-S(u)) / (alpha exp(-sum z^2/2) + (1 - alpha) K / V).
// A work item is `count` consecutive samples of one stream; a thread holds one
// configuration in registers.  The Fourier basis enters as compile-time
// constants (its cosines and sines are evaluated by the compiler), so the
// transforms between mode coefficients and lattice variables are separable
// sums of fused multiply-adds with literal operands: nt nx (nx + nt) per
// sample.  Sums, reduction and records are those of the plain Monte Carlo
// kernel.
#include <type_traits>
#include <utility>

#include "device.hpp"
#include "is_internal.h"
#include "normals.hpp"

#ifndef BFI_NX
#error "compile with -DBFI_NX=<nx> -DBFI_NT=<nt>"
#endif

namespace bfi {
namespace {

// ---------------------------------------------- compile-time Fourier basis

constexpr double kTwoPi = 6.283185307179586476925286766559;

constexpr double ct_sqrt(double x)
{
    double r = x > 1.0 ? x : 1.0;
    for (int i = 0; i < 64; ++i)
        r = 0.5 * (r + x / r);
    return r;
}

// sin and cos of 2 pi t for t in [0, 1/8]: Taylor series (the last term kept
// is below 1e-25 there)
constexpr double ct_sin_turn(double t)
{
    const double x = kTwoPi * t;
    double term = x, sum = x;
    for (int k = 1; k < 12; ++k) {
        term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
        sum += term;
    }
    return sum;
}
constexpr double ct_cos_turn(double t)
{
    const double x = kTwoPi * t;
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 12; ++k) {
        term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
        sum += term;
    }
    return sum;
}

// cos and sin of 2 pi p / q: the angle is reduced to [0, 1/8] turn exactly, in
// units of 1/(8q) turn, by the symmetries of the circle
constexpr double ct_cos_frac(long p, long q)
{
    long t = 8 * (p % q);
    double sign = 1.0;
    if (t > 4 * q)
        t = 8 * q - t;                 // cos(2 pi - x) = cos x
    if (t > 2 * q) {
        t = 4 * q - t;                 // cos(pi - x) = -cos x
        sign = -1.0;
    }
    return t > q ? sign * ct_sin_turn(static_cast<double>(2 * q - t) / (8.0 * q))
                 : sign * ct_cos_turn(static_cast<double>(t) / (8.0 * q));
}
constexpr double ct_sin_frac(long p, long q)
{
    long t = 8 * (p % q);
    double sign = 1.0;
    if (t > 4 * q) {
        t = 8 * q - t;                 // sin(2 pi - x) = -sin x
        sign = -1.0;
    }
    if (t > 2 * q)
        t = 4 * q - t;                 // sin(pi - x) = sin x
    return t > q ? sign * ct_cos_turn(static_cast<double>(2 * q - t) / (8.0 * q))
                 : sign * ct_sin_turn(static_cast<double>(t) / (8.0 * q));
}

// component m of vector b of the real orthonormal Fourier basis of period n
constexpr double ct_basis(int n, int b, int m)
{
    if (b == 0)
        return 1.0 / ct_sqrt(n);
    if (n % 2 == 0 && b == n - 1)
        return (m % 2 ? -1.0 : 1.0) / ct_sqrt(n);
    const int k = (b + 1) / 2;
    const double s = ct_sqrt(2.0 / n);
    return s * (b % 2 ? ct_cos_frac(static_cast<long>(k) * m, n)
                      : ct_sin_frac(static_cast<long>(k) * m, n));
}

template <int I>
using Ic = std::integral_constant<int, I>;

template <int B, int E, class F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (B < E) {
        f(Ic<B>{});
        static_for<B + 1, E>(f);
    }
}

// The separable transforms between lattice variables and mode coefficients:
// one pass along space (nx x nx constants) and one along time (nt x nt), every
// coefficient a compile-time constant; terms whose coefficient is exactly zero
// are left out.
template <class T, int NX, int NT>
struct Transform {
    static constexpr int D = NX * NT;

    // lattice variables from mode coefficients: u = E a
    __device__ __forceinline__ static void inverse(const T (&a)[D], T (&u)[D])
    {
        T w[NT][NX];  // w[bt][m] = sum_bx Bx[bx][m] a[bt, bx]
        static_for<0, NT>([&](auto bt) {
            static_for<0, NX>([&](auto m) {
                T s = T(0);
                static_for<0, NX>([&](auto bx) {
                    constexpr double c = ct_basis(NX, decltype(bx)::value, decltype(m)::value);
                    if constexpr (c != 0.0)
                        s = dev::fma_t(T(c), a[decltype(bt)::value * NX + decltype(bx)::value], s);
                });
                w[decltype(bt)::value][decltype(m)::value] = s;
            });
        });
        static_for<0, NT>([&](auto l) {
            static_for<0, NX>([&](auto m) {
                T s = T(0);
                static_for<0, NT>([&](auto bt) {
                    constexpr double c = ct_basis(NT, decltype(bt)::value, decltype(l)::value);
                    if constexpr (c != 0.0)
                        s = dev::fma_t(T(c), w[decltype(bt)::value][decltype(m)::value], s);
                });
                u[decltype(l)::value * NX + decltype(m)::value] = s;
            });
        });
    }

    // mode coefficients from lattice variables: a = E^T u
    __device__ __forceinline__ static void forward(const T (&u)[D], T (&a)[D])
    {
        T w[NT][NX];  // w[l][bx] = sum_m Bx[bx][m] u[l, m]
        static_for<0, NT>([&](auto l) {
            static_for<0, NX>([&](auto bx) {
                T s = T(0);
                static_for<0, NX>([&](auto m) {
                    constexpr double c = ct_basis(NX, decltype(bx)::value, decltype(m)::value);
                    if constexpr (c != 0.0)
                        s = dev::fma_t(T(c), u[decltype(l)::value * NX + decltype(m)::value], s);
                });
                w[decltype(l)::value][decltype(bx)::value] = s;
            });
        });
        static_for<0, NT>([&](auto bt) {
            static_for<0, NX>([&](auto bx) {
                T s = T(0);
                static_for<0, NT>([&](auto l) {
                    constexpr double c = ct_basis(NT, decltype(bt)::value, decltype(l)::value);
                    if constexpr (c != 0.0)
                        s = dev::fma_t(T(c), w[decltype(l)::value][decltype(bx)::value], s);
                });
                a[decltype(bt)::value * NX + decltype(bx)::value] = s;
            });
        });
    }
};

// ------------------------------------------------------------- sampling

// log(exp(g1) + exp(g2)) with g2 possibly -inf
__device__ __forceinline__ double log_add(double g1, double g2)
{
    const double mx = fmax(g1, g2), mn = fmin(g1, g2);
    return mx + log1p(exp(mn - mx));
}
__device__ __forceinline__ float log_add(float g1, float g2)
{
    constexpr float kLog2e = 1.44269504088896340736f, kLn2 = 0.69314718055994530942f;
    const float mx = fmaxf(g1, g2), mn = fminf(g1, g2);
    return mx + kLn2 * __builtin_amdgcn_logf(1.0f + __builtin_amdgcn_exp2f((mn - mx) * kLog2e));
}

// One sample of the Gaussian component: coefficients from normals, the point
// by the inverse transform; returns sum over Gaussian modes of z^2/2.
template <class T, int NX, int NT>
__device__ __forceinline__ T gaussian_point(uint64_t index, uint32_t id_lo, uint32_t id_hi,
                                            uint32_t key_lo, uint32_t key_hi,
                                            const T (&scale)[NX * NT], bool uniform0,
                                            T (&u)[NX * NT])
{
    constexpr int D = NX * NT;
    constexpr int kPairs = (D + 1) / 2;
    constexpr int NB = (2 * kPairs + 1 + 3) / 4;  // words: the pairs, then one
    T a[D];
    T hz = T(0);
    const uint64_t q0 = index * NB;
    uint32_t blk[4];
#pragma unroll
    for (int p = 0; p < kPairs; ++p) {
        if ((p & 1) == 0)
            dev::philox_block(q0 + (p >> 1), id_lo, id_hi, key_lo, key_hi, blk);
        T zc, zs;
        dev::box_muller(blk[2 * (p & 1)], blk[2 * (p & 1) + 1], zc, zs);
        const int j0 = 2 * p, j1 = 2 * p + 1;
        a[j0] = scale[j0] * zc;
        const T h0 = T(0.5) * zc * zc;
        // a uniform constant mode leaves the exponent (its normal is unused)
        hz += (j0 == 0 && uniform0) ? T(0) : h0;
        if (j1 < D) {
            a[j1] = scale[j1] * zs;
            hz += T(0.5) * zs * zs;
        }
    }
    if (uniform0) {
        // the constant mode: word 2 ceil(d/2), uniform over [-R, R]
        constexpr int w = 2 * kPairs;
        if constexpr ((w >> 2) != ((w - 1) >> 2))
            dev::philox_block(q0 + (w >> 2), id_lo, id_hi, key_lo, key_hi, blk);
        const double v = __fma_rn(static_cast<double>(blk[w & 3]), 0x1p-32, 0x1p-33);
        a[0] = static_cast<T>(static_cast<double>(scale[0]) * (2.0 * v - 1.0));
    }
    Transform<T, NX, NT>::inverse(a, u);
    return hz;
}

// One sample of the uniform component: the plain sampler's words and point map
// over the cube, then the Gaussian exponent of that point.
template <class T, int NX, int NT>
__device__ __forceinline__ T uniform_point(uint64_t index, uint32_t id_lo, uint32_t id_hi,
                                           uint32_t key_lo, uint32_t key_hi, T map_base,
                                           T map_scale, const T (&inv_scale)[NX * NT],
                                           bool uniform0, T (&u)[NX * NT])
{
    constexpr int D = NX * NT;
    constexpr int NB = (D + 3) / 4;
    const uint64_t q0 = index * NB;
    uint32_t blk[4];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        if ((k & 3) == 0)
            dev::philox_block(q0 + (k >> 2), id_lo, id_hi, key_lo, key_hi, blk);
        u[k] = dev::map_word(blk[k & 3], map_scale, map_base);
    }
    T a[D];
    Transform<T, NX, NT>::forward(u, a);
    T hz = T(0);
#pragma unroll
    for (int j = 0; j < D; ++j) {
        const T z = a[j] * inv_scale[j];
        const T term = T(0.5) * z * z;
        hz += (j == 0 && uniform0) ? T(0) : term;
    }
    return hz;
}

// ---------------------------------------------------------------- kernel

constexpr float kShiftGap = 64.0f;
constexpr float kLog2e = 1.44269504088896340736f;

template <int NX, int NT, int PREC, int BLOCK, bool AVG>
__global__ void __launch_bounds__(BLOCK) is_kernel(IsArgs ia)
{
    using T = std::conditional_t<PREC == kFP64, double, float>;
    constexpr int D = NX * NT;
    constexpr int NW = BLOCK / 64;
    constexpr int NR = AVG ? NX / 2 + 1 : NX;
    constexpr int NF = 2 + 3 * NR;
    constexpr bool kHalfPair = AVG && NX % 2 == 0 && NX > 1;
    constexpr int kRecord = 2 + 3 * NX;
    const McArgs &a = ia.mc;
    __shared__ double red[NW][NF];
    __shared__ float red_sigma[NW];
    __shared__ uint32_t next_item;
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;

    const IsTable *tab = ia.table;
    const T log_ga = static_cast<T>(dev::load_uniform(&tab->log_ga));
    const T log_un = static_cast<T>(dev::load_uniform(&tab->log_un));
    const bool uniform0 = dev::load_uniform(&tab->uniform0) != 0;
    T lo, hi, map_base, map_scale;
    if constexpr (PREC == kFP64) {
        lo = dev::load_uniform(&tab->lo64);
        hi = dev::load_uniform(&tab->hi64);
        map_base = dev::load_uniform(&tab->map_base64);
        map_scale = dev::load_uniform(&tab->map_scale64);
    } else {
        lo = dev::load_uniform(&tab->lo32);
        hi = dev::load_uniform(&tab->hi32);
        map_base = dev::load_uniform(&tab->map_base32);
        map_scale = dev::load_uniform(&tab->map_scale32);
    }
    const T *scale_g = PREC == kFP64 ? reinterpret_cast<const T *>(tab->scale64)
                                     : reinterpret_cast<const T *>(tab->scale32);
    const T *inv_scale_g = PREC == kFP64 ? reinterpret_cast<const T *>(tab->inv_scale64)
                                         : reinterpret_cast<const T *>(tab->inv_scale32);
    const T inv_sites = T(1) / T(D);

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

        // weight and sums of one point; hz = its sum z^2/2
        auto accumulate = [&](const T (&u)[D], T hz, bool inside) {
            auto gen = [&](int l, T(&out)[NX], T) {
#pragma unroll
                for (int m = 0; m < NX; ++m)
                    out[m] = u[l * NX + m];
            };
            T first[NX];
            const T S = dev::action<T, NX, NT>(gen, first, coef, mass);
            // -log of the weight W / K
            const T L = S + log_add(log_ga - hz, log_un);
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
                w = inside ? exp(-L) : 0.0;
                const double t = pr_scale * w;
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    const double v = t * pr[r];
                    acc[2 + r] += v;
                    acc[2 + NR + r] = __fma_rn(v, v, acc[2 + NR + r]);
                    acc[2 + 2 * NR + r] = __fma_rn(v, w, acc[2 + 2 * NR + r]);
                }
            } else {
                if (inside && L < sigma - kShiftGap) {
                    rescale(exp(static_cast<double>(L) - static_cast<double>(sigma)));
                    sigma = L;
                }
                const float w32 = inside ? __builtin_amdgcn_exp2f((sigma - L) * kLog2e) : 0.0f;
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
        };

        // one sample loop per component, each with its own mode constants in
        // scalar registers
        if (id & kIsUniformStream) {
            T inv_scale[D];
#pragma unroll
            for (int j = 0; j < D; ++j)
                inv_scale[j] = dev::load_uniform(inv_scale_g + j);
            for (uint32_t k = 0; k < a.samples_per_thread; ++k) {
                const uint32_t local = k * BLOCK + tid;
                if (local >= wi.count)
                    break;
                T u[D];
                const T hz = uniform_point<T, NX, NT>(first_index + local, id_lo, id_hi, P.seed_lo,
                                                      P.seed_hi, map_base, map_scale, inv_scale,
                                                      uniform0, u);
                accumulate(u, hz, true);  // inside the cube by construction
            }
        } else {
            T scale[D];
#pragma unroll
            for (int j = 0; j < D; ++j)
                scale[j] = dev::load_uniform(scale_g + j);
            for (uint32_t k = 0; k < a.samples_per_thread; ++k) {
                const uint32_t local = k * BLOCK + tid;
                if (local >= wi.count)
                    break;
                T u[D];
                const T hz = gaussian_point<T, NX, NT>(first_index + local, id_lo, id_hi,
                                                       P.seed_lo, P.seed_hi, scale, uniform0, u);
                // inside the cube: its smallest and largest coordinates
                // (three-operand min/max; a short-circuit test per coordinate
                // compiles to a chain of divergent branches)
                T umin = u[0], umax = u[0];
#pragma unroll
                for (int j = 1; j < D; ++j) {
                    umin = fmin(umin, u[j]);
                    umax = fmax(umax, u[j]);
                }
                const bool inside = lo <= umin && umax <= hi;
                accumulate(u, hz, inside);
            }
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
            rec[1] = static_cast<double>(block_sigma);
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

template <int NX, int NT, int PREC>
__global__ void __launch_bounds__(256) is_debug_kernel(IsDebugArgs a)
{
    using T = std::conditional_t<PREC == kFP64, double, float>;
    constexpr int D = NX * NT;
    const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= a.n)
        return;
    const IsTable *tab = a.table;
    T scale[D], inv_scale[D];
    T map_base, map_scale;
    for (int k = 0; k < D; ++k) {
        if constexpr (PREC == kFP64) {
            scale[k] = tab->scale64[k];
            inv_scale[k] = tab->inv_scale64[k];
        } else {
            scale[k] = tab->scale32[k];
            inv_scale[k] = tab->inv_scale32[k];
        }
    }
    if constexpr (PREC == kFP64) {
        map_base = tab->map_base64;
        map_scale = tab->map_scale64;
    } else {
        map_base = tab->map_base32;
        map_scale = tab->map_scale32;
    }
    const uint32_t id_lo = static_cast<uint32_t>(a.id), id_hi = static_cast<uint32_t>(a.id >> 32);
    T u[D];
    T hz;
    if (a.id & kIsUniformStream)
        hz = uniform_point<T, NX, NT>(a.index[i], id_lo, id_hi, tab->seed_lo, tab->seed_hi,
                                      map_base, map_scale, inv_scale, tab->uniform0 != 0, u);
    else
        hz = gaussian_point<T, NX, NT>(a.index[i], id_lo, id_hi, tab->seed_lo, tab->seed_hi,
                                       scale, tab->uniform0 != 0, u);
    for (int k = 0; k < D; ++k)
        a.u_out[i * D + k] = static_cast<double>(u[k]);
    a.hz_out[i] = static_cast<double>(hz);
}

template <int NX, int NT, int PREC, int BLOCK, bool AVG>
hipError_t is_launch_one(const LaunchSpec &spec, const IsArgs &args, hipStream_t stream)
{
    hipLaunchKernelGGL((is_kernel<NX, NT, PREC, BLOCK, AVG>), dim3(spec.grid), dim3(BLOCK), 0,
                       stream, args);
    return hipGetLastError();
}

template <int NX, int NT, int PREC, int BLOCK, bool AVG>
hipError_t is_info_one(KernelInfo *info)
{
    hipFuncAttributes attr;
    hipError_t e = hipFuncGetAttributes(
        &attr, reinterpret_cast<const void *>(&is_kernel<NX, NT, PREC, BLOCK, AVG>));
    if (e != hipSuccess)
        return e;
    int blocks = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, is_kernel<NX, NT, PREC, BLOCK, AVG>,
                                                     BLOCK, 0);
    if (e != hipSuccess)
        return e;
    info->vgprs = attr.numRegs;
    info->sgprs = 0;
    info->blocks_per_cu = blocks;
    return hipSuccess;
}

template <int NX, int NT, template <int, int, int, int, bool> class Op, bool AVG, class... Args>
hipError_t is_dispatch_obs(const LaunchSpec &spec, Args &&...args)
{
    const bool f64 = spec.prec == kFP64;
    switch (spec.block) {
    case 64:
        return f64 ? Op<NX, NT, kFP64, 64, AVG>::run(spec, args...)
                   : Op<NX, NT, kFP32Shifted, 64, AVG>::run(spec, args...);
    case 128:
        return f64 ? Op<NX, NT, kFP64, 128, AVG>::run(spec, args...)
                   : Op<NX, NT, kFP32Shifted, 128, AVG>::run(spec, args...);
    case 256:
        return f64 ? Op<NX, NT, kFP64, 256, AVG>::run(spec, args...)
                   : Op<NX, NT, kFP32Shifted, 256, AVG>::run(spec, args...);
    default:
        return hipErrorInvalidValue;
    }
}

template <int NX, int NT, template <int, int, int, int, bool> class Op, class... Args>
hipError_t is_dispatch(const LaunchSpec &spec, Args &&...args)
{
    if (spec.split)
        return hipErrorNotSupported;
    switch (spec.obs) {
    case 0:
        return is_dispatch_obs<NX, NT, Op, false>(spec, args...);
    case 1:
        return is_dispatch_obs<NX, NT, Op, true>(spec, args...);
    default:
        return hipErrorInvalidValue;
    }
}

template <int NX, int NT, int PREC, int BLOCK, bool AVG>
struct IsLaunchOp {
    static hipError_t run(const LaunchSpec &spec, const IsArgs &args, hipStream_t stream)
    {
        return is_launch_one<NX, NT, PREC, BLOCK, AVG>(spec, args, stream);
    }
};

template <int NX, int NT, int PREC, int BLOCK, bool AVG>
struct IsInfoOp {
    static hipError_t run(const LaunchSpec &, KernelInfo *info)
    {
        return is_info_one<NX, NT, PREC, BLOCK, AVG>(info);
    }
};

}  // namespace

template <int NX, int NT>
hipError_t launch_is_shape(const LaunchSpec &spec, const IsArgs &args, hipStream_t stream)
{
    if constexpr (NX * NT > kIsMaxD) {
        (void)spec, (void)args, (void)stream;
        return hipErrorNotSupported;
    } else {
        return is_dispatch<NX, NT, IsLaunchOp>(spec, args, stream);
    }
}

template <int NX, int NT>
hipError_t is_kernel_info_shape(const LaunchSpec &spec, KernelInfo *info)
{
    if constexpr (NX * NT > kIsMaxD) {
        (void)spec, (void)info;
        return hipErrorNotSupported;
    } else {
        return is_dispatch<NX, NT, IsInfoOp>(spec, info);
    }
}

template <int NX, int NT>
hipError_t launch_is_debug_shape(const IsDebugArgs &args, hipStream_t stream)
{
    if constexpr (NX * NT > kIsMaxD) {
        (void)args, (void)stream;
        return hipErrorNotSupported;
    } else {
        const unsigned grid = static_cast<unsigned>((args.n + 255) / 256);
        if (grid == 0)
            return hipSuccess;
        if (args.prec == kFP64)
            hipLaunchKernelGGL((is_debug_kernel<NX, NT, kFP64>), dim3(grid), dim3(256), 0, stream,
                               args);
        else
            hipLaunchKernelGGL((is_debug_kernel<NX, NT, kFP32Shifted>), dim3(grid), dim3(256), 0,
                               stream, args);
        return hipGetLastError();
    }
}

template hipError_t launch_is_shape<BFI_NX, BFI_NT>(const LaunchSpec &, const IsArgs &,
                                                    hipStream_t);
template hipError_t is_kernel_info_shape<BFI_NX, BFI_NT>(const LaunchSpec &, KernelInfo *);
template hipError_t launch_is_debug_shape<BFI_NX, BFI_NT>(const IsDebugArgs &, hipStream_t);

}  // namespace bfi
