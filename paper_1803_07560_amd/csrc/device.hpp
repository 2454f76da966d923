// Device building blocks for gfx950: counter-based point generation, the
// lattice action of Eq. Gen2, and wavefront reductions.  One thread holds one
// lattice configuration in registers; everything is fully unrolled over the
// compile-time lattice shape.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace bfi {
namespace dev {
// Polynomial steps of the FP64 weight's exponential as one three-operand
// v_fma_f64 each.  Left to itself the compiler keeps the loop-invariant
// coefficients in VGPRs and rewrites every step as a register copy plus the
// two-address v_fmac_f64, one more vector instruction per step.
//   FmaVgprCoef: the coefficient (the addend) stays in a VGPR pair -- the faster
//     choice where registers are to spare (d <= 32);
//   FmaSgprCoef: scalar moves rematerialize it in an SGPR pair before each step,
//     which holds no VGPRs (the 16x4 kernels then do not spill) at the cost of
//     those scalar moves.
//   Coefficients sharing a low word (1/3! and 1/4!, 1/7! and 1/8!) would be
//   held once and their pairs rebuilt with a copy per sample: FmaVgprCoef
//   therefore holds each as a value of its own, made opaque once per object;
//   FmaVgprConst leaves them constants the compiler may rematerialize, which
//   costs those copies but no registers where pressure peaks elsewhere.
}  // namespace dev
}  // namespace bfi

#define BFI_HD __device__
#include "exp64.hpp"

namespace bfi {
namespace dev {
struct FmaVgprCoef {
    double c[12];
    __device__ FmaVgprCoef()
    {
#pragma unroll
        for (int j = 0; j < 12; ++j) {
            c[j] = expk::kInvFact[j];
            asm volatile("" : "+v"(c[j]));
        }
    }
    __device__ double coef(int j) const { return c[j]; }
    __device__ static double step(double a, double b, double c)
    {
        double d;
        asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
        return d;
    }
};
struct FmaVgprConst {
    __device__ static constexpr double coef(int j) { return expk::kInvFact[j]; }
    __device__ static double step(double a, double b, double c)
    {
        return FmaVgprCoef::step(a, b, c);
    }
};
struct FmaSgprCoef {
    __device__ static constexpr double coef(int j) { return expk::kInvFact[j]; }
    __device__ static double step(double a, double b, double c)
    {
        double d;
        asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "s"(c));
        return d;
    }
};
}  // namespace dev
}  // namespace bfi

namespace bfi {
namespace dev {

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): round multipliers and the
// Weyl increments of the key schedule.
constexpr uint32_t kPhiloxMulA = 0xD2511F53u;
constexpr uint32_t kPhiloxMulB = 0xCD9E8D57u;
constexpr uint32_t kPhiloxWeylA = 0x9E3779B9u;
constexpr uint32_t kPhiloxWeylB = 0xBB67AE85u;

// Full 32x32 -> 64-bit product in one instruction.  On gfx950 v_mad_u64_u32
// issues at the rate of v_mul_lo_u32 and v_mul_hi_u32 (measured), so one wide
// multiply replaces the separate low and high halves the compiler would pick.
// Pure register arithmetic: the carry-out goes to vcc, declared clobbered.
__device__ __forceinline__ uint64_t mul_wide(uint32_t a, uint32_t b)
{
    uint64_t r;
    asm("v_mad_u64_u32 %0, vcc, %1, %2, 0" : "=v"(r) : "v"(a), "s"(b) : "vcc");
    return r;
}

// One Philox4x32-10 block for counter (lo32(q), hi32(q), lo32(id), hi32(id)).
__device__ __forceinline__ void philox_block(uint64_t q, uint32_t id_lo, uint32_t id_hi,
                                             uint32_t key_lo, uint32_t key_hi, uint32_t out[4])
{
    uint32_t c0 = static_cast<uint32_t>(q), c1 = static_cast<uint32_t>(q >> 32);
    uint32_t c2 = id_lo, c3 = id_hi;
    uint32_t k0 = key_lo, k1 = key_hi;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t pa = mul_wide(c0, kPhiloxMulA);
        // round 0 multiplies the subvolume id, uniform across the block: left to
        // the compiler it becomes a scalar multiply
        const uint64_t pb = round == 0 ? static_cast<uint64_t>(kPhiloxMulB) * c2
                                       : mul_wide(c2, kPhiloxMulB);
        // three-input xor in one v_bitop3_b32 (truth table 0x96)
        c0 = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(pb >> 32), c1, k0, 0x96);
        c2 = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(pa >> 32), c3, k1, 0x96);
        c1 = static_cast<uint32_t>(pb);
        c3 = static_cast<uint32_t>(pa);
        k0 += kPhiloxWeylA;
        k1 += kPhiloxWeylB;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

// The share of Philox4x32-10 that is the same for every block of a work item
// whose counters keep one upper word c1 = hi32(q): round 0 multiplies the id
// word, so word 0 after it, and round 1's product of that word, are the
// item's; round 2's word 3 is too.  Computed once per item (scalar registers).
struct PhiloxItem {
    uint32_t w1_r1;    // word 1 after round 0: lo(B id_lo)
    uint32_t x2_r0;    // round 0, word 2: id_hi ^ k1
    uint32_t x0_r1;    // round 1, word 0: w1_r1 ^ (k0 + Weyl A)
    uint32_t x2_r1;    // round 1, word 2: hi(A w0_r1) ^ (k1 + Weyl B)
    uint32_t x2_r2;    // round 2, word 2: lo(A w0_r1) ^ (k1 + 2 Weyl B)
    uint32_t k0, k1;   // key
};

__device__ __forceinline__ PhiloxItem philox_item(uint32_t c1, uint32_t id_lo, uint32_t id_hi,
                                                  uint32_t key_lo, uint32_t key_hi)
{
    PhiloxItem p;
    const uint64_t b0 = static_cast<uint64_t>(kPhiloxMulB) * id_lo;
    const uint32_t w0_r1 = static_cast<uint32_t>(b0 >> 32) ^ c1 ^ key_lo;
    const uint64_t a1 = static_cast<uint64_t>(kPhiloxMulA) * w0_r1;
    p.w1_r1 = static_cast<uint32_t>(b0);
    p.x2_r0 = id_hi ^ key_hi;
    p.x0_r1 = p.w1_r1 ^ (key_lo + kPhiloxWeylA);
    p.x2_r1 = static_cast<uint32_t>(a1 >> 32) ^ (key_hi + kPhiloxWeylB);
    p.x2_r2 = static_cast<uint32_t>(a1) ^ (key_hi + 2u * kPhiloxWeylB);
    p.k0 = key_lo;
    p.k1 = key_hi;
    return p;
}

// a * b + c in one instruction; the addend is a VGPR pair (one scalar operand
// per instruction: b).
__device__ __forceinline__ uint64_t mad_wide(uint32_t a, uint32_t b, uint64_t c)
{
    uint64_t r;
    asm("v_mad_u64_u32 %0, vcc, %1, %2, %3" : "=v"(r) : "v"(a), "s"(b), "v"(c) : "vcc");
    return r;
}

// philox_block for counter (c0, c1, id_lo, id_hi) with the item's share `p`
// (same c1, id and key), given round 0's product a0 = c0 * kPhiloxMulA: the
// same words, two wide multiplies and one xor fewer.
__device__ __forceinline__ void philox_rounds_item(uint64_t a0, const PhiloxItem &p,
                                                   uint32_t out[4])
{
    // round 0: only word 2's product depends on the block
    const uint32_t w2 = static_cast<uint32_t>(a0 >> 32) ^ p.x2_r0;
    const uint32_t w3 = static_cast<uint32_t>(a0);
    // round 1: word 0 and its product are the item's
    const uint64_t b1 = mul_wide(w2, kPhiloxMulB);
    const uint32_t v0 = static_cast<uint32_t>(b1 >> 32) ^ p.x0_r1;
    const uint32_t v1 = static_cast<uint32_t>(b1);
    const uint32_t v2 = w3 ^ p.x2_r1;
    // round 2: word 3 is the item's
    uint32_t k0 = p.k0 + 2u * kPhiloxWeylA, k1 = p.k1 + 2u * kPhiloxWeylB;
    const uint64_t a2 = mul_wide(v0, kPhiloxMulA);
    const uint64_t b2 = mul_wide(v2, kPhiloxMulB);
    uint32_t c0n = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(b2 >> 32), v1, k0, 0x96);
    uint32_t c2n = static_cast<uint32_t>(a2 >> 32) ^ p.x2_r2;
    uint32_t c1n = static_cast<uint32_t>(b2);
    uint32_t c3n = static_cast<uint32_t>(a2);
#pragma unroll
    for (int round = 3; round < 10; ++round) {
        k0 += kPhiloxWeylA;
        k1 += kPhiloxWeylB;
        const uint64_t pa = mul_wide(c0n, kPhiloxMulA);
        const uint64_t pb = mul_wide(c2n, kPhiloxMulB);
        c0n = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(pb >> 32), c1n, k0, 0x96);
        c2n = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(pa >> 32), c3n, k1, 0x96);
        c1n = static_cast<uint32_t>(pb);
        c3n = static_cast<uint32_t>(pa);
    }
    out[0] = c0n;
    out[1] = c1n;
    out[2] = c2n;
    out[3] = c3n;
}

__device__ __forceinline__ void philox_block_item(uint32_t c0, const PhiloxItem &p,
                                                  uint32_t out[4])
{
    philox_rounds_item(mul_wide(c0, kPhiloxMulA), p, out);
}

// Block c0 = lo + j of a sample whose blocks lo .. lo + NB - 1 do not wrap in
// 32 bits (the item keeps one upper word): (lo + j) A = lo A + j A, so the
// counter's add rides in round 0's multiply as its addend `jA` = j A.
__device__ __forceinline__ void philox_block_item_at(uint32_t lo, uint64_t jA,
                                                     const PhiloxItem &p, uint32_t out[4])
{
    philox_rounds_item(mad_wide(lo, kPhiloxMulA, jA), p, out);
}

// Word -> coordinate: u = fma(x, scale, base), one rounding.
__device__ __forceinline__ double map_word(uint32_t x, double scale, double base)
{
    return __fma_rn(static_cast<double>(x), scale, base);
}
__device__ __forceinline__ float map_word(uint32_t x, float scale, float base)
{
    return __fmaf_rn(static_cast<float>(x), scale, base);
}

template <class T>
struct Coef {
    T k_diag, c_adv, c_visc, inv_2Dtau, half_m2;
    __device__ __forceinline__ explicit Coef(const ActionCoef &c)
        : k_diag(static_cast<T>(c.k_diag)), c_adv(static_cast<T>(c.c_adv)),
          c_visc(static_cast<T>(c.c_visc)), inv_2Dtau(static_cast<T>(c.inv_2Dtau)),
          half_m2(static_cast<T>(c.half_m2)) {}
};

__device__ __forceinline__ double fma_t(double a, double b, double c) { return __fma_rn(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __fmaf_rn(a, b, c); }

// Sum of R^2 over the sites of one time slice: `cur` is slice l, `nxt` slice
// l+1 (periodic in time), neighbours in space taken periodically.
template <class T, int NX>
__device__ __forceinline__ T slice_r2(const T (&cur)[NX], const T (&nxt)[NX], const Coef<T> &c,
                                      T acc)
{
#pragma unroll
    for (int m = 0; m < NX; ++m) {
        const T v = cur[m];
        const T vr = cur[(m + 1) % NX];
        const T vl = cur[(m + NX - 1) % NX];
        const T t = fma_t(c.c_adv, vr - vl, c.k_diag);
        T R = fma_t(v, t, nxt[m]);
        R = fma_t(-c.c_visc, vr + vl, R);
        acc = fma_t(R, R, acc);
    }
    return acc;
}

template <class T, int NX>
__device__ __forceinline__ T slice_u2(const T (&cur)[NX], T acc)
{
#pragma unroll
    for (int m = 0; m < NX; ++m)
        acc = fma_t(cur[m], cur[m], acc);
    return acc;
}

// The action S for one configuration delivered slice by slice:
// gen(l, out, token) fills time slice l; `token` is the running sum of R^2,
// which a generator may tie its work to (see the Monte Carlo kernel) so that
// slice l+1 is not produced before slice l-1 has been consumed.  Slice 0 stays
// live (it closes the time period and carries the observables); at most three
// slices are live at once.
template <class T, int NX, int NT, class Gen>
__device__ __forceinline__ T action(Gen &&gen, T (&first)[NX], const Coef<T> &c, bool mass)
{
    gen(0, first, T(0));
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
#pragma unroll
            for (int m = 0; m < NX; ++m)
                nxt[m] = first[m];
        }
        r2 = slice_r2<T, NX>(cur, nxt, c, r2);
        if (mass)
            u2 = slice_u2<T, NX>(cur, u2);
#pragma unroll
        for (int m = 0; m < NX; ++m)
            cur[m] = nxt[m];
    }
    T S = r2 * c.inv_2Dtau;
    if (mass)
        S = fma_t(c.half_m2, u2, S);
    return S;
}

// The actions of an antithetic pair: gen(l, a, b, token) writes time slice l of
// both points (from the same words), slice by slice as in action().
template <class T, int NX, int NT, class Gen>
__device__ __forceinline__ void action_pair(Gen &&gen, T (&first_a)[NX], T (&first_b)[NX],
                                            const Coef<T> &c, bool mass, T &s_a, T &s_b)
{
    gen(0, first_a, first_b, T(0));
    T cur_a[NX], cur_b[NX];
#pragma unroll
    for (int m = 0; m < NX; ++m) {
        cur_a[m] = first_a[m];
        cur_b[m] = first_b[m];
    }
    T r2a = T(0), r2b = T(0), u2a = T(0), u2b = T(0);
#pragma unroll
    for (int l = 0; l < NT; ++l) {
        T nxt_a[NX], nxt_b[NX];
        if (l + 1 < NT) {
            gen(l + 1, nxt_a, nxt_b, r2a + r2b);
        } else {
#pragma unroll
            for (int m = 0; m < NX; ++m) {
                nxt_a[m] = first_a[m];
                nxt_b[m] = first_b[m];
            }
        }
        r2a = slice_r2<T, NX>(cur_a, nxt_a, c, r2a);
        r2b = slice_r2<T, NX>(cur_b, nxt_b, c, r2b);
        if (mass) {
            u2a = slice_u2<T, NX>(cur_a, u2a);
            u2b = slice_u2<T, NX>(cur_b, u2b);
        }
#pragma unroll
        for (int m = 0; m < NX; ++m) {
            cur_a[m] = nxt_a[m];
            cur_b[m] = nxt_b[m];
        }
    }
    s_a = r2a * c.inv_2Dtau;
    s_b = r2b * c.inv_2Dtau;
    if (mass) {
        s_a = fma_t(c.half_m2, u2a, s_a);
        s_b = fma_t(c.half_m2, u2b, s_b);
    }
}

// Load a value every lane of the wavefront reads at the same address and keep
// it in scalar registers: the struct is read dword by dword and each dword is
// made wave-uniform, so the compiler holds it in SGPRs instead of VGPRs.
template <class T>
__device__ __forceinline__ T load_uniform(const T *p)
{
    static_assert(sizeof(T) % 4 == 0, "dword-sized structs only");
    T out;
    const uint32_t *src = reinterpret_cast<const uint32_t *>(p);
    uint32_t *dst = reinterpret_cast<uint32_t *>(&out);
#pragma unroll
    for (int i = 0; i < static_cast<int>(sizeof(T) / 4); ++i)
        dst[i] = __builtin_amdgcn_readfirstlane(src[i]);
    return out;
}

// Butterfly sum across the 64 lanes of a wavefront; every lane ends with the
// same bits (each step adds the same two operands in both partner lanes).
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ float wave_min(float v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v = fminf(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ double wave_min(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v = fmin(v, __shfl_xor(v, off, 64));
    return v;
}

}  // namespace dev
}  // namespace bfi
