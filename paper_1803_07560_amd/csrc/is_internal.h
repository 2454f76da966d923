// Internal interface of the Gaussian-proposal sampler (is_kernels.hip) for the
// host runtime.  Not part of the public ABI.
//
// Proposal: the Gaussian of the action's quadratic part (Eq. Gen2 without the
// nonlinear term), diagonal in the real Fourier basis of the lattice, mixed
// with the uniform density of the box.  Mode j = bt*nx + bx is the product of
// time vector bt and space vector bx of the one-dimensional real bases
// (vector b of period n: 0 constant, 2k-1 cosine and 2k sine of frequency
// k < n/2, n-1 alternating for even n, all normalised).
#pragma once

#include "internal.h"

namespace bfi {

// Largest lattice the sampler is compiled for: the point and its mode
// coefficients are held in registers.
constexpr int kIsMaxD = 32;

// Everything the sampler needs besides the stream ids and offsets, one table
// per plan in device memory.  The box is a cube [lo, hi]^d.
struct IsTable {
    double scale64[kIsMaxD];      // per mode: standard deviation (Gaussian) or R (uniform mode 0)
    double inv_scale64[kIsMaxD];  // 1 / scale
    float scale32[kIsMaxD];
    float inv_scale32[kIsMaxD];
    double lo64, hi64;            // the box: indicator of the Gaussian component
    double map_base64, map_scale64;  // uniform component: u = fma(x, map_scale, map_base)
    float lo32, hi32, map_base32, map_scale32;
    // log of (mixture density x K) = log(exp(log_ga - sum z^2/2) + exp(log_un)):
    // log_ga = log alpha, log_un = log(1 - alpha) + log K - log V (-inf if absent)
    double log_ga, log_un;
    int32_t uniform0;  // 1: the constant mode is drawn uniformly over [-R, R]
    uint32_t seed_lo, seed_hi;  // debug hook only (kernels take the seed from the plan)
    int32_t pad;
};

struct IsArgs {
    McArgs mc;             // work items over streams; item_split unused
    const IsTable *table;
};

// Test hook: the points (and sum z^2/2) of one stream at given sample indices.
struct IsDebugArgs {
    const IsTable *table;
    const uint64_t *index;     // n sample indices
    double *u_out;             // n x d
    double *hz_out;            // n
    uint64_t n;
    uint64_t id;
    int32_t prec;
};

// Stream ids with this bit set draw from the uniform density of the box.
constexpr uint64_t kIsUniformStream = uint64_t(1) << 63;

template <int NX, int NT>
hipError_t launch_is_shape(const LaunchSpec &spec, const IsArgs &args, hipStream_t stream);
template <int NX, int NT>
hipError_t is_kernel_info_shape(const LaunchSpec &spec, KernelInfo *info);
template <int NX, int NT>
hipError_t launch_is_debug_shape(const IsDebugArgs &args, hipStream_t stream);

#define BFI_DECLARE_IS_SHAPE(NX, NT)                                                         \
    extern template hipError_t launch_is_shape<NX, NT>(const LaunchSpec &, const IsArgs &,    \
                                                       hipStream_t);                         \
    extern template hipError_t is_kernel_info_shape<NX, NT>(const LaunchSpec &, KernelInfo *); \
    extern template hipError_t launch_is_debug_shape<NX, NT>(const IsDebugArgs &, hipStream_t);
BFI_SHAPES(BFI_DECLARE_IS_SHAPE)
#undef BFI_DECLARE_IS_SHAPE

}  // namespace bfi
