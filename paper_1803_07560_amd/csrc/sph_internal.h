// Internal interface of the sampler in spherical coordinates (sph_kernels.hip)
// for the host runtime.  Not part of the public ABI.
//
// The cube [-B, B]^d is cut into radial shells rho_lo <= |u| < rho_hi; each
// shell is sampled uniformly in its volume (direction from normalised normals,
// radius rho = rho_hi (t + v (1 - t))^(1/d) with t = (rho_lo / rho_hi)^d) and a
// sample weighs exp(-S) inside the cube, 0 outside.
#pragma once

#include "internal.h"

namespace bfi {

// Largest lattice the sampler is compiled for (the normals and the point are
// held in registers).
constexpr int kSphMaxD = 32;

struct SphArgs {
    McArgs mc;              // work items over shells (EvalParams: ids, offsets, coef, seed)
    const double *shell64;  // per shell: rho_hi, t
    const float *shell32;   // the same in FP32
    double box64;           // B
    float box32;
};

// Test hook: the points of one shell at given sample indices.
struct SphDebugArgs {
    const uint64_t *index;  // n sample indices
    double *out;            // n x d
    uint64_t n;
    uint64_t id;
    double rho_hi, t;
    uint32_t seed_lo, seed_hi;
    int32_t prec;
};

template <int NX, int NT>
hipError_t launch_sph_shape(const LaunchSpec &spec, const SphArgs &args, hipStream_t stream);
template <int NX, int NT>
hipError_t sph_kernel_info_shape(const LaunchSpec &spec, KernelInfo *info);
template <int NX, int NT>
hipError_t launch_sph_debug_shape(const SphDebugArgs &args, hipStream_t stream);

#define BFI_DECLARE_SPH_SHAPE(NX, NT)                                                          \
    extern template hipError_t launch_sph_shape<NX, NT>(const LaunchSpec &, const SphArgs &,    \
                                                        hipStream_t);                          \
    extern template hipError_t sph_kernel_info_shape<NX, NT>(const LaunchSpec &, KernelInfo *); \
    extern template hipError_t launch_sph_debug_shape<NX, NT>(const SphDebugArgs &, hipStream_t);
BFI_SHAPES(BFI_DECLARE_SPH_SHAPE)
#undef BFI_DECLARE_SPH_SHAPE

}  // namespace bfi
