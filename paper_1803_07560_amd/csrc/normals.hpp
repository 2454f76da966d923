// Standard normals from Philox words on the device (Box-Muller), shared by the
// samplers that draw Gaussian numbers: the Gaussian-proposal sampler and the
// sampler in spherical coordinates.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bfi {
namespace dev {

// Box-Muller: a standard normal pair from two words, u = (x + 1/2) 2^-32,
// radius sqrt(-2 ln u1), angle 2 pi u2.
__device__ __forceinline__ void box_muller(uint32_t x1, uint32_t x2, double &zc, double &zs)
{
    const double u1 = __fma_rn(static_cast<double>(x1), 0x1p-32, 0x1p-33);
    const double u2 = __fma_rn(static_cast<double>(x2), 0x1p-32, 0x1p-33);
    const double r = sqrt(-2.0 * log(u1));
    double s, c;
    sincospi(2.0 * u2, &s, &c);
    zc = r * c;
    zs = r * s;
}
// FP32: hardware log2, square root and sine/cosine (whose argument is in
// turns, so the angle 2 pi u2 is u2 itself)
__device__ __forceinline__ void box_muller(uint32_t x1, uint32_t x2, float &zc, float &zs)
{
    const float u1 = __fmaf_rn(static_cast<float>(x1), 0x1p-32f, 0x1p-33f);
    const float u2 = __fmaf_rn(static_cast<float>(x2), 0x1p-32f, 0x1p-33f);
    constexpr float kMinus2Ln2 = -1.38629436111989061883f;
    const float r = __builtin_amdgcn_sqrtf(kMinus2Ln2 * __builtin_amdgcn_logf(u1));
    zc = r * __builtin_amdgcn_cosf(u2);
    zs = r * __builtin_amdgcn_sinf(u2);
}

}  // namespace dev
}  // namespace bfi
