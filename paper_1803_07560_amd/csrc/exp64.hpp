// e^x in double precision for the weights e^{-S} of the FP64 form, where the
// action S >= 0 (x <= 0; also right up to x = 709, beyond which it gives +inf).
// Plain C++ on clang/GCC builtins, so the same arithmetic compiles for the GPU
// and for a host check; the includer sets BFI_HD (e.g. __device__).
//
// Method (Cody and Waite's argument reduction, then a Taylor series):
//   k = rint(x / ln 2),  r = (x - k ln2_hi) - k ln2_lo,  |r| <= ln 2 / 2 + tiny.
//   ln2_hi holds the leading 41 significant bits of ln 2, so k ln2_hi is exact for
//   |k| < 2^12 and x - k ln2_hi is exact; ln2_lo = ln 2 - ln2_hi rounded.
//   e^r = sum_{j=0..13} r^j / j! in Horner form: the first omitted term,
//   (ln2/2)^14 / 14!, is below 2^-57 of e^r.
//   e^x = 2^k e^r by ldexp, which rounds once into the subnormal range.
// x below -746 is raised to -746, whose exponential already rounds to 0, so -inf
// gives 0; NaN stays NaN.  One compare, two selects, 18 double operations.
#pragma once

#ifndef BFI_HD
#define BFI_HD
#endif

namespace bfi {
namespace expk {
// 1/ln 2, and ln 2 split as described above (derived from ln 2 to 60 digits)
constexpr double kInvLn2 = 0x1.71547652b82fep+0;
constexpr double kLn2Hi = 0x1.62e42fefa3000p-1;
constexpr double kLn2Lo = 0x1.3de6af278ece6p-42;
// 1/j!, j = 2..13, rounded to double
constexpr double kInvFact[12] = {
    0x1.0000000000000p-1,  0x1.5555555555555p-3,  0x1.5555555555555p-5,  0x1.1111111111111p-7,
    0x1.6c16c16c16c17p-10, 0x1.a01a01a01a01ap-13, 0x1.a01a01a01a01ap-16, 0x1.71de3a556c734p-19,
    0x1.27e4fb7789f5cp-22, 0x1.ae64567f544e4p-26, 0x1.1eed8eff8d898p-29, 0x1.6124613a86d09p-33};
}  // namespace expk

// The fused multiply-add of the polynomial steps and where its coefficients
// come from; a caller may pass its own (same arithmetic, another encoding or
// register class), as the GPU kernels do.
struct BuiltinFma {
    BFI_HD static double step(double a, double b, double c) { return __builtin_fma(a, b, c); }
    BFI_HD static constexpr double coef(int j) { return expk::kInvFact[j]; }
};

template <class Fma = BuiltinFma>
BFI_HD inline double exp_weight(double x, const Fma &fma = Fma())
{
    x = x < -746.0 ? -746.0 : x;
    const double k = __builtin_rint(x * expk::kInvLn2);
    double r = __builtin_fma(-k, expk::kLn2Hi, x);
    r = __builtin_fma(-k, expk::kLn2Lo, r);
    double p = fma.coef(11);
    for (int j = 10; j >= 0; --j)
        p = fma.step(p, r, fma.coef(j));
    p = fma.step(p, r, 1.0);
    p = fma.step(p, r, 1.0);
    return __builtin_ldexp(p, static_cast<int>(k));
}
}  // namespace bfi
