// Host check of the FP64 weight exponential the kernels use (exp64.hpp): the
// same IEEE operations (fma, rint, ldexp) compiled for the host give the same
// bits as on the GPU.  Against expl (64-bit significand): the largest error in
// units in the last place over random arguments, and the special values.
// Prints "max_ulp <e> frac_above_half <f>" and the specials as hex floats.
#include <cmath>
#include <cstdio>
#include <random>

#include "exp64.hpp"

static double ulp_error(double got, long double want)
{
    const double w = static_cast<double>(want);
    if (w == 0.0)
        return got == 0.0 ? 0.0 : 1e300;
    double ulp = std::nextafter(std::fabs(w), INFINITY) - std::fabs(w);
    if (std::fabs(w) < 0x1p-1022)
        ulp = 0x1p-1074;
    return static_cast<double>(std::fabs(static_cast<long double>(got) - want) /
                               static_cast<long double>(ulp));
}

int main()
{
    std::mt19937_64 gen(20260311);
    std::uniform_real_distribution<double> wide(-746.0, 0.0), unit(-1.0, 0.0), mid(-40.0, 0.0);
    double worst = 0.0, worst_x = 0.0;
    long above_half = 0;
    const long n = 3000000;
    for (long i = 0; i < n; ++i) {
        const double x = i % 3 == 0 ? wide(gen) : i % 3 == 1 ? unit(gen) : mid(gen);
        const double e = ulp_error(bfi::exp_weight(x), expl(static_cast<long double>(x)));
        above_half += e > 0.5;
        if (e > worst) {
            worst = e;
            worst_x = x;
        }
    }
    std::printf("max_ulp %.6f at %a frac_above_half %.6f\n", worst, worst_x,
                static_cast<double>(above_half) / n);
    const double special[] = {0.0, -0.0, -1e-300, -0x1p-1074, -745.0, -745.2, -746.0, -1e308,
                              -INFINITY, NAN, 1.0, 709.0, 710.0};
    for (double x : special)
        std::printf("%a %a\n", x, bfi::exp_weight(x));
    return 0;
}
