// Host build of the solver's FP64 logarithm and exponential (the same inline
// functions the phase pass of the Eq. (15) local terms runs on the GPU),
// printing log_fp64(x) and exp_fp64(x) for values read from stdin.
#include <cstdio>
#include "gsn_kernels.hpp"

int main()
{
    double x;
    while (std::scanf("%lf", &x) == 1) std::printf("%.17g %.17g\n", gsn::log_fp64(x), gsn::exp_fp64(x));
    return 0;
}
