// Host build of the solver's FP64 sincos (the same inline function the phase
// pass runs on the GPU), printing sin, cos for angles read from stdin.
#include <cstdio>
#include "gsn_kernels.hpp"

int main()
{
    double th;
    while (std::scanf("%lf", &th) == 1) {
        double s, c;
        gsn::sincos_fp64(th, &s, &c);
        std::printf("%.17g %.17g\n", s, c);
    }
    return 0;
}
