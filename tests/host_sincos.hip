// Host build of the solver's FP64 sincos routines (the same inline functions
// the phase passes run on the GPU), printing sin, cos of sincos_fp64 and then
// of the table form sincos_tab for angles read from stdin.
#include <cstdio>
#include "gsn_kernels.hpp"

int main()
{
    double2 tab[gsn::kSinCosTable];
    gsn::fill_sincos_table(tab);
    double th;
    while (std::scanf("%lf", &th) == 1) {
        double s, c, s2, c2;
        gsn::sincos_fp64(th, &s, &c);
        gsn::sincos_tab(th, tab, &s2, &c2);
        std::printf("%.17g %.17g %.17g %.17g\n", s, c, s2, c2);
    }
    return 0;
}
