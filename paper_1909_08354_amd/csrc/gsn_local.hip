// gsn_local.hip -- kernels of the local terms of Eq. (15) (polytropic pressure
// and Bohm potential) for the single-grid solver: the density pass that also
// transforms sqrt(rho), the general phase pass, its energy form, and the
// Laplacian multiplier pass.  One tile per block, in the tile configuration of
// each schedule variant (the persistent variants share the configuration of
// their one-tile-per-block counterparts).  Instantiated here, in a translation
// unit of its own, so the library's objects build in parallel.
#include <hip/hip_runtime.h>

#include "gsn_host.hpp"

template <int N, int V> static LKernels make_local_kernels()
{
    using C = Cfg<N, V>;
    constexpr int E = C::E, LL = C::LM_LINES, EL = C::EM_LINES;
    LKernels k;
    k.density = k_density<N, E, EL, false, true>;
    k.density_store = k_density<N, E, EL, true, true>;
    k.phase = k_phase_local<N, E, EL, false, false>;
    k.phase_real = k_phase_local<N, E, EL, false, true>;
    k.phase_energy = k_phase_local<N, E, EL, true, false>;
    k.lm_lap = k_lm<N, E, LL, LM_LAP>;
    return k;
}

template <int N> static const LKernels *local_table(int v)
{
    // variants 2 and 3 use the tile configuration of 0 and 1
    static const LKernels k[3] = {make_local_kernels<N, 0>(), make_local_kernels<N, 1>(),
                                  make_local_kernels<N, 4>()};
    return &k[v == 4 ? 2 : (v & 1)];
}

const LKernels *local_kernels_for(int N, int v)
{
    if (v < 0 || v >= kNumVariants) v = 0;
    switch (N) {
    case 8: return local_table<8>(v);
    case 16: return local_table<16>(v);
    case 32: return local_table<32>(v);
    case 64: return local_table<64>(v);
    case 128: return local_table<128>(v);
    case 256: return local_table<256>(v);
    case 512: return local_table<512>(v);
    case 1024: return local_table<1024>(v);
    case 2048: return local_table<2048>(v);
    default: return nullptr;
    }
}
