// gsn_c128.hip -- kernel tables of the FP64-storage (complex128) grids: the
// one-tile-per-block passes of every schedule variant's tile configuration,
// instantiated with double2 values in HBM and in LDS, so a step rounds
// nothing below FP64.  The persistent variants (p16, p8) use the tile
// configuration of e16 / e8 here.  Kept in its own translation unit so the
// library's objects build in parallel.
#include <hip/hip_runtime.h>

#include "gsn_host.hpp"

template <int N, int V> static NKernels make_kernels_c128()
{
    using C = Cfg<N, V>;
    using D = double2;
    // complex128 LDS slots: a strided tile keeps within 128 KiB
    constexpr int LL = 16L * C::LM_LINES * N > 131072L ? (int)(131072L / (16L * N)) : C::LM_LINES;
    constexpr int E = C::E, EL = C::EM_LINES;
    NKernels k;
    k.E = E;
    k.TPL = C::TPL;
    k.lm_lines = LL;
    k.em_lines = EL;
    k.em_fwd = k_em_fft<N, E, EL, -1, D>;
    k.em_inv = k_em_fft<N, E, EL, 1, D>;
    k.density = k_density<N, E, EL, false, false, D>;
    k.density_store = k_density<N, E, EL, true, false, D>;
    k.density_real = nullptr;   // no potential readout on these grids
    k.phase = k_phase<N, E, EL, false, false, D>;
    k.phase_real = k_phase<N, E, EL, false, true, D>;
    k.phase_energy = k_phase<N, E, EL, true, false, D>;
    k.potential = nullptr;
    k.lm_fwd = k_lm<N, E, LL, LM_FWD, D>;
    k.lm_inv = k_lm<N, E, LL, LM_INV, D>;
    k.lm_kin = k_lm<N, E, LL, LM_KIN, D>;
    k.lm_kern = k_lm<N, E, LL, LM_KERN, D>;
    k.lm_kin_energy = k_lm<N, E, LL, LM_KIN_ENERGY, D>;
    for (int m = 0; m < 4; ++m) k.lmp[m] = nullptr;
    k.em_pipe = false;
    return k;
}

template <int N> static const NKernels *table_c128(int v)
{
    static const NKernels k[3] = {make_kernels_c128<N, 0>(), make_kernels_c128<N, 1>(), make_kernels_c128<N, 4>()};
    return &k[v == 4 ? 2 : (v & 1)];
}

const NKernels *kernels_for_c128(int N, int v)
{
    if (v < 0 || v >= kNumVariants) v = 0;
    switch (N) {
    case 8: return table_c128<8>(v);
    case 16: return table_c128<16>(v);
    case 32: return table_c128<32>(v);
    case 64: return table_c128<64>(v);
    case 128: return table_c128<128>(v);
    case 256: return table_c128<256>(v);
    case 512: return table_c128<512>(v);
    case 1024: return table_c128<1024>(v);
    case 2048: return table_c128<2048>(v);
    default: return nullptr;
    }
}

hipError_t launch_mass_c128(const void *psi, long long P, double *partials, int nb, hipStream_t s)
{
    hipLaunchKernelGGL((k_mass<256, double2>), dim3(nb), dim3(256), 0, s, (const double2 *)psi, P, partials);
    return hipGetLastError();
}

hipError_t launch_readout_c128(const void *psi, void *dst, int dst_c128, long long P, const DevState *st,
                               hipStream_t s)
{
    if (dst_c128)
        hipLaunchKernelGGL((k_readout<true, double2>), dim3(1024), dim3(256), 0, s, (const double2 *)psi, dst, P, st);
    else
        hipLaunchKernelGGL((k_readout<false, double2>), dim3(1024), dim3(256), 0, s, (const double2 *)psi, dst, P, st);
    return hipGetLastError();
}

hipError_t launch_from_c64(const void *src, void *dst, long long P, hipStream_t s)
{
    hipLaunchKernelGGL(k_from_c64, dim3(1024), dim3(256), 0, s, (const float2 *)src, (double2 *)dst, P);
    return hipGetLastError();
}
