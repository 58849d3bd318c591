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
    k.source[0][0] = k_source<N, E, EL, false, false>;
    k.source[0][1] = k_source<N, E, EL, false, true>;
    k.source[1][0] = k_source<N, E, EL, true, false>;
    k.source[1][1] = k_source<N, E, EL, true, true>;
    k.density_p[0] = k.density_p[1] = nullptr;
    for (int i = 0; i < 8; ++i) {
        k.phase_p[i >> 2][(i >> 1) & 1][i & 1] = nullptr;
        k.source_p[i >> 2][(i >> 1) & 1][i & 1] = nullptr;
    }
    if constexpr (C::PIPE) {
        k.density_p[0] = k_densityp_bohm<N, E, EL, false>;
        k.density_p[1] = k_densityp_bohm<N, E, EL, true>;
    }
    // the persistent phase pass holds two prefetched spectra, two rows and the
    // static potential: only at 8 points per thread does that fit the registers
    if constexpr (C::PIPE && E == 8) {
        k.phase_p[0][0][0] = k_phasep_local<N, E, EL, false, false, false>;
        k.phase_p[0][0][1] = k_phasep_local<N, E, EL, false, false, true>;
        k.phase_p[0][1][0] = k_phasep_local<N, E, EL, false, true, false>;
        k.phase_p[0][1][1] = k_phasep_local<N, E, EL, false, true, true>;
        k.phase_p[1][0][0] = k_phasep_local<N, E, EL, true, false, false>;
        k.phase_p[1][0][1] = k_phasep_local<N, E, EL, true, false, true>;
        k.phase_p[1][1][0] = k_phasep_local<N, E, EL, true, true, false>;
        k.phase_p[1][1][1] = k_phasep_local<N, E, EL, true, true, true>;
        k.source_p[0][0][1] = k_sourcep<N, E, EL, false, false, true>;
        k.source_p[0][1][0] = k_sourcep<N, E, EL, false, true, false>;
        k.source_p[0][1][1] = k_sourcep<N, E, EL, false, true, true>;
        k.source_p[1][0][1] = k_sourcep<N, E, EL, true, false, true>;
        k.source_p[1][1][0] = k_sourcep<N, E, EL, true, true, false>;
        k.source_p[1][1][1] = k_sourcep<N, E, EL, true, true, true>;
    }
    return k;
}

template <int N> static const LKernels *local_table(int v)
{
    // the one-tile kernels of variants 2 and 3 are those of 0 and 1 (same
    // tiles); 2 and 3 add the persistent forms
    static const LKernels k[5] = {make_local_kernels<N, 0>(), make_local_kernels<N, 1>(),
                                  make_local_kernels<N, 2>(), make_local_kernels<N, 3>(),
                                  make_local_kernels<N, 4>()};
    return &k[v];
}

// Fields of the non-minimal coupling on a grid (see nmc_point): one thread
// per point, x_j = -L/2 + j L/N per axis, minimum-image distance from c.
__global__ void k_nmc_fields(int ndim, int n0, int n1, int n2, double L0, double L1, double L2, double c0,
                             double c1, double c2, double lambda, double r0, double nu, double r_min,
                             float *gamma, float *beta, float *V, long long P)
{
    const int n[3] = {n0, n1, n2};
    const double L[3] = {L0, L1, L2}, c[3] = {c0, c1, c2};
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < P;
         q += (long long)gridDim.x * blockDim.x) {
        long long rem = q;
        double r2 = 0.0;
        for (int d = ndim - 1; d >= 0; --d) {
            const int j = (int)(rem % n[d]);
            rem /= n[d];
            double x = -0.5 * L[d] + j * (L[d] / n[d]) - c[d];
            x -= L[d] * floor(x / L[d] + 0.5);
            r2 += x * x;
        }
        double gm, bt, v;
        nmc_point(sqrt(r2), lambda, r0, nu, r_min, &gm, &bt, &v);
        if (gamma) gamma[q] = (float)gm;
        if (beta) beta[q] = (float)bt;
        if (V) V[q] = (float)v;
    }
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

hipError_t launch_nmc_fields(int ndim, const int *n, const double *L, const double *c, double lambda, double r0,
                             double nu, double r_min, float *gamma, float *beta, float *V, hipStream_t stream)
{
    long long P = 1;
    int nn[3] = {1, 1, 1};
    double LL[3] = {1.0, 1.0, 1.0}, cc[3] = {0.0, 0.0, 0.0};
    for (int d = 0; d < ndim; ++d) {
        nn[d] = n[d];
        LL[d] = L[d];
        cc[d] = c[d];
        P *= n[d];
    }
    hipLaunchKernelGGL(k_nmc_fields, dim3(2048), dim3(256), 0, stream, ndim, nn[0], nn[1], nn[2], LL[0], LL[1],
                       LL[2], cc[0], cc[1], cc[2], lambda, r0, nu, r_min, gamma, beta, V, P);
    return hipGetLastError();
}
