// gsn_host.hpp -- host-side helpers shared by the single-grid and batched
// solvers: error reporting, the per-length kernel tables with their schedule
// variants, and FP64 table generation.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "gsn.h"
#include "gsn_kernels.hpp"

using namespace gsn;

// ------------------------------------------------------------------ errors
// The last error message of this host thread (defined in gsn_api.hip).
extern thread_local std::string g_last_error;

static inline gsn_status fail(gsn_status s, const std::string &msg)
{
    g_last_error = msg;
    return s;
}

#define HIP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(GSN_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));    \
    } while (0)


// ------------------------------------------------------------------ kernel tables per N
struct NKernels {
    int E, TPL, lm_lines, em_lines;
    void (*em_fwd)(EmArgs);
    void (*em_inv)(EmArgs);
    void (*density)(EmArgs);
    void (*density_store)(EmArgs);
    void (*density_real)(EmArgs);   // real-space psi rows in (potential readout)
    void (*phase)(EmArgs);
    void (*phase_real)(EmArgs);
    void (*phase_energy)(EmArgs);
    void (*potential)(EmArgs);
    void (*lm_fwd)(LmArgs);
    void (*lm_inv)(LmArgs);
    void (*lm_kin)(LmArgs);
    void (*lm_kern)(LmArgs);
    void (*lm_kin_energy)(LmArgs);
    // pipelined persistent forms of LM_FWD .. LM_KERN (null: not in this variant)
    void (*lmp[4])(LmArgs);
    int lmp_threads = 0;   // their block size when it is not lm_threads()
    // density / phase entries are the pipelined persistent kernels
    bool em_pipe;
    int lm_threads() const { return lm_lines * TPL; }
    int em_threads() const { return em_lines * TPL; }
};

// Schedule variants: E points per thread (16 or 8) for every pass kind, and
// for the strided-axis (LM), density and phase passes either one tile per
// block or persistent blocks that prefetch their next tile ("p16", "p8");
// "s8" is the small-tile form for small grids.  The EM tile holds
// 256/TPL rows (at most 64); the LM tile holds LINES columns chosen so that a
// tile moves 128-byte contiguous segments per row where the block's thread
// budget allows (long lines get 64- or 32-byte segments).  On 512-point lines
// the strided passes of "p8" run in the two-butterfly form (16 points per
// thread of the same 8-point plan, two 512-thread blocks per CU, the next tile
// loaded after the stores), bitwise equal to the one-butterfly form.  The
// batched solver offers the first kNumBatchVariants.
constexpr int kNumVariants = 5;
constexpr int kNumBatchVariants = 4;
static const char *kVariantNames[kNumVariants] = {"e16", "e8", "p16", "p8", "s8"};

// "s8": 8 points per thread with the smallest tiles that still fill a
// wavefront (one row pair per block where a row takes 64 threads, four
// strided lines per block), for grids too small to give every CU a tile.
template <int N, int V> struct Cfg {
    static constexpr bool SMALL = V == 4;
    static constexpr int E0 = (V & 1) || SMALL ? 8 : 16;
    static constexpr bool PIPE = V == 2 || V == 3;
    static constexpr int E = N < E0 ? N : E0;
    static constexpr int TPL = N / E;
    // 16 lines (128-byte row segments; more for very short lines) while the
    // block stays within its thread budget: 512 threads at 16 points per
    // thread (above that the registers spill), 1024 at 8
    static constexpr int LM_MAXT = E0 >= 16 ? 512 : 1024;
    static constexpr int LM_WANT = TPL <= 4 ? 64 : TPL <= 8 ? 32 : 16;
    static constexpr int LM_LINES = SMALL ? (TPL >= 16 ? 4 : 64 / TPL)
                                          : LM_WANT * TPL <= LM_MAXT ? LM_WANT : LM_MAXT / TPL;
    static constexpr int EM_LINES = SMALL ? (TPL >= 64 ? 1 : 64 / TPL)
                                          : (256 / TPL) > 64 ? 64 : (256 / TPL) < 1 ? 1 : 256 / TPL;
};

// Kernel table of length N, schedule variant v (defined in gsn_api.hip, the
// only translation unit that instantiates the single-grid kernels of the Kerr
// model).
const NKernels *kernels_for(int N, int v = 0);

// Kernel table of the FP64-storage (complex128) grids, one tile per block in
// the tile configuration of variant v (defined in gsn_c128.hip), and its
// storage-specific helpers: mass partials, read-out with the global phase
// (to complex128 or complex64), and complex64 input.
const NKernels *kernels_for_c128(int N, int v = 0);
hipError_t launch_mass_c128(const void *psi, long long P, double *partials, int nb, hipStream_t s);
hipError_t launch_readout_c128(const void *psi, void *dst, int dst_c128, long long P, const DevState *st,
                               hipStream_t s);
hipError_t launch_from_c64(const void *src, void *dst, long long P, hipStream_t s);

// Kernels of the local terms of Eq. (15) (pressure and Bohm potential) of
// length N in the tile configuration of schedule variant v; one tile per block
// (defined in gsn_local.hip).
struct LKernels {
    void (*density)(EmArgs);         // also the half spectrum of sqrt(rho)
    void (*density_store)(EmArgs);   // ... and stores real-space psi
    void (*phase)(EmArgs);
    void (*phase_real)(EmArgs);
    void (*phase_energy)(EmArgs);
    void (*lm_lap)(LmArgs);          // FFT, -|k|^2, inverse FFT
    void (*source[2][2])(EmArgs);    // [real-space psi in][lap(rho) in]
    // persistent prefetching forms (null outside the p16 / p8 variants):
    // density with sqrt(rho) [stores psi]; phase [real-space psi][Bohm][static potential]
    void (*density_p[2])(EmArgs);
    void (*phase_p[2][2][2])(EmArgs);
    void (*source_p[2][2][2])(EmArgs);   // [real-space psi in][lap(rho) in][gamma field]
};
const LKernels *local_kernels_for(int N, int v = 0);

// Fill the non-minimal-coupling fields (any output may be null) of an ndim
// grid with extents n, lengths L and centre c on the stream.
hipError_t launch_nmc_fields(int ndim, const int *n, const double *L, const double *c, double lambda, double r0,
                             double nu, double r_min, float *gamma, float *beta, float *V, hipStream_t stream);

// Blocks of kernel fn (threads per block) resident on the whole device at
// once (occupancy x compute units): the grid of a persistent kernel; 0 if
// the runtime cannot say.  Cached per kernel and device.
int persistent_blocks(const void *fn, int threads);

// wavenumber of DFT index j on an axis with N points and length L
static inline double wavenumber(int j, int N, double L)
{
    const int jj = j < N / 2 ? j : j - N;
    return 2.0 * M_PI * (double)jj / L;
}

static inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

static inline bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
