/*
 * gsn.h -- C ABI of the MI355X (gfx950) split-step Schroedinger-Newton solver.
 *
 * The library advances the generalised Schroedinger-Newton system of
 * arXiv:1909.08354 (Sec. II, Eq. (1)-(2)) in its optics form, Eq. (3) with
 * k = k0 = 1:
 *
 *     i d(psi)/dz = -a lap(psi) - (g |psi|^2 + phi) psi,
 *     phi_hat(k)  = K(k) rho_hat(k),  rho = |psi|^2,
 *     K(k)        = c_newton/|k|^2 [k != 0] + c_yukawa/(|k|^2 + m_yukawa^2) + c_contact,
 *
 * i.e. Eq. (1) with A = -a, B = -1, G(rho) = -g rho, and the Fourier form of
 * Eq. (2) / Eq. (4) / Eq. (5) / Eq. (8) with constant coefficients (Newtonian
 * 1/k^2 plus its Yukawa-type correction plus a contact term; Eq. (12) with
 * alpha = 0 is c_newton = gamma, c_contact = -beta).  The time step is the
 * symmetric split-step Fourier method with a spectral solve for the potential
 * (Sec. III).  The Newtonian k = 0 term is dropped; the uniform part K(0) <rho>
 * of the potential is a pure global phase that is accumulated in FP64 and
 * applied when psi is read.
 *
 * Grid: 2-D or 3-D, C order (slowest axis first, last axis contiguous),
 * periodic, every extent a power of two in [8, 2048]; x_j = -L/2 + j L/N.
 * psi is complex, interleaved (re, im), P = prod(n) elements.
 *
 * Precision: psi, rho and phi are stored in HBM as complex64/float; all FFT
 * arithmetic, phases and multipliers run in FP64 in registers; mass, energy
 * and the k = 0 potential term are FP64 reductions.
 *
 * Conventions shared by every call:
 *   - every function returns gsn_status; nothing throws, nothing aborts;
 *   - gsn_last_error() returns a thread-local message for the last failure;
 *   - arguments are validated before any HIP call;
 *   - no call keeps a caller pointer after it returns, except the workspace
 *     given to gsn_create / gsn_batch_create / gsn_corrector_create, which the
 *     caller owns and must keep alive (and unused by others) until destroy;
 *   - work is queued on the stream given at creation (NULL = default stream);
 *     calls documented as synchronising wait for that stream;
 *   - one host thread per handle at a time.
 */
#ifndef GSN_H
#define GSN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GSN_OK = 0,
    GSN_EINVAL = 1,        /* bad argument (null pointer, bad size, non-finite value) */
    GSN_EUNSUPPORTED = 2,  /* valid but not supported (extent not a power of two in range) */
    GSN_EWORKSPACE = 3,    /* workspace too small or misaligned (needs 256-byte alignment) */
    GSN_EHIP = 4,          /* a HIP runtime call failed; see gsn_last_error() */
    GSN_ENONFINITE = 5,    /* the fused FP64 mass became NaN or Inf */
    GSN_ESTATE = 6         /* call out of order (e.g. step before psi/coefficients are set) */
} gsn_status;

typedef enum { GSN_C64 = 0, GSN_C128 = 1 } gsn_dtype;

typedef struct gsn_grid_ *gsn_grid;

/* K(k) = c_newton/|k|^2 [k != 0] + c_yukawa/(|k|^2 + m_yukawa^2) + c_contact
   (Eq. (2) in Fourier form; Eq. (4)-(5) give the Yukawa family with
   m_yukawa = 1/sigma or sqrt(2q/nu); Eq. (8) gives Newton plus Yukawa). */
typedef struct {
    double c_newton;
    double c_yukawa;
    double m_yukawa;   /* must be > 0 when c_yukawa != 0 */
    double c_contact;
} gsn_kernel;

/* Bytes of device workspace gsn_create needs for this grid (ndim 2 or 3,
   n[] in C order).  Includes psi, the half-spectrum of rho/phi, an energy
   scratch copy of psi, FP64 reduction partials and FP64 tables. */
gsn_status gsn_workspace_bytes(int ndim, const int32_t n[], size_t *bytes);

/* Create a solver on the current HIP device.  d_workspace: device pointer,
   256-byte aligned, at least gsn_workspace_bytes() bytes, owned by the caller.
   L[]: box lengths > 0 (C order).  hip_stream: a hipStream_t or NULL.
   Defaults after creation: a = 1/2, g = 0, dz = 0 (must be set), kernel = 0. */
gsn_status gsn_create(gsn_grid *out, int ndim, const int32_t n[], const double L[],
                      void *d_workspace, size_t bytes, void *hip_stream);

/* The same for a grid whose values live in HBM as complex128 (storage =
   GSN_C128): psi and the rho / phi half spectra in FP64 and every LDS
   exchange in FP64, so no value of a step is rounded below double precision
   (the precision of the paper's own runs); twice the bytes per point.
   storage = GSN_C64 is gsn_workspace_bytes / gsn_create.  FP64-storage grids
   run the one-tile-per-block passes in every schedule variant (p16 and p8 use
   the tile configuration of e16 and e8); the Eq. (15) local terms, source
   fields, potential readout and corrected steps stay complex64-only
   (GSN_EUNSUPPORTED).  gsn_set_psi / gsn_get_psi convert either dtype. */
gsn_status gsn_workspace_bytes_ex(int ndim, const int32_t n[], int storage, size_t *bytes);
gsn_status gsn_create_ex(gsn_grid *out, int ndim, const int32_t n[], const double L[], int storage,
                         void *d_workspace, size_t bytes, void *hip_stream);
gsn_status gsn_destroy(gsn_grid grid);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): the same
   grid as gsn_create (complex64 storage), with its workspace in the library's
   static per-device array of 64 MiB instead of a caller buffer; nothing is
   allocated on the device.  Grids whose gsn_workspace_bytes exceed 64 MiB are
   rejected with GSN_EWORKSPACE.  The array is shared by every such grid on a
   device, so one may be alive per device at a time: a second call before
   gsn_destroy of the first returns GSN_ESTATE (without that check two grids
   would race on the same memory).  The array keeps the last grid's contents;
   creation resets every value a step reads before writing it.  Each GPU the
   library runs on holds its copy until the process ends. */
gsn_status gsn_create_static(gsn_grid *out, int ndim, const int32_t n[], const double L[], void *hip_stream);

/* Set the nonlocal kernel (see gsn_kernel).  All values finite. */
gsn_status gsn_set_kernel(gsn_grid grid, const gsn_kernel *kernel);

/* Set the kinetic coefficient a (Eq. (3): 1/2), the local coefficient g
   (Kerr; Eq. (16) with n = 2 gives g = -2w) and the step dz (finite, != 0). */
gsn_status gsn_set_coefficients(gsn_grid grid, double a_kin, double g_local, double dz);

/* Eq. (1)-(2) with their own constants:
     i psi_t = A lap psi + B phi psi + G psi,   lap phi + C phi = D |psi|^2,
   G = -g |psi|^2 (- the local terms below).  Sets the kinetic coefficient
   a = -A (a later gsn_set_coefficients sets a again) and the kernel
   K = B D / (|k|^2 - C): the Newtonian member c_newton = B D for C = 0, else
   the screened member c_yukawa = B D with squared mass -C, which for C > 0 is
   the resonant Helmholtz kernel.  C > 0 equal to |k|^2 of a grid wavenumber
   (relative tolerance 1e-12) has no periodic solution: GSN_EINVAL.  The
   optics forms: Eq. (3) with k = k0 = 1 is A = -1/2, B = -1 (phi = Delta n);
   the thermo-optic Eq. (4) is C = -1/sigma^2, D = -zeta mu / kappa; the
   nematic Eq. (5) divided by nu is C = -2q/nu, D = -2/nu.  Synchronising. */
gsn_status gsn_set_equation(gsn_grid grid, double A, double B, double C, double D);

/* Local terms of Eq. (15) (Sec. II C): replace the Kerr term g rho of the
   phase by the local potential
     U = g rho + c_pressure f_n(max(rho, rho_floor))
               + c_bohm lap(sqrt rho) / (2 max(sqrt rho, sqrt rho_floor)),
     f_n(rho) = ln rho (n = 1),  n/(n-1) rho^(n-1) (n > 1 or n < 0),
   the polytropic pressure potential and the Bohm potential, with lap the
   spectral Laplacian.  Eq. (15) divided by nu maps to a = nu/2,
   c_bohm = -nu, c_pressure = -w/nu and c_newton = gamma/nu (for
   lap phi_N = gamma rho).  rho_floor >= 0 keeps ln rho, negative powers and the
   division finite where the density vanishes; it must be > 0 when the pressure
   term has n <= 1 or the Bohm term is on.  All zero (the default) is the Kerr
   model.  The Bohm term adds one real-to-complex transform pair per step (the
   passes "y_fwd_sqrt", "laplacian", "y_inv_lap"); the density and phase passes
   with these terms run one tile per block in every schedule variant.
   Validation failures return GSN_EINVAL and leave the grid unchanged.
   Synchronising. */
gsn_status gsn_set_local_terms(gsn_grid grid, double c_pressure, double n_pressure, double c_bohm,
                               double rho_floor);

/* Position-dependent coupling (Eq. (9)-(12)) and a static potential: the
   kernel acts on the source s = gamma(x) rho + beta(x) lap(rho) instead of rho,
   and V_ext(x) joins the phase, i psi_z = ... - (U + phi + V_ext) psi.  gamma,
   beta and V_ext are device arrays of count = P floats in C order (any other
   count with a field given: GSN_EINVAL), owned by the caller;
   the grid reads them on every step until they are replaced or cleared (pass
   NULL for an absent field: gamma = 1, beta = 0, V_ext = 0), so they must stay
   alive and unchanged meanwhile.  The pure non-minimal coupling of Eq. (12)
   (alpha = 0), lap phi_N = beta lap rho + gamma rho, with phi_C of Eq. (11), is
   c_newton = 1/nu with V_ext = -phi_C/nu (gsn_nmc_fields fills all three).
   beta adds the passes "y_fwd_src", "lap_rho", "y_inv_src" and every source
   field the x pass "x_source".  While gamma or beta is set the kernel must have
   K(0) = 0 (no screened or contact part: stepping returns GSN_EUNSUPPORTED),
   and gsn_energy, gsn_potential and gsn_step_corrected return
   GSN_EUNSUPPORTED; with V_ext alone the energy's local part includes
   -dV sum V_ext rho.  Synchronising. */
gsn_status gsn_set_source_fields(gsn_grid grid, const float *gamma, const float *beta, const float *V_ext,
                                 size_t count);

/* Fill caller device arrays of P floats with the fields of the pure
   non-minimal coupling on this grid's points (Eq. (9)-(11)): with r the
   periodic (minimum-image) distance from center (ndim doubles; NULL = the
   origin) and u = (r0 / (r + r0))^lambda,
     gamma = (1 - u) / 2,  beta = lambda u / (r + r0),  V_ext = -ln(1 - u) / nu,
   the last with r raised to r_min, since phi_C = ln(1 - u) diverges at the
   centre.  r0 = M / (4 pi) is the Schwarzschild radius of the mass M.  Any
   output may be NULL; count is the length of each output (at least P).  lambda, r0, r_min > 0 and nu != 0, else GSN_EINVAL.
   Synchronising. */
gsn_status gsn_nmc_fields(gsn_grid grid, double lambda, double r0, double nu, const double *center,
                          double r_min, float *gamma, float *beta, float *V_ext, size_t count);

/* Load psi (P complex values, C order) from host (src_on_device = 0) or
   device memory, as complex64 or complex128.  Resets the global phase and the
   step count.  Synchronising for host sources. */
gsn_status gsn_set_psi(gsn_grid grid, const void *src, int src_on_device, int dtype);

/* Advance nsteps >= 0 symmetric split steps (Sec. III):
   L(dz/2) [N(dz) L(dz)]^(nsteps-1) N(dz) L(dz/2).  Asynchronous on the stream;
   a non-finite fused mass is reported by the next synchronising call. */
gsn_status gsn_step(gsn_grid grid, int64_t nsteps);

/* Wait for queued work; returns GSN_ENONFINITE if any step's mass was not finite. */
gsn_status gsn_sync(gsn_grid grid);

/* Copy psi (with the accumulated global phase applied in FP64) to host or
   device memory as complex64 or complex128.  Synchronising. */
gsn_status gsn_get_psi(gsn_grid grid, void *dst, int dst_on_device, int dtype);

/* FP64 mass M = dV sum |psi|^2 of the current state.  Synchronising. */
gsn_status gsn_mass(gsn_grid grid, double *mass);

/* FP64 energy of the current state (the Hamiltonian of the equation):
   e[0] total, e[1] kinetic a dV/P sum |k|^2 |psi_hat|^2, e[2] local
   -(g/2) dV sum rho^2 - c_pressure dV sum G_n(rho) + (c_bohm/2) dV sum |grad sqrt rho|^2
   (G_n' = f_n(max(rho, rho_floor)); the Bohm part is evaluated as
   -(c_bohm/2) dV sum sqrt(rho) lap(sqrt rho)) - dV sum V_ext rho, e[3] nonlocal
   -(1/2) dV sum rho phi.  Synchronising. */
gsn_status gsn_energy(gsn_grid grid, double e[4]);

/* Global phase accumulated since gsn_set_psi (FP64) and steps taken. */
gsn_status gsn_phase(gsn_grid grid, double *theta, int64_t *steps);

/* Per-pass timing: runs nsteps steady-state steps on the grid's stream, each
   pass launched with a start and a stop HIP event bound to its dispatch
   (hipExtLaunchKernel), so that an event pair spans the kernel's own
   execution and the launches follow each other as in gsn_step, with no
   marker between them; writes the average milliseconds per launch of each
   pass into ms[] (npass entries, order as gsn_pass_name()).  The state is
   advanced exactly as gsn_step(nsteps) would.  Synchronising. */
gsn_status gsn_profile_passes(gsn_grid grid, int64_t nsteps, double *ms, int npass);
int gsn_pass_count(gsn_grid grid);
const char *gsn_pass_name(gsn_grid grid, int i);
/* Model HBM bytes per point that pass i moves (reads + writes). */
double gsn_pass_bytes_per_point(gsn_grid grid, int i);

/* FFT schedule variants.  Every pass can run with 16 or 8 points per thread
   (variant 0 "e16", variant 1 "e8"); variants 2 "p16" and 3 "p8" run the
   strided-axis, density and phase passes with persistent blocks that
   prefetch their next tile while transforming the current one (the
   operations of e16 / e8; on 512-point strided lines p8 runs the same
   8-point plan with 16 points per thread in two blocks per compute unit,
   loading its next tile after the stores, bitwise equal to e8); variant 4
   "s8" uses 8 points per thread with the
   smallest tiles that fill a wavefront, for grids too small to give every
   compute unit a tile.  A variant changes the Stockham radix plan, the
   tile shape and the LDS footprint, never the result beyond rounding.
   gsn_autotune times every variant of every pass of this grid (iters launches
   each, on a scratch copy of psi: the state is not modified) and keeps the
   fastest.  If the environment variable GSN_AUTOTUNE_CACHE names a file,
   choices are read from it (key: GPU architecture, grid shape, pass) and new
   ones appended.  Synchronising. */
int gsn_variant_count(void);
const char *gsn_variant_name(int v);
gsn_status gsn_autotune(gsn_grid grid, int iters);
/* Nonlinear sub-step layout.  Mode 0: the phase pass recomputes psi from its
   x-spectrum (the density pass writes only the rho half spectrum).  Mode 1:
   the density pass also writes real-space psi in place, and the phase pass
   reads it instead of transforming again (+8 bytes per point, two fewer FFTs
   per pair of rows).  Both give the same result up to rounding; gsn_autotune
   picks one by timing whole steps (kinetic passes and nonlinear sub-step). */
gsn_status gsn_set_nonlinear_mode(gsn_grid grid, int mode);
gsn_status gsn_get_nonlinear_mode(gsn_grid grid, int *mode);
/* Current variant of every pass (npass >= gsn_pass_count entries). */
gsn_status gsn_get_schedule(gsn_grid grid, int *variants, int npass);
gsn_status gsn_set_schedule(gsn_grid grid, const int *variants, int npass);

/* ---------------------------------------------------------------- batches
   Many independent 2-D instances of uneven sizes, each with its own kernel
   K(k), coefficients a, g, dz and box, advanced together (parameter sweeps
   over the gravity model).  Instances of one shape form a group; each pass of
   a group is one launch over all its members, and every group's chain of
   launches is one branch of a single captured hipGraph, so gsn_batch_step is
   one hipGraphLaunch.  Results equal count independent gsn_grid runs up to
   rounding.  n and L are count x 2 arrays (C order per instance). */
typedef struct gsn_batch_ *gsn_batch;
gsn_status gsn_batch_workspace_bytes(int count, int ndim, const int32_t *n, size_t *bytes);
/* count in [1, 4096]; ndim must be 2.  Same workspace and stream rules as
   gsn_create. */
gsn_status gsn_batch_create(gsn_batch *out, int count, int ndim, const int32_t *n, const double *L,
                            void *d_workspace, size_t bytes, void *hip_stream);
gsn_status gsn_batch_destroy(gsn_batch batch);
/* Set instance i's kernel, coefficients and psi (host or device, c64/c128);
   resets its global phase.  Synchronising. */
gsn_status gsn_batch_set(gsn_batch batch, int i, const gsn_kernel *kernel, double a_kin, double g_local,
                         double dz, const void *psi, int src_on_device, int dtype);
/* Advance every instance by nsteps symmetric steps (same schedule as
   gsn_step); ordered after earlier work on the creation stream. */
gsn_status gsn_batch_step(gsn_batch batch, int64_t nsteps);
gsn_status gsn_batch_sync(gsn_batch batch);
gsn_status gsn_batch_get(gsn_batch batch, int i, void *dst, int dst_on_device, int dtype);
/* FP64 mass of every instance into masses[count].  Synchronising. */
gsn_status gsn_batch_mass(gsn_batch batch, double *masses);
gsn_status gsn_batch_phase(gsn_batch batch, int i, double *theta, int64_t *steps);
/* Execution mode: 0 = one captured hipGraph per step count (default);
   1 = one persistent kernel: 512-thread blocks pull (phase, instance, tile)
   work items in order from the queue of the XCD they run on (each instance
   belongs to one XCD's queue, the instances spread by size) and wait
   (bounded) on per-instance completion counters, so instances overlap across
   passes; extents 128..1024 only (GSN_EUNSUPPORTED otherwise); a wait that
   exceeds its spin limit, or a queue left undrained because no block ran on
   its XCD, is reported as GSN_EHIP by the next synchronising call;
   2 = the grouped launches of mode 0 issued directly. */
gsn_status gsn_batch_set_mode(gsn_batch batch, int mode);
/* Persistent-mode wait bound (iterations of ~50 ns, default 2^22) and a test
   hook: fail_item >= 0 makes the block that pulls that work item raise the
   queue error instead of running it (every block then leaves its loop), so the
   failure path can be exercised without a real stall; -1 disables it. */
gsn_status gsn_batch_set_queue_limits(gsn_batch batch, unsigned spin_limit, long long fail_item);
/* Variant per pass family {kinetic, density, kernel, phase, x entry/exit}
   (nfam >= 5): 0 "e16" / 1 "e8" (one tile per block), 2 "p16" / 3 "p8"
   (persistent blocks walking the tiles of every instance of a shape group,
   prefetching the next tile; used for a group only when all its instances
   share box lengths, a and dz, else that group runs variant - 2; x entry/exit
   always one tile per block), and the nonlinear mode (as
   gsn_set_nonlinear_mode). */
gsn_status gsn_batch_set_schedule(gsn_batch batch, const int *variants, int nfam, int nonlinear_mode);
/* Autotuner of the batched launch (the best FFT tile and radix schedule
   depends on the mesh size, Sec. III): for every shape group, times each
   variant of each pass family with the other families fixed -- the column
   passes first, then the density and phase passes under both nonlinear modes,
   then the x entry/exit pair -- over iters (1..10000) whole split steps of
   that group alone, and keeps the fastest per group.  The timed passes run in
   place on the instances' own buffers, so every instance must be set
   (GSN_ESTATE otherwise); their psi and global phase are saved to host memory
   first and restored afterwards, so the states are unchanged.  With the
   environment variable GSN_AUTOTUNE_CACHE naming a file, choices are read
   from it (keyed by GPU architecture, shape and family) and new ones
   appended.  Synchronising. */
gsn_status gsn_batch_autotune(gsn_batch batch, int iters);
/* The schedule of instance i's shape group: variants[5] per family as in
   gsn_batch_set_schedule (nfam >= 5) and its nonlinear mode. */
gsn_status gsn_batch_get_schedule(gsn_batch batch, int i, int *variants, int nfam, int *nonlinear_mode);

/* ---------------------------------------------------------------- learned corrector
   A 4-layer 3x3 convolutional network with circular padding (3 -> 32 -> 32 ->
   32 -> 2 channels, ReLU after the first three; 19970 parameters) that maps
   (Re psi_c, Im psi_c, phi_c) of a coarse split step (ratio * dz) to the
   residual psi_fine - psi_c of the equivalent ratio fine steps.  bfloat16
   weights and activations, FP32 accumulation on the matrix cores, FP32
   master weights and Adam moments.  This is not part of the paper's method:
   the plain fine-step solver stays the reference for its error and its fallback.
   Flat FP32 parameter vector, per layer: w[tap][cout][cin] (tap = 3 dy + dx,
   input offset (dy-1, dx-1)) then bias[cout].  Images are H x W with H*W a
   multiple of 64; device buffers are psi complex64 H*W and phi float H*W. */
typedef struct gsn_corrector_ *gsn_corrector;
gsn_status gsn_corrector_workspace_bytes(int H, int W, int max_batch, size_t *bytes);
gsn_status gsn_corrector_create(gsn_corrector *out, int H, int W, int max_batch, void *d_workspace,
                                size_t bytes, void *hip_stream);
gsn_status gsn_corrector_destroy(gsn_corrector c);
/* Load FP32 master weights (n == 19970, host) and reset the Adam state. */
gsn_status gsn_corrector_set_weights(gsn_corrector c, const float *w, size_t n);
gsn_status gsn_corrector_get_weights(gsn_corrector c, float *w, size_t n);
/* Input feature scales (Re, Im, phi) and the residual scale s_out: the net
   sees scaled inputs and predicts residual / s_out. */
gsn_status gsn_corrector_set_scales(gsn_corrector c, const float in_scale[3], float out_scale);
/* Pack image slot b from device psi (complex64) and phi (float). */
gsn_status gsn_corrector_pack(gsn_corrector c, int b, const void *psi, const float *phi);
/* Training target of slot b: (psi_fine - psi_coarse) / s_out (device buffers). */
gsn_status gsn_corrector_pack_target(gsn_corrector c, int b, const void *psi_fine, const void *psi_coarse);
/* Forward pass over slots 0..B-1; optional copy of the output (B*H*W*2 FP32). */
gsn_status gsn_corrector_forward(gsn_corrector c, int B, float *out_dev);
/* Forward + MSE + backward over slots 0..B-1 without updating: gradient of
   the loss w.r.t. the flat parameters to grad_host (19970 floats) and the
   loss.  Synchronising. */
gsn_status gsn_corrector_gradients(gsn_corrector c, int B, float *grad_host, float *loss);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on slots 0..B-1. */
gsn_status gsn_corrector_train_step(gsn_corrector c, int B, float lr, float *loss);
/* psi_out = psi_c + s_out * (r0 + i r1) with the last forward output of slot b. */
gsn_status gsn_corrector_apply(gsn_corrector c, int b, const void *psi_c, void *psi_out);

/* Coarse steps: coarse_ratio * dz per step, same schedule (0 disables). */
gsn_status gsn_set_coarse_ratio(gsn_grid grid, int ratio);
gsn_status gsn_step_coarse(gsn_grid grid, int64_t nsteps);
/* phi of the current psi (without its uniform k = 0 part) into a device
   float buffer of P values.  Asynchronous. */
gsn_status gsn_potential(gsn_grid grid, float *phi_dev);
/* ncoarse corrected coarse steps on a 2-D grid: coarse step, potential, net,
   psi += s_out * residual.  Every audit_every-th step (0 = never) the same
   step is redone with coarse_ratio fine steps; if the relative L2 distance
   between the corrected and fine states exceeds tol the fine state is kept
   (a fallback).  Reports the fallbacks and the worst audited error.
   Synchronising when audits run. */
gsn_status gsn_step_corrected(gsn_grid grid, gsn_corrector c, int64_t ncoarse, int audit_every, double tol,
                              int64_t *n_fallbacks, double *max_audit_err);

/* Human-readable message for the last failure on this thread. */
const char *gsn_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GSN_H */
