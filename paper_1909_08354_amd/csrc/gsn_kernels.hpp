// gsn_kernels.hpp -- the HBM passes of one split step on gfx950.
//
// State between passes is complex64 in HBM.  Each pass loads a tile of lines,
// runs FFTs in FP64 registers (Stockham, LDS exchange as complex64), applies a
// fused pointwise stage and stores the tile back.  Two tile shapes:
//   * EM ("element-major", the contiguous x axis): a block owns whole rows;
//     consecutive lanes hold consecutive points of a row.
//   * LM ("line-major", strided y / z axes): a block owns LINES adjacent
//     columns along x of one slice; consecutive lanes hold adjacent columns, so
//     every load and store is a contiguous LINES*8-byte segment.
//
// Normalisation (F = unnormalised forward DFT, G = unnormalised inverse):
//   psi_x = F_x psi is the state inside a run of steps;
//   kinetic sub-step:  psi_x <- G_y G_z [M / (Ny Nz)] F_z F_y psi_x  (3-D)
//                      psi_x <- G_y [M / Ny] F_y psi_x                (2-D)
//   density:           rho_x = F_x |G_x psi_x / Nx|^2   (half spectrum)
//   potential:         phi_x = G_y G_z [K / (Ny Nz)] F_z F_y rho_x
//   phase:             psi_x <- F_x[ (G_x psi_x / Nx) exp(i (g rho + G_x phi_x / Nx) dz) ]
// Powers of two make every scale exact.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <utility>

#include "gsn_fft.hpp"

namespace gsn {

struct DevState {
    double theta;      // accumulated global phase K(0) <rho> dz (FP64)
    double mass_sum;   // sum |psi|^2 of the last nonlinear sub-step (no dV)
    long long steps;   // nonlinear sub-steps taken since set_psi
    int nonfinite;     // set when a fused mass was NaN/Inf
    int pad;
};

// ---------------------------------------------------------------- EM passes
struct EmArgs {
    float2 *psi;          // rows of N complex
    float2 *half;         // rows of N/2 complex (half spectrum, bins 0..N/2-1)
    float2 *nyq;          // one complex per row (bin N/2)
    const double2 *tw;    // exp(-2 pi i q / N), q < N
    int nlines;           // rows (plain FFT) or row pairs (density / phase)
    double scale;         // plain FFT output scale
    double g, dz;         // phase stage
    double *partials;     // per-block FP64 partials
    float *phi;           // potential readout destination (real rows of N)
    const double2 *sct;   // (cos, sin) of j pi/128, j < 256 (pipelined phase pass)
    // local terms of Eq. (15) (the general density and phase passes):
    // U = g rho + cp f(max(rho, rfl)) + cb2 lap(s) / max(s, sfl), s = sqrt(rho),
    // f = ln rho (pmode 1) or pfac rho^pn1 (pmode 2, pfac = n/(n-1), pn1 = n-1)
    float2 *half2;        // half spectrum of s, then lap(s) (Bohm term)
    float2 *nyq2;
    double cp, pfac, pn1, cb2, rfl, sfl;
    double f_fl, F_fl;    // f and its antiderivative F at the floor (pressure energy)
    int pmode;            // 0: no pressure term, 1: ln rho, 2: power law
    int bohm;             // 1: Bohm term
    // position-dependent coupling (Eq. (9)-(12)): the kernel acts on
    // s = gam rho + bet lap(rho); vext joins the phase (real fields of P
    // values, C order; null: gam = 1, bet = 0, vext = 0)
    const float *gam, *bet, *vext;
};

template <int N, int E> struct EmShape {
    static constexpr int TPL = N / E;
};

template <int N, int E, int LINES> struct EmTile {
    static constexpr int TPL = N / E;
    static constexpr int NT = LINES * TPL;
    static constexpr int LDS = LINES * EmLayout<N, E>::PITCH;   // float2 slots
};
template <int N, int E, int LINES> struct LmTile {
    static constexpr int TPL = N / E;
    static constexpr int NT = LINES * TPL;
    static constexpr int LDS = LINES * N;
};

// Complex values in HBM: complex64 (float2, the default everywhere) or
// complex128 (double2, the FP64-storage grids).  The argument structs carry
// complex64 pointers; an FP64-storage kernel reinterprets them as double2
// arrays (the host sets them to double2 buffers), and its LDS slots are
// double2 too, so no value is rounded below FP64 anywhere in the step.
__device__ __forceinline__ dc ld_c(const float2 &v) { return from_f2(v); }
__device__ __forceinline__ dc ld_c(const double2 &v) { return from_d2(v); }
template <class ST> __device__ __forceinline__ ST st_c(dc v);
template <> __device__ __forceinline__ float2 st_c<float2>(dc v) { return to_f2(v); }
template <> __device__ __forceinline__ double2 st_c<double2>(dc v) { return make_double2(v.x, v.y); }
// real values kept between stages of one pass (phi rows): float or double
template <class ST> struct RealOf { using T = float; };
template <> struct RealOf<double2> { using T = double; };
// The E points q[(t + TPL e) es] of one line, every load issued before any
// is used: a line past the grid's last (act false) reads the line at `safe`
// instead of branching around its loads, and is zeroed.  A branch per load
// would make the thread wait for each load in turn.
template <int E, int TPL, class ST>
__device__ __forceinline__ void load_line(const ST *q, const ST *safe, long long es, bool act, int t, dc (&v)[E])
{
    const ST *src = act ? q : safe;
    ST raw[E];
#pragma unroll
    for (int e = 0; e < E; ++e) raw[e] = src[(long long)(t + TPL * e) * es];
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = act ? ld_c(raw[e]) : mk(0.0, 0.0);
}

// Plain row FFT (entry/exit of a run of steps, energy evaluation).
template <int N, int E, int LINES, int S, class ST>
__device__ __forceinline__ void em_fft_tile(const EmArgs &a, int tile, ST *lds)
{
    constexpr int TPL = N / E;
    const int tid = threadIdx.x, t = tid % TPL, l = tid / TPL;
    const int row = tile * LINES + l;
    const bool act = row < a.nlines;
    const EmLayout<N, E> lay{l * EmLayout<N, E>::PITCH};
    dc v[E];
    ST *p = (ST *)a.psi + (long long)row * N;
    load_line<E, TPL>(p, (const ST *)a.psi, 1, act, t, v);
    fft<N, E, S>(v, t, lay, lds, a.tw);
    if (act) {
#pragma unroll
        for (int e = 0; e < E; ++e) p[t + TPL * e] = st_c<ST>(scl(v[e], a.scale));
    }
}

// Density pass: psi = G_x psi_x / N for two rows, rho = |psi|^2, FP64 partial
// of sum rho, then one forward FFT of Z = rho_0 + i rho_1 and the split
// X_0[k] = (Z[k] + conj Z[N-k]) / 2, X_1[k] = (Z[k] - conj Z[N-k]) / (2i).
//
// STORE_PSI: also write psi (real space) back over the two psi_x rows, so the
// phase pass can skip its two inverse x transforms (+8 bytes per point).
//
// REAL_IN: the rows hold psi in real space (not x-spectral); the inverse x
// transforms are skipped (the potential readout of a state between calls).
// Split the spectrum Z = X_0 + i X_1 of two real rows held in v (one exchange
// through LDS, so bin k can see bin N-k) into X_0[k] = (Z[k] + conj Z[N-k]) / 2,
// X_1[k] = (Z[k] - conj Z[N-k]) / (2i); store bins 0..N/2-1 to the half rows
// r0, r1 and the real bin N/2 to nyq.
template <int N, int E, class LT, class ST>
__device__ __forceinline__ void store_real_pair(const dc (&v)[E], bool act, int t, const EmLayout<N, E> &lay,
                                                LT *lds, ST *half, ST *nyq, long long r0, long long r1)
{
    constexpr int TPL = N / E;
#pragma unroll
    for (int e = 0; e < E; ++e) lds_put(lds, lay(t + TPL * e), v[e]);
    exchange_sync<EmLayout<N, E>::WAVE_LOCAL>();
    if (act) {
        ST *h0 = half + r0 * (N / 2), *h1 = half + r1 * (N / 2);
#pragma unroll
        for (int e = 0; e < E / 2; ++e) {
            const int k = t + TPL * e;
            const dc z = v[e];
            const dc zc = conj(lds_get(lds, lay((N - k) & (N - 1))));
            const dc s = add(z, zc), d = sub(z, zc);
            h0[k] = st_c<ST>(scl(s, 0.5));
            h1[k] = st_c<ST>(mk(0.5 * d.y, -0.5 * d.x));
        }
        if (t == 0) {
            const dc z = v[E / 2];   // bin N/2: both halves are real
            nyq[r0] = st_c<ST>(mk(z.x, 0.0));
            nyq[r1] = st_c<ST>(mk(z.y, 0.0));
        }
    }
}

// BOHM: also transform s = sqrt(rho) of both rows the same way into half2 /
// nyq2 (the Bohm potential of Eq. (15) needs lap(s)).
template <int N, int E, int LINES, bool STORE_PSI, bool REAL_IN = false, bool BOHM = false, class ST>
__device__ __forceinline__ void density_tile(const EmArgs &a, int tile, ST *lds, double *sh)
{
    static_assert(!(STORE_PSI && REAL_IN), "real-space input is not stored back");
    constexpr int TPL = N / E, NT = LINES * TPL;
    const int tid = threadIdx.x, t = tid % TPL, l = tid / TPL;
    const int pair = tile * LINES + l;
    const bool act = pair < a.nlines;
    const EmLayout<N, E> lay{l * EmLayout<N, E>::PITCH};
    const long long r0 = 2LL * pair, r1 = r0 + 1;
    const double inv_n = 1.0 / N;
    const double rs = REAL_IN ? 1.0 : inv_n * inv_n;   // |psi|^2 scale
    dc v[E];
    double rho0[E];
    ST *p0 = (ST *)a.psi + r0 * N, *p1 = (ST *)a.psi + r1 * N;
    load_line<E, TPL>(p0, (const ST *)a.psi, 1, act, t, v);
    if constexpr (!REAL_IN) fft<N, E, 1>(v, t, lay, lds, a.tw);
#pragma unroll
    for (int e = 0; e < E; ++e) rho0[e] = norm2(v[e]) * rs;
    if constexpr (STORE_PSI) {
        if (act) {
#pragma unroll
            for (int e = 0; e < E; ++e) p0[t + TPL * e] = st_c<ST>(scl(v[e], inv_n));
        }
    }
    load_line<E, TPL>(p1, (const ST *)a.psi, 1, act, t, v);
    if constexpr (!REAL_IN) fft<N, E, 1>(v, t, lay, lds, a.tw);
    if constexpr (STORE_PSI) {
        if (act) {
#pragma unroll
            for (int e = 0; e < E; ++e) p1[t + TPL * e] = st_c<ST>(scl(v[e], inv_n));
        }
    }
    double msum = 0.0;
    dc w[BOHM ? E : 1];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const double rho1 = norm2(v[e]) * rs;
        msum += rho0[e] + rho1;
        if constexpr (BOHM) w[e] = mk(sqrt(rho0[e]), sqrt(rho1));
        v[e] = mk(rho0[e], rho1);
    }
    fft<N, E, -1>(v, t, lay, lds, a.tw);
    store_real_pair<N, E>(v, act, t, lay, lds, (ST *)a.half, (ST *)a.nyq, r0, r1);
    if constexpr (BOHM) {
        exchange_sync<EmLayout<N, E>::WAVE_LOCAL>();   // the split above has read LDS
        fft<N, E, -1>(w, t, lay, lds, a.tw);
        store_real_pair<N, E>(w, act, t, lay, lds, (ST *)a.half2, (ST *)a.nyq2, r0, r1);
    }
    const double bs = block_sum<NT>(msum, sh);
    if (tid == 0) a.partials[tile] = bs;
}

// Full x-spectrum Z = X_0 + i X_1 of two real rows r0, r1 from their half
// spectra (X[N-k] = conj X[k]; the DC and Nyquist bins are real).
template <int N, int E, class ST>
__device__ __forceinline__ void load_real_pair(const ST *half, const ST *nyq, bool act, int t, long long r0,
                                               long long r1, dc (&z)[E])
{
    constexpr int TPL = N / E;
    // every load issued before any is used (rows past the grid's last read
    // pair 0 and are zeroed; the lane that takes the Nyquist bin reads bin 0
    // there); a branch per bin would make the thread wait for each in turn
    if (!act) {
        r0 = 0;
        r1 = 1;
    }
    const ST *h0 = half + r0 * (N / 2), *h1 = half + r1 * (N / 2);
    ST a0[E], a1[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = t + TPL * e;
        const int idx = e < E / 2 ? k : (N - k) & (N / 2 - 1);
        a0[e] = h0[idx];
        a1[e] = h1[idx];
    }
    const ST n0 = nyq[r0], n1 = nyq[r1];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        dc x0, x1;
        if (e < E / 2) {
            x0 = ld_c(a0[e]);
            x1 = ld_c(a1[e]);
            if (t + TPL * e == 0) { x0.y = 0.0; x1.y = 0.0; }
        } else if (e == E / 2 && t == 0) {
            x0 = mk((double)n0.x, 0.0);
            x1 = mk((double)n1.x, 0.0);
        } else {
            x0 = conj(ld_c(a0[e]));
            x1 = conj(ld_c(a1[e]));
        }
        if (!act) x0 = x1 = mk(0.0, 0.0);
        z[e] = mk(x0.x - x1.y, x0.y + x1.x);
    }
}

template <int N, int E, class ST = float2>
__device__ __forceinline__ void load_phi_pair(const EmArgs &a, bool act, int t, long long r0, long long r1,
                                              dc (&z)[E])
{
    load_real_pair<N, E>((const ST *)a.half, (const ST *)a.nyq, act, t, r0, r1, z);
}

// Potential readout: phi rows (without the uniform k = 0 part) as float.
template <int N, int E, int LINES>
__device__ __forceinline__ void potential_tile(const EmArgs &a, int tile, float2 *lds)
{
    constexpr int TPL = N / E;
    const int tid = threadIdx.x, t = tid % TPL, l = tid / TPL;
    const int pair = tile * LINES + l;
    const bool act = pair < a.nlines;
    const EmLayout<N, E> lay{l * EmLayout<N, E>::PITCH};
    const long long r0 = 2LL * pair, r1 = r0 + 1;
    dc z[E];
    load_phi_pair<N, E>(a, act, t, r0, r1, z);
    fft<N, E, 1>(z, t, lay, lds, a.tw);
    if (act) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            a.phi[r0 * N + t + TPL * e] = (float)(z[e].x / N);
            a.phi[r1 * N + t + TPL * e] = (float)(z[e].y / N);
        }
    }
}

// Phase pass.  Rebuild the full x-spectrum of two phi rows from their half
// spectra (X[N-k] = conj X[k]; DC and Nyquist real), one inverse FFT gives
// phi_0 + i phi_1.  Then per row: psi = G_x psi_x / N, multiply by
// exp(i (g |psi|^2 + phi) dz) in FP64, F_x, store.  ENERGY: instead of the
// phase, accumulate sum rho*phi and sum rho^2 and store nothing.
// sin and cos in FP64: reduce th = k (pi/2) + r with |r| <= pi/4 (pi/2 split in
// three parts, Cody-Waite), then the Taylor series of sin (to r^17) and cos (to
// r^18), whose truncation error is below 1e-19 on |r| <= pi/4.  The reduction
// is exact while |k| < 2^20 (|th| < 1.6e6); beyond that the absolute error
// grows like |th| * 1e-16, which only matters for phases no step should reach.
__host__ __device__ __forceinline__ void sincos_fp64(double th, double *s, double *c)
{
    constexpr double kTwoOverPi = 0.63661977236758134308;
    // pi/2 = kP1 + kP2 + kP3 (+ 1e-37): kP1 and kP2 carry 33 significant bits
    // each, so kf * kP1 and kf * kP2 are exact for |kf| < 2^20
    constexpr double kP1 = 1.5707963267341256e+00;
    constexpr double kP2 = 6.077100506303966e-11;
    constexpr double kP3 = 2.0222662487959506e-21;
    const double kf = rint(th * kTwoOverPi);
    double r = fma(-kf, kP1, th);
    r = fma(-kf, kP2, r);
    r = fma(-kf, kP3, r);
    const double r2 = r * r;
    // sin r = r (1 - r^2/3! + r^4/5! - ... - r^16/17!)
    double ps = -1.0 / 355687428096000.0;                 // -1/17!
    ps = fma(ps, r2, 1.0 / 1307674368000.0);               //  1/15!
    ps = fma(ps, r2, -1.0 / 6227020800.0);                 // -1/13!
    ps = fma(ps, r2, 1.0 / 39916800.0);                    //  1/11!
    ps = fma(ps, r2, -1.0 / 362880.0);                     // -1/9!
    ps = fma(ps, r2, 1.0 / 5040.0);                        //  1/7!
    ps = fma(ps, r2, -1.0 / 120.0);
    ps = fma(ps, r2, 1.0 / 6.0);
    const double sr = fma(-r * r2, ps, r);
    // cos r = 1 - r^2/2! + r^4/4! - ... + r^18/18!
    double pc = 1.0 / 6402373705728000.0;                  //  1/18!
    pc = fma(pc, r2, -1.0 / 20922789888000.0);             // -1/16!
    pc = fma(pc, r2, 1.0 / 87178291200.0);                 //  1/14!
    pc = fma(pc, r2, -1.0 / 479001600.0);                  // -1/12!
    pc = fma(pc, r2, 1.0 / 3628800.0);                     //  1/10!
    pc = fma(pc, r2, -1.0 / 40320.0);                      // -1/8!
    pc = fma(pc, r2, 1.0 / 720.0);                         //  1/6!
    pc = fma(pc, r2, -1.0 / 24.0);                         // -1/4!
    pc = fma(pc, r2, 0.5);                                 //  1/2!
    const double cr = fma(-r2, pc, 1.0);
    const int q = (int)(kf - 4.0 * floor(kf * 0.25));   // k mod 4 in [0, 4)
    const double ss = (q & 1) ? cr : sr, cc = (q & 1) ? sr : cr;
    *s = (q & 2) ? -ss : ss;
    *c = ((q + 1) & 2) ? -cc : cc;
}

// sin and cos in FP64 from a table: th = j pi/128 + r with |r| <= pi/256 (the
// three parts of pi/2 above scaled by 1/64; each step is one FMA, whose exact
// product keeps the reduced argument accurate to its own rounding while j fits
// the table index, |th| < 5e7); tab[j mod 256] = (cos, sin)(j pi/128), and
// sin r, cos r from their Taylor series to r^5 and r^6 (truncation below 1e-17
// on |r| <= pi/256), combined by the angle-addition formulas.
constexpr int kSinCosTable = 256;

__host__ __device__ __forceinline__ void sincos_tab(double th, const double2 *tab, double *s, double *c)
{
    constexpr double k128OverPi = 40.743665431525205957;
    constexpr double kQ1 = 1.5707963267341256e+00 / 64.0;
    constexpr double kQ2 = 6.077100506303966e-11 / 64.0;
    constexpr double kQ3 = 2.0222662487959506e-21 / 64.0;
    const double jf = rint(th * k128OverPi);
    double r = fma(-jf, kQ1, th);
    r = fma(-jf, kQ2, r);
    r = fma(-jf, kQ3, r);
    const double2 cs = tab[(int)jf & (kSinCosTable - 1)];
    const double r2 = r * r;
    const double sr = fma(r * r2, fma(r2, 1.0 / 120.0, -1.0 / 6.0), r);
    const double cr = fma(r2, fma(r2, fma(r2, -1.0 / 720.0, 1.0 / 24.0), -0.5), 1.0);
    *s = fma(cs.y, cr, cs.x * sr);
    *c = fma(cs.x, cr, -(cs.y * sr));
}

// Natural logarithm in FP64 for finite x > 0: x = m 2^e with m in
// [sqrt(1/2), sqrt(2)), f = m - 1, u = f / (2 + f) (|u| <= 0.1716) and
// ln m = 2 atanh(u) = 2 (u + u^3/3 + ... + u^21/21) (the remainder is below
// 2e-18 relative), plus e ln 2 with ln 2 split into a 32-bit head (so e times
// it is exact) and its tail.
__host__ __device__ __forceinline__ double log_fp64(double x)
{
    constexpr double kLn2Hi = 0.6931471806019545;
    constexpr double kLn2Lo = -4.2009150726810846e-11;
    int e;
    double m = frexp(x, &e);   // m in [1/2, 1)
    if (m < 0.70710678118654752) {
        m *= 2.0;
        e -= 1;
    }
    const double f = m - 1.0;
    const double u = f / (2.0 + f);
    const double z = u * u;
    double p = 1.0 / 21.0;
    p = fma(p, z, 1.0 / 19.0);
    p = fma(p, z, 1.0 / 17.0);
    p = fma(p, z, 1.0 / 15.0);
    p = fma(p, z, 1.0 / 13.0);
    p = fma(p, z, 1.0 / 11.0);
    p = fma(p, z, 1.0 / 9.0);
    p = fma(p, z, 1.0 / 7.0);
    p = fma(p, z, 1.0 / 5.0);
    p = fma(p, z, 1.0 / 3.0);
    const double lm = fma(2.0 * u * z, p, 2.0 * u);
    const double ed = (double)e;
    return fma(ed, kLn2Hi, fma(ed, kLn2Lo, lm));
}

// e^y in FP64: y = k ln 2 + r with |r| <= ln(2)/2 (the same two-part ln 2),
// e^r from its Taylor series to r^14 (remainder below 5e-18 relative), scaled
// by 2^k.  Arguments are clamped to [-746, 709.7]: 0 below, finite above.
__host__ __device__ __forceinline__ double exp_fp64(double y)
{
    constexpr double kLog2E = 1.4426950408889634;
    constexpr double kLn2Hi = 0.6931471806019545;
    constexpr double kLn2Lo = -4.2009150726810846e-11;
    y = fmin(fmax(y, -746.0), 709.7);
    const double k = rint(y * kLog2E);
    double r = fma(-k, kLn2Hi, y);
    r = fma(-k, kLn2Lo, r);
    // sum r^j / j!, j = 0..14, by Horner
    double p = 1.0 / 87178291200.0;         // 1/14!
    p = fma(p, r, 1.0 / 6227020800.0);      // 1/13!
    p = fma(p, r, 1.0 / 479001600.0);       // 1/12!
    p = fma(p, r, 1.0 / 39916800.0);        // 1/11!
    p = fma(p, r, 1.0 / 3628800.0);         // 1/10!
    p = fma(p, r, 1.0 / 362880.0);          // 1/9!
    p = fma(p, r, 1.0 / 40320.0);           // 1/8!
    p = fma(p, r, 1.0 / 5040.0);            // 1/7!
    p = fma(p, r, 1.0 / 720.0);             // 1/6!
    p = fma(p, r, 1.0 / 120.0);             // 1/5!
    p = fma(p, r, 1.0 / 24.0);              // 1/4!
    p = fma(p, r, 1.0 / 6.0);               // 1/3!
    p = fma(p, r, 0.5);                     // 1/2!
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    return ldexp(p, (int)k);
}

// Fields of the pure non-minimal coupling, Eq. (9)-(11), at distance r from
// the centre: u = (r0/(r + r0))^lambda, gamma = (1 - u)/2, beta = lambda u/(r + r0),
// V = -ln(1 - u_c)/nu with u_c at max(r, r_min) (phi_C diverges at r = 0).
__host__ __device__ __forceinline__ void nmc_point(double r, double lambda, double r0, double nu, double r_min,
                                                   double *gamma, double *beta, double *V)
{
    const double u = exp_fp64(lambda * log_fp64(r0 / (r + r0)));
    *gamma = 0.5 * (1.0 - u);
    *beta = lambda * u / (r + r0);
    const double rc = fmax(r, r_min);
    const double uc = exp_fp64(lambda * log_fp64(r0 / (rc + r0)));
    *V = -log_fp64(1.0 - uc) / nu;
}

// The table sincos_tab reads, computed in extended precision and rounded.
inline void fill_sincos_table(double2 *tab)
{
    for (int j = 0; j < kSinCosTable; ++j) {
        const long double ang = (long double)j * 3.14159265358979323846264338327950288L / 128.0L;
        tab[j] = make_double2((double)cosl(ang), (double)sinl(ang));
    }
}

//
// REAL_IN: the psi rows already hold psi in real space (written by the density
// pass with STORE_PSI), so the inverse x transform is skipped.
template <int N, int E, int LINES, bool ENERGY, bool REAL_IN, class ST>
__device__ __forceinline__ void phase_tile(const EmArgs &a, int tile, ST *lds, double *sh)
{
    constexpr int TPL = N / E, NT = LINES * TPL;
    using RT = typename RealOf<ST>::T;
    const int tid = threadIdx.x, t = tid % TPL, l = tid / TPL;
    const int pair = tile * LINES + l;
    const bool act = pair < a.nlines;
    const EmLayout<N, E> lay{l * EmLayout<N, E>::PITCH};
    const long long r0 = 2LL * pair, r1 = r0 + 1;
    const double inv_n = 1.0 / N;
    dc z[E];
    load_phi_pair<N, E, ST>(a, act, t, r0, r1, z);
    fft<N, E, 1>(z, t, lay, lds, a.tw);
    // phi of both rows, kept in the storage precision (float for complex64)
    RT phi0[E], phi1[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        phi0[e] = (RT)(z[e].x * inv_n);
        phi1[e] = (RT)(z[e].y * inv_n);
    }
    double acc0 = 0.0, acc1 = 0.0;
#pragma unroll 1
    for (int half = 0; half < 2; ++half) {
        ST *p = (ST *)a.psi + (half ? r1 : r0) * N;
        dc v[E];
        load_line<E, TPL>(p, (const ST *)a.psi, 1, act, t, v);
        if constexpr (!REAL_IN) fft<N, E, 1>(v, t, lay, lds, a.tw);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const dc ps = REAL_IN ? v[e] : scl(v[e], inv_n);
            const double rho = norm2(ps);
            const double phi = (double)(half ? phi1[e] : phi0[e]);
            if constexpr (ENERGY) {
                acc0 += rho * phi;
                acc1 += rho * rho;
            } else {
                double s, c;
                sincos_fp64(fma(a.g, rho, phi) * a.dz, &s, &c);
                v[e] = cmul(ps, mk(c, s));
            }
        }
        if constexpr (!ENERGY) {
            fft<N, E, -1>(v, t, lay, lds, a.tw);
            if (act) {
#pragma unroll
                for (int e = 0; e < E; ++e) p[t + TPL * e] = st_c<ST>(v[e]);
            }
        }
    }
    if constexpr (ENERGY) {
        const double b0 = block_sum<NT>(acc0, sh);
        const double b1 = block_sum<NT>(acc1, sh);
        if (tid == 0) {
            a.partials[4 * tile] = b0;
            a.partials[4 * tile + 1] = b1;
            a.partials[4 * tile + 2] = 0.0;
            a.partials[4 * tile + 3] = 0.0;
        }
    }
}

// 1/sqrt(x) in FP64 for x > 0: the hardware estimate refined by two Newton
// steps y <- y + y (1 - x y^2) / 2.
__device__ __forceinline__ double rsqrt_fp64(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
    y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
    return y;
}

// Local terms of Eq. (15) for the E points of one row: U = g rho + pressure +
// Bohm (see EmArgs); pmode and bohm are uniform, so each term is one branch
// around its loop.  1 / max(sqrt rho, sqrt floor) = 1 / sqrt(max(rho, floor)).
// The power law's floor is at least 1e-300 so that its logarithm is finite.
template <int E>
__device__ __forceinline__ void local_potential(const EmArgs &a, const double (&rho)[E], const float (&lap)[E],
                                                double (&U)[E])
{
#pragma unroll
    for (int e = 0; e < E; ++e) U[e] = a.g * rho[e];
    if (a.pmode == 1) {
#pragma unroll
        for (int e = 0; e < E; ++e) U[e] = fma(a.cp, log_fp64(fmax(rho[e], a.rfl)), U[e]);
    } else if (a.pmode == 2) {
        const double fl = fmax(a.rfl, 1e-300), cpf = a.cp * a.pfac;
#pragma unroll
        for (int e = 0; e < E; ++e) U[e] = fma(cpf, exp_fp64(a.pn1 * log_fp64(fmax(rho[e], fl))), U[e]);
    }
    if (a.bohm) {
#pragma unroll
        for (int e = 0; e < E; ++e) U[e] = fma(a.cb2 * (double)lap[e], rsqrt_fp64(fmax(rho[e], a.rfl)), U[e]);
    }
}

// Antiderivative G of the floored pressure potential f(max(rho, floor)):
// F(rho) above the floor (F = rho ln rho - rho, or rho^n / (n-1)), and
// F(floor) + (rho - floor) f(floor) below it.
__device__ __forceinline__ double pressure_energy_density(const EmArgs &a, double rho)
{
    if (rho < a.rfl || rho <= 0.0) return fma(rho - a.rfl, a.f_fl, a.F_fl);
    const double lr = log_fp64(rho);
    return a.pmode == 1 ? rho * (lr - 1.0) : a.pfac / (a.pn1 + 1.0) * rho * exp_fp64(a.pn1 * lr);
}

// (fft() ends with a barrier after its last LDS read, so transforms follow
// each other without one; a split that reads LDS needs one before the next.)
//
// Phase pass with the local terms of Eq. (15): as phase_tile, plus (a.bohm)
// lap(s) of both rows from the half2 spectrum, and the local potential U of
// local_potential in place of g rho.  ENERGY: per tile the sums of rho phi,
// rho^2, c_p G(rho) + V rho (pressure and static potential) and s lap(s)
// (Bohm).
template <int N, int E, int LINES, bool ENERGY, bool REAL_IN>
__device__ __forceinline__ void phase_local_tile(const EmArgs &a, int tile, float2 *lds, double *sh)
{
    constexpr int TPL = N / E, NT = LINES * TPL;
    const int tid = threadIdx.x, t = tid % TPL, l = tid / TPL;
    const int pair = tile * LINES + l;
    const bool act = pair < a.nlines;
    const EmLayout<N, E> lay{l * EmLayout<N, E>::PITCH};
    const long long r0 = 2LL * pair, r1 = r0 + 1;
    const double inv_n = 1.0 / N;
    dc z[E];
    load_real_pair<N, E>(a.half, a.nyq, act, t, r0, r1, z);
    fft<N, E, 1>(z, t, lay, lds, a.tw);
    float phi0[E], phi1[E], lap0[E], lap1[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        phi0[e] = (float)(z[e].x * inv_n);
        phi1[e] = (float)(z[e].y * inv_n);
        lap0[e] = 0.0f;
        lap1[e] = 0.0f;
    }
    if (a.bohm) {   // uniform over the grid
        load_real_pair<N, E>(a.half2, a.nyq2, act, t, r0, r1, z);
        fft<N, E, 1>(z, t, lay, lds, a.tw);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            lap0[e] = (float)(z[e].x * inv_n);
            lap1[e] = (float)(z[e].y * inv_n);
        }
    }
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
#pragma unroll 1
    for (int half = 0; half < 2; ++half) {
        float2 *p = a.psi + (half ? r1 : r0) * N;
        dc v[E];
        load_line<E, TPL>(p, (const float2 *)a.psi, 1, act, t, v);
        // the static potential of the row, loaded before the transform
        float vx[E];
#pragma unroll
        for (int e = 0; e < E; ++e) vx[e] = 0.0f;
        if (a.vext) {   // uniform pointer
            const float *vr = a.vext + (act ? (half ? r1 : r0) * N + t : 0);
#pragma unroll
            for (int e = 0; e < E; ++e) vx[e] = vr[TPL * e];
        }
        if constexpr (!REAL_IN) fft<N, E, 1>(v, t, lay, lds, a.tw);
        double rho[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if constexpr (!REAL_IN) v[e] = scl(v[e], inv_n);
            rho[e] = norm2(v[e]);
        }
        if constexpr (ENERGY) {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                acc0 += rho[e] * (double)(half ? phi1[e] : phi0[e]);
                acc1 += rho[e] * rho[e];
                if (a.pmode) acc2 = fma(a.cp, pressure_energy_density(a, rho[e]), acc2);
                acc2 = fma((double)vx[e], rho[e], acc2);
                acc3 += sqrt(rho[e]) * (double)(half ? lap1[e] : lap0[e]);
            }
        } else {
            double U[E];
            float lap[E];
#pragma unroll
            for (int e = 0; e < E; ++e) lap[e] = half ? lap1[e] : lap0[e];
            local_potential<E>(a, rho, lap, U);
#pragma unroll
            for (int e = 0; e < E; ++e) U[e] += (double)vx[e];
#pragma unroll
            for (int e = 0; e < E; ++e) {
                double sn, cs;
                sincos_tab((U[e] + (double)(half ? phi1[e] : phi0[e])) * a.dz, a.sct, &sn, &cs);
                v[e] = cmul(v[e], mk(cs, sn));
            }
        }
        if constexpr (!ENERGY) {
            fft<N, E, -1>(v, t, lay, lds, a.tw);
            if (act) {
#pragma unroll
                for (int e = 0; e < E; ++e) p[t + TPL * e] = to_f2(v[e]);
            }
        }
    }
    if constexpr (ENERGY) {
        const double b0 = block_sum<NT>(acc0, sh);
        const double b1 = block_sum<NT>(acc1, sh);
        const double b2 = block_sum<NT>(acc2, sh);
        const double b3 = block_sum<NT>(acc3, sh);
        if (tid == 0) {
            a.partials[4 * tile] = b0;
            a.partials[4 * tile + 1] = b1;
            a.partials[4 * tile + 2] = b2;
            a.partials[4 * tile + 3] = b3;
        }
    }
}

// Source pass of the position-dependent coupling (Eq. (12) with coefficient
// fields): for two rows, s = gam rho + bet lap(rho) with rho = |psi|^2 (psi
// x-spectral, or real-space with REAL_IN) and, with LAP, lap(rho) from the
// rows' half spectra (already carried through the other axes with -|k|^2);
// then the real transform of s replaces those half spectra in place (each
// tile reads its own two rows before writing them).
template <int N, int E, int LINES, bool REAL_IN, bool LAP>
__device__ __forceinline__ void source_tile(const EmArgs &a, int tile, float2 *lds)
{
    constexpr int TPL = N / E;
    const int tid = threadIdx.x, t = tid % TPL, l = tid / TPL;
    const int pair = tile * LINES + l;
    const bool act = pair < a.nlines;
    const EmLayout<N, E> lay{l * EmLayout<N, E>::PITCH};
    const long long r0 = 2LL * pair, r1 = r0 + 1;
    const double inv_n = 1.0 / N;
    const double rs = REAL_IN ? 1.0 : inv_n * inv_n;
    dc z[E];
    float lap0[E], lap1[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        lap0[e] = 0.0f;
        lap1[e] = 0.0f;
    }
    if constexpr (LAP) {
        load_real_pair<N, E>(a.half, a.nyq, act, t, r0, r1, z);
        fft<N, E, 1>(z, t, lay, lds, a.tw);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            lap0[e] = (float)(z[e].x * inv_n);
            lap1[e] = (float)(z[e].y * inv_n);
        }
    }
    double s0[E];
#pragma unroll 1
    for (int h = 0; h < 2; ++h) {
        const long long r = h ? r1 : r0;
        const float2 *p = a.psi + r * N;
        dc v[E];
        load_line<E, TPL>(p, (const float2 *)a.psi, 1, act, t, v);
        // the row's coefficients, loaded before the transform so the loads
        // overlap it (uniform branches on the field pointers)
        float gv[E], bv[E];
        const long long fo = act ? r * N + t : 0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            gv[e] = 1.0f;
            bv[e] = 0.0f;
        }
        if (a.gam) {
#pragma unroll
            for (int e = 0; e < E; ++e) gv[e] = a.gam[fo + TPL * e];
        }
        if (LAP && a.bet) {
#pragma unroll
            for (int e = 0; e < E; ++e) bv[e] = a.bet[fo + TPL * e];
        }
        if constexpr (!REAL_IN) fft<N, E, 1>(v, t, lay, lds, a.tw);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            double sv = (double)gv[e] * (norm2(v[e]) * rs);
            if constexpr (LAP) sv = fma((double)bv[e], (double)(h ? lap1[e] : lap0[e]), sv);
            if (h) z[e] = mk(s0[e], sv);
            else s0[e] = sv;
        }
    }
    fft<N, E, -1>(z, t, lay, lds, a.tw);
    store_real_pair<N, E>(z, act, t, lay, lds, a.half, a.nyq, r0, r1);
}

// ---------------------------------------------------------------- LM passes
// A segment is a set of lines along the pass axis: line lg of outer slice o
// starts at ptr + o*os + lg*ls, its points are es apart.  For the multiplier
// stages the two other wavenumber indices of line (o, lg) are
//   c1 = c1f + lg*c1l + o*c1o,  c2 = c2f + lg*c2l + o*c2o.
struct Seg {
    float2 *ptr;
    long long es, ls, os;
    int nlines, ngroups, ntiles;
    int c1f, c1l, c1o, c2f, c2l, c2o;
};

enum LmMode { LM_FWD = 0, LM_INV = 1, LM_KIN = 2, LM_KERN = 3, LM_KIN_ENERGY = 4, LM_LAP = 5 };

struct LmArgs {
    Seg s0, s1;              // s1 used for tiles >= s0.ntiles (ntiles 0 if absent)
    const double2 *tw;       // twiddles of the pass length
    double scale;            // output scale (FWD / INV) or multiplier scale
    const double2 *kin1, *kin2, *kinp;   // kinetic factor tables exp(-i a k_d^2 h)
    const double *k2_1, *k2_2, *k2_p;    // k_d^2 tables
    double cN, cY, mY2, c0;              // kernel K(k)
    double *partials;                    // per-block FP64 partials (energy)
    // fused end-of-step reduction in block 0 (after the density pass)
    const double *mass_parts;
    int nmass;
    int reduce;
    double k0_dz_over_P;
    DevState *st;
};

template <int N, int E, int LINES, int MODE, class ST>
__device__ __forceinline__ void lm_tile(const LmArgs &a, int tile_in, ST *lds, double *sh)
{
    constexpr int TPL = N / E, NT = LINES * TPL;
    const int tid = threadIdx.x, l = tid % LINES, t = tid / LINES;
    int tile = tile_in;
    const bool second = tile >= a.s0.ntiles;
    const Seg sg = second ? a.s1 : a.s0;
    if (second) tile -= a.s0.ntiles;
    const int o = tile / sg.ngroups, grp = tile - o * sg.ngroups;
    const int lg = grp * LINES + l;
    const bool act = lg < sg.nlines;
    ST *base = (ST *)sg.ptr + (long long)o * sg.os + (long long)lg * sg.ls;
    const LmLayout<LINES> lay{l};
    dc v[E];
    load_line<E, TPL>(base, (const ST *)sg.ptr, sg.es, act, t, v);

    if constexpr (MODE == LM_FWD || MODE == LM_INV) {
        fft<N, E, MODE == LM_FWD ? -1 : 1>(v, t, lay, lds, a.tw);
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = scl(v[e], a.scale);
    } else {
        // inactive lanes (lg >= nlines) read table entry 0, never past the end
        const int c1 = act ? sg.c1f + lg * sg.c1l + o * sg.c1o : 0;
        const int c2 = act ? sg.c2f + lg * sg.c2l + o * sg.c2o : 0;
        fft<N, E, -1>(v, t, lay, lds, a.tw);
        if constexpr (MODE == LM_KIN) {
            const dc m12 = scl(cmul(from_d2(a.kin1[c1]), from_d2(a.kin2[c2])), a.scale);
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] = cmul(v[e], cmul(m12, from_d2(a.kinp[t + TPL * e])));
        } else if constexpr (MODE == LM_KERN) {
            // K = c0 + (cN (k2 + m^2) + cY k2) / (k2 (k2 + m^2)), one reciprocal
            // (hardware estimate refined by two Newton steps to FP64 accuracy)
            const double q12 = a.k2_1[c1] + a.k2_2[c2];
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const double k2 = q12 + a.k2_p[t + TPL * e];
                const double km = k2 + a.mY2;
                const double num = fma(a.cN, km, a.cY * k2);
                const double den = k2 * km;
                double r = __builtin_amdgcn_rcp(den);
                r = fma(r, fma(-den, r, 1.0), r);
                r = fma(r, fma(-den, r, 1.0), r);
                // k = 0: the uniform potential is a global phase, not part of phi
                const double K = k2 > 0.0 ? fma(num, r, a.c0) : 0.0;
                v[e] = scl(v[e], K * a.scale);
            }
        } else if constexpr (MODE == LM_LAP) {
            // the Laplacian: -|k|^2 (Bohm potential)
            const double q12 = a.k2_1[c1] + a.k2_2[c2];
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] = scl(v[e], -(q12 + a.k2_p[t + TPL * e]) * a.scale);
        } else if constexpr (MODE == LM_KIN_ENERGY) {
            const double q12 = a.k2_1[c1] + a.k2_2[c2];
            double acc = 0.0;
            if (act) {
#pragma unroll
                for (int e = 0; e < E; ++e) acc += (q12 + a.k2_p[t + TPL * e]) * norm2(v[e]);
            }
            const double bs = block_sum<NT>(acc, sh);
            if (tid == 0) a.partials[tile_in] = bs;
        }
        if constexpr (MODE != LM_KIN_ENERGY) fft<N, E, 1>(v, t, lay, lds, a.tw);
    }
    if constexpr (MODE != LM_KIN_ENERGY) {
        if (act) {
#pragma unroll
            for (int e = 0; e < E; ++e) base[(long long)(t + TPL * e) * sg.es] = st_c<ST>(v[e]);
        }
    }
    if (a.reduce && tile_in == 0) {
        double s = 0.0;
        for (int i = tid; i < a.nmass; i += NT) s += a.mass_parts[i];
        s = block_sum<NT>(s, sh);
        if (tid == 0) {
            a.st->mass_sum = s;
            a.st->theta += a.k0_dz_over_P * s;
            a.st->steps += 1;
            if (!isfinite(s)) a.st->nonfinite = 1;
        }
    }
}

// ---------------------------------------------------------------- pipelined LM passes
// Persistent blocks walk the tiles tile = blockIdx.x + k gridDim.x.  Before
// the transforms of one tile run, the points of the next tile (and its
// per-line multiplier factors) are already requested into registers, so
// their HBM latency hides behind the arithmetic.  Twiddles and per-position
// tables are copied to LDS once per block: no vector-memory load is issued
// between a prefetch and its use, so waiting for one never waits for another.
// Points move through buffer loads and stores whose per-point offsets are
// scalar (wave-uniform), so addressing costs no vector instructions.  The
// host uses this form only when a tile spans less than 2^31 bytes.
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void *p)
{
    // raw buffer: stride 0, range 2^31 - 1 bytes, gfx9 data-format word
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, 0x7fffffff, 0x00020000);
}
__device__ __forceinline__ float2 buf_ld2(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff)
{
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ __forceinline__ void buf_st2(float2 v, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, 0);
}

// A pointer read from memory (a grouped pass's argument array) is generic;
// generic accesses count on both the vector-memory and the scalar/LDS
// counters, so a wait for them would also wait for every prefetch in flight.
// The arrays live in global memory: say so.
template <class T> __device__ __forceinline__ __attribute__((address_space(1))) T *gmem(T *p)
{
    return (__attribute__((address_space(1))) T *)p;
}
// element i of a global double2 / float2 array (the vector types' operators
// take generic references, so go through the scalar components)
__device__ __forceinline__ double2 gld(const double2 *p, long long i)
{
    const auto q = gmem((const double *)p) + 2 * i;
    return make_double2(q[0], q[1]);
}
__device__ __forceinline__ float2 gld(const float2 *p, long long i)
{
    const auto q = gmem((const float *)p) + 2 * i;
    return make_float2(q[0], q[1]);
}
__device__ __forceinline__ void gst(float2 *p, long long i, float2 v)
{
    const auto q = gmem((float *)p) + 2 * i;
    q[0] = v.x;
    q[1] = v.y;
}

// Where the lanes of a block find tile `tile` of an LM pass.  A lane whose
// line lies past the end of its segment takes the segment's last line: it
// loads, transforms and stores exactly what that line's own lane does (the
// same values to the same addresses), so no load or store is predicated and
// every iteration issues the same vector-memory operations.
struct LmWhere {
    __amdgpu_buffer_rsrc_t r;   // tile base (uniform)
    unsigned voff;              // this lane's line start, bytes
    unsigned step;              // bytes between positions t + TPL e and t + TPL (e + 1)
    int c1, c2;                 // multiplier table indices of this lane's line
};

template <int N, int E, int LINES>
__device__ __forceinline__ LmWhere lm_where(const LmArgs &a, int tile, int l, int t)
{
    constexpr int TPL = N / E;
    const bool second = tile >= a.s0.ntiles;
    const Seg &sg = second ? a.s1 : a.s0;
    if (second) tile -= a.s0.ntiles;
    const int o = tile / sg.ngroups, grp = tile - o * sg.ngroups;
    const int lg0 = grp * LINES;
    const int lg = min(lg0 + l, sg.nlines - 1);
    LmWhere w;
    w.r = buf_rsrc(sg.ptr + (long long)o * sg.os + (long long)lg0 * sg.ls);
    w.voff = (unsigned)(((long long)(lg - lg0) * sg.ls + (long long)t * sg.es) * 8);
    w.step = (unsigned)(sg.es * TPL * 8);
    w.c1 = sg.c1f + lg * sg.c1l + o * sg.c1o;
    w.c2 = sg.c2f + lg * sg.c2l + o * sg.c2o;
    return w;
}

// An empty asm that takes x as input and output: code that computes x stays
// before this point.
__device__ __forceinline__ void pin(dc &x) { asm volatile("" : "+v"(x.x), "+v"(x.y)); }

template <int E, int... I>
__device__ __forceinline__ void convert_pinned(dc (&v)[E], const float2 (&p)[E], std::integer_sequence<int, I...>)
{
    ((v[I] = from_f2(p[I]), pin(v[I])), ...);
}

template <int E> struct LmPrefetch {
    float2 p[E];
    double2 f1, f2;   // kinetic factors kin1[c1], kin2[c2]
    double q1, q2;    // |k|^2 parts k2_1[c1], k2_2[c2]
};

// Issue the loads of one tile.  live = false (no tile left): every lane loads
// the tile base point E times instead, so the count of vector-memory
// operations per iteration stays fixed and costs one cache line.
template <int N, int E, int LINES, int MODE>
__device__ __forceinline__ void lm_fetch(const LmArgs &a, const LmWhere &w, bool live, LmPrefetch<E> &f)
{
    const unsigned vo = live ? w.voff : 0u, st = live ? w.step : 0u;
#pragma unroll
    for (int e = 0; e < E; ++e) f.p[e] = buf_ld2(w.r, vo, e * st);
    if constexpr (MODE == LM_KIN) {
        f.f1 = gld(a.kin1, live ? w.c1 : 0);
        f.f2 = gld(a.kin2, live ? w.c2 : 0);
    } else if constexpr (MODE == LM_KERN) {
        f.q1 = gmem(a.k2_1)[live ? w.c1 : 0];
        f.q2 = gmem(a.k2_2)[live ? w.c2 : 0];
    }
}

// Where the tiles of a pipelined pass come from: one grid (tile t of its
// argument struct) or the instances of a batch group (tile t is tile t mod tpi
// of instance t / tpi; the structs sit in a device array and are read with
// scalar loads, since t is uniform across the block).
template <class A> struct Src1 {
    static constexpr bool GROUPED = false;
    A a;   // by value: the fields then stay scalar values after inlining
    int n;
    __device__ __forceinline__ int ntiles() const { return n; }
    __device__ __forceinline__ int per_instance() const { return n; }
    __device__ __forceinline__ const A &args(int) const { return a; }
    __device__ __forceinline__ int local(int tile) const { return tile; }
};
template <class A> struct SrcG {
    static constexpr bool GROUPED = true;
    const A *__restrict__ arr;
    int tpi, count;
    __device__ __forceinline__ int ntiles() const { return tpi * count; }
    __device__ __forceinline__ int per_instance() const { return tpi; }
    __device__ __forceinline__ const A &args(int tile) const { return arr[tile / tpi]; }
    __device__ __forceinline__ int local(int tile) const { return tile - (tile / tpi) * tpi; }
};

// Tile order for strided tiles narrower than a 128-byte line (LINES x 8 bytes
// < 128): blocks are dispatched round-robin over the 8 XCDs and a persistent
// grid is a multiple of 16, so tiles t and t + 8 run at the same time on two
// blocks of one XCD.  Within each run of 16 tiles of an instance they get
// adjacent line groups: the line the two tiles share is then fetched into
// that XCD's L2 once, not into two L2s (every tile still runs once; the order
// only pairs them up).
template <class Src> struct SrcPaired {
    static constexpr bool GROUPED = Src::GROUPED;
    Src s;
    __device__ __forceinline__ int ntiles() const { return s.ntiles(); }
    __device__ __forceinline__ int per_instance() const { return s.per_instance(); }
    __device__ __forceinline__ const auto &args(int t) const { return s.args(t); }
    __device__ __forceinline__ int local(int t) const
    {
        const int l = s.local(t), base = l & ~15;
        return base + 16 > s.per_instance() ? l : base + 2 * (l & 7) + ((l >> 3) & 1);
    }
};
template <int LINES, class Src> __device__ __forceinline__ auto lm_order(const Src &s)
{
    if constexpr (LINES * 8 < 128) return SrcPaired<Src>{s};
    else return s;
}

// FP64 sum of the density pass's mass partials, folded into the state
// (global phase, step count, non-finite flag); every thread of the block calls it.
template <int NT>
__device__ __forceinline__ void reduce_mass(const LmArgs &a, double *sh)
{
    double s = 0.0;
    for (int i = threadIdx.x; i < a.nmass; i += NT) s += gmem(a.mass_parts)[i];
    s = block_sum<NT>(s, sh);
    if (threadIdx.x == 0) {
        auto st = gmem(a.st);
        st->mass_sum = s;
        st->theta += a.k0_dz_over_P * s;
        st->steps += 1;
        if (!isfinite(s)) st->nonfinite = 1;
    }
}

// LDS of a persistent LM block: the tile and the reduction scratch, then the
// twiddles and the mode's per-axis table while they fit in the 160 KiB of a
// CU (long lines with wide tiles leave no room: those tables are then read
// from global memory, where every block reads the same few KiB).
template <int N, int E, int LINES, int MODE, class LT> struct LmpLds {
    static constexpr long kLimit = 160L * 1024;
    static constexpr long BASE = (long)sizeof(LT) * LmTile<N, E, LINES>::LDS + 8L * (LmTile<N, E, LINES>::NT / 64 + 1);
    static constexpr long TAB = MODE == LM_KIN ? 16L * N : MODE == LM_KERN ? 8L * N : 0;
    static constexpr bool TW = BASE + 16L * N + TAB <= kLimit;   // twiddles in LDS
    static constexpr bool TB = BASE + TAB + (TW ? 16L * N : 0) <= kLimit;   // mode table in LDS
};

// Tables shared by every tile (and, in a group, by every instance: the host
// only groups instances whose tables are identical) go to LDS once (TW_L,
// TB_L); otherwise twl / kpl / k2l point at the global tables.
template <int N, int E, int LINES, int MODE, class LT, class Src, bool TW_L = true, bool TB_L = true>
__device__ __forceinline__ void lmp_body(const Src &src, LT *lds, const double2 *twl, const double2 *kpl,
                                         const double *k2l, double *sh)
{
    constexpr int TPL = N / E, NT = LINES * TPL;
    static_assert(MODE == LM_FWD || MODE == LM_INV || MODE == LM_KIN || MODE == LM_KERN, "mode");
    const int tid = threadIdx.x, l = tid % LINES, t = tid / LINES;
    {
        const LmArgs &a0 = src.args(0);
        for (int i = tid; i < N; i += NT) {
            if constexpr (TW_L) const_cast<double2 *>(twl)[i] = gld(a0.tw, i);
            if constexpr (MODE == LM_KIN && TB_L) const_cast<double2 *>(kpl)[i] = gld(a0.kinp, i);
            if constexpr (MODE == LM_KERN && TB_L) const_cast<double *>(k2l)[i] = gmem(a0.k2_p)[i];
        }
        if constexpr (!Src::GROUPED) {
            if (a0.reduce && blockIdx.x == 0) reduce_mass<NT>(a0, sh);
        }
    }
    __syncthreads();
    const int ntiles = src.ntiles();
    int tile = blockIdx.x;
    if (tile >= ntiles) return;
    const LmLayout<LINES> lay{l};
    LmPrefetch<E> f;
    lm_fetch<N, E, LINES, MODE>(src.args(tile), lm_where<N, E, LINES>(src.args(tile), src.local(tile), l, t), true, f);
    dc v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = from_f2(f.p[e]);
    // this tile's line factors, taken before the prefetch reuses f
    dc m12 = mk(0.0, 0.0);
    double q12 = 0.0;
    if constexpr (MODE == LM_KIN) m12 = scl(cmul(from_d2(f.f1), from_d2(f.f2)), src.args(tile).scale);
    if constexpr (MODE == LM_KERN) q12 = f.q1 + f.q2;
    for (;;) {
        const LmArgs &a = src.args(tile);
        const int nxt = tile + gridDim.x;
        const bool more = nxt < ntiles;
        {
            const int pf = more ? nxt : tile;
            const LmArgs &an = src.args(pf);
            lm_fetch<N, E, LINES, MODE>(an, lm_where<N, E, LINES>(an, src.local(pf), l, t), more, f);
        }
        if constexpr (Src::GROUPED) {
            if (a.reduce && src.local(tile) == 0) reduce_mass<NT>(a, sh);
        }
        if constexpr (MODE == LM_FWD || MODE == LM_INV) {
            fft<N, E, MODE == LM_FWD ? -1 : 1>(v, t, lay, lds, twl);
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] = scl(v[e], a.scale);
        } else {
            fft<N, E, -1>(v, t, lay, lds, twl);
            if constexpr (MODE == LM_KIN) {
#pragma unroll
                for (int e = 0; e < E; ++e) v[e] = cmul(v[e], cmul(m12, from_d2(kpl[t + TPL * e])));
            } else {
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    // branch-free: k = 0 divides by 1 and is then zeroed
                    const double k2 = q12 + k2l[t + TPL * e];
                    const bool pos = k2 > 0.0;
                    const double km = k2 + a.mY2;
                    const double num = fma(a.cN, km, a.cY * k2);
                    const double den = pos ? k2 * km : 1.0;
                    double r = __builtin_amdgcn_rcp(den);
                    r = fma(r, fma(-den, r, 1.0), r);
                    r = fma(r, fma(-den, r, 1.0), r);
                    const double K = pos ? fma(num, r, a.c0) : 0.0;
                    v[e] = scl(v[e], K * a.scale);
                }
            }
            fft<N, E, 1>(v, t, lay, lds, twl);
        }
        const LmWhere w = lm_where<N, E, LINES>(a, src.local(tile), l, t);
#pragma unroll
        for (int e = 0; e < E; ++e) buf_st2(to_f2(v[e]), w.r, w.voff, e * w.step);
        if (!more) break;
        // convert here, where the only outstanding operations are this
        // iteration's loads and stores (the empty asm keeps the compiler from
        // sinking the conversion into the loop header, whose wait would then
        // also have to cover the path from the first fetch: vmcnt(0))
        convert_pinned(v, f.p, std::make_integer_sequence<int, E>{});
        if constexpr (MODE == LM_KIN) {
            m12 = scl(cmul(from_d2(f.f1), from_d2(f.f2)), src.args(nxt).scale);
            pin(m12);
        }
        if constexpr (MODE == LM_KERN) {
            q12 = f.q1 + f.q2;
            asm volatile("" : "+v"(q12));
        }
        tile = nxt;
    }
}

// ---------------------------------------------------------------- two-butterfly LM pass
// The persistent strided pass for lines of N = 8^S points with 16 points per
// thread: each thread runs two radix-8 butterflies per stage, so a 16-line
// tile of 512-point lines takes 512 threads.  Between stages the values stay
// in registers as the complex64 numbers the LDS exchange holds (widened to
// FP64 one butterfly at a time); the forward transform's last stage, the
// pointwise multiplier and the inverse transform's first stage run back to
// back per butterfly in FP64, and the last stage stores its outputs directly.
// At N = 512 a thread then fits 128 VGPRs and a block's LDS (tile, twiddles,
// per-axis table) 80 KiB, so two blocks share a CU and one block's barriers
// and memory waits are covered by the other's work; the next tile is loaded
// after the stores, not prefetched.  Every butterfly, twiddle and rounding
// point is that of the 8-point plan (Plan<N, 8>), so the results are bitwise
// those of the one-butterfly passes k_lm / k_lmp with E = 8.
template <int N> struct R8 {
    static constexpr int E = 16, TPL = N / E;
    static constexpr int stages()
    {
        int s = 0;
        long p = 1;
        while (p < N) { p *= 8; ++s; }
        return s;
    }
    static constexpr bool POW8 = [] { long p = 1; while (p < N) p *= 8; return p == N; }();
    static constexpr int ns(int st)
    {
        int p = 1;
        for (int i = 0; i < st; ++i) p *= 8;
        return p;
    }
    // twiddle indices (j mod Ns) r N / (8 Ns) stay below this
    static constexpr int TWN = (N / 8 - 1) * 7 + 1;
};

// Butterfly m (0 or 1) of stage ST: j = t + TPL m takes positions j + r N / 8,
// held in u[m + 2 r]; twiddled and transformed in FP64 into a.
template <int N, int S, int ST>
__device__ __forceinline__ void r8_in(const float2 (&u)[16], int m, int t, const double2 *__restrict__ tw, dc (&a)[8])
{
    constexpr int NS = R8<N>::ns(ST), STEP = N / (NS * 8);
    const int j = t + R8<N>::TPL * m;
#pragma unroll
    for (int r = 0; r < 8; ++r) a[r] = from_f2(u[m + 2 * r]);
    if constexpr (NS > 1) {
        const int jm = j & (NS - 1);
#pragma unroll
        for (int r = 1; r < 8; ++r) {
            dc w = from_d2(tw[jm * r * STEP]);
            if constexpr (S > 0) w.y = -w.y;
            a[r] = cmul(a[r], w);
        }
    }
    dft<8, S>(a);
}

// Outputs of butterfly m of a stage that is not the last: LDS positions
// expand(j) + r Ns.
template <int N, int ST, class Lay>
__device__ __forceinline__ void r8_out(const dc (&a)[8], int m, int t, const Lay &lay, float2 *lds)
{
    constexpr int NS = R8<N>::ns(ST);
    const int j = t + R8<N>::TPL * m;
    const int base = (j / NS) * NS * 8 + (j & (NS - 1));
#pragma unroll
    for (int r = 0; r < 8; ++r) lds_put(lds, lay(base + r * NS), a[r]);
}

// The exchange after a stage: u[e] takes position t + TPL e.
template <int N, class Lay>
__device__ __forceinline__ void r8_exchange(float2 (&u)[16], int t, const Lay &lay, const float2 *lds)
{
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 16; ++e) u[e] = lds[lay(t + R8<N>::TPL * e)];
    __syncthreads();
}

// Stages ST .. STOP - 1 of a transform, each ending in an exchange.
template <int N, int S, int ST, int STOP, class Lay>
__device__ __forceinline__ void r8_stages(float2 (&u)[16], int t, const Lay &lay, float2 *lds,
                                          const double2 *__restrict__ tw)
{
    if constexpr (ST < STOP) {
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            dc a[8];
            r8_in<N, S, ST>(u, m, t, tw, a);
            r8_out<N, ST>(a, m, t, lay, lds);
        }
        r8_exchange<N>(u, t, lay, lds);
        r8_stages<N, S, ST + 1, STOP>(u, t, lay, lds, tw);
    }
}

__device__ __forceinline__ void pin_f2(float2 &x) { asm volatile("" : "+v"(x.x), "+v"(x.y)); }

template <int N, int LINES, int MODE, class Src>
__device__ __forceinline__ void lmp2_body(const Src &src, float2 *lds, double2 *twl, double2 *kpl, double *k2l,
                                          double *sh)
{
    using P = R8<N>;
    constexpr int E = P::E, TPL = P::TPL, NT = LINES * TPL, LAST = P::stages() - 1;
    static_assert(P::POW8 && LAST >= 1, "two-butterfly pass: N = 8^S, S >= 2");
    static_assert(MODE == LM_FWD || MODE == LM_INV || MODE == LM_KIN || MODE == LM_KERN, "mode");
    const int tid = threadIdx.x, l = tid % LINES, t = tid / LINES;
    {
        const LmArgs &a0 = src.args(0);
        for (int i = tid; i < N; i += NT) {
            if (i < P::TWN) twl[i] = gld(a0.tw, i);
            if constexpr (MODE == LM_KIN) kpl[i] = gld(a0.kinp, i);
            if constexpr (MODE == LM_KERN) k2l[i] = gmem(a0.k2_p)[i];
        }
        if constexpr (!Src::GROUPED) {
            if (a0.reduce && blockIdx.x == 0) reduce_mass<NT>(a0, sh);
        }
    }
    __syncthreads();
    const int ntiles = src.ntiles();
    int tile = blockIdx.x;
    if (tile >= ntiles) return;
    const LmLayout<LINES> lay{l};
    LmPrefetch<E> f;
    lm_fetch<N, E, LINES, MODE>(src.args(tile), lm_where<N, E, LINES>(src.args(tile), src.local(tile), l, t), true, f);
    float2 u[E];
#pragma unroll
    for (int e = 0; e < E; ++e) u[e] = f.p[e];
    dc m12 = mk(0.0, 0.0);
    double q12 = 0.0;
    if constexpr (MODE == LM_KIN) m12 = scl(cmul(from_d2(f.f1), from_d2(f.f2)), src.args(tile).scale);
    if constexpr (MODE == LM_KERN) q12 = f.q1 + f.q2;
    for (;;) {
        const LmArgs &a = src.args(tile);
        const int nxt = tile + gridDim.x;
        const bool more = nxt < ntiles;
        if constexpr (Src::GROUPED) {
            if (a.reduce && src.local(tile) == 0) reduce_mass<NT>(a, sh);
        }
        constexpr int SF = MODE == LM_INV ? 1 : -1;   // sign of the (first) transform
        r8_stages<N, SF, 0, LAST>(u, t, lay, lds, twl);
        if constexpr (MODE == LM_KIN || MODE == LM_KERN) {
            // forward last stage, multiplier, inverse first stage (no twiddles)
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                dc z[8];
                r8_in<N, -1, LAST>(u, m, t, twl, z);
                // kinetic factors: no LDS read moves above this point (hoisted
                // next to the twiddles they need 3 VGPRs more than the 128 of
                // two blocks per CU, and the spill reaches HBM); 0x27F lets
                // every other kind of instruction cross
                if constexpr (MODE == LM_KIN) __builtin_amdgcn_sched_barrier(0x27F);
                const int j = t + TPL * m;
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const int pos = j + (N / 8) * r;
                    if constexpr (MODE == LM_KIN) {
                        z[r] = cmul(z[r], cmul(m12, from_d2(kpl[pos])));
                    } else {
                        // branch-free: k = 0 divides by 1 and is then zeroed
                        const double k2 = q12 + k2l[pos];
                        const bool pos_k = k2 > 0.0;
                        const double km = k2 + a.mY2;
                        const double num = fma(a.cN, km, a.cY * k2);
                        const double den = pos_k ? k2 * km : 1.0;
                        double rc = __builtin_amdgcn_rcp(den);
                        rc = fma(rc, fma(-den, rc, 1.0), rc);
                        rc = fma(rc, fma(-den, rc, 1.0), rc);
                        const double K = pos_k ? fma(num, rc, a.c0) : 0.0;
                        z[r] = scl(z[r], K * a.scale);
                    }
                }
                dft<8, 1>(z);
                r8_out<N, 0>(z, m, t, lay, lds);
            }
            r8_exchange<N>(u, t, lay, lds);
            r8_stages<N, 1, 1, LAST>(u, t, lay, lds, twl);
        }
        constexpr int SL = MODE == LM_FWD ? -1 : 1;   // sign of the last stage
        const LmWhere w = lm_where<N, E, LINES>(a, src.local(tile), l, t);
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            dc z[8];
            r8_in<N, SL, LAST>(u, m, t, twl, z);
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                if constexpr (MODE == LM_FWD || MODE == LM_INV) z[r] = scl(z[r], a.scale);
                buf_st2(to_f2(z[r]), w.r, w.voff, (m + 2 * r) * w.step);
            }
        }
        if (!more) break;
        // the next tile: no register prefetch (it would not fit 128 VGPRs);
        // the other block on the CU works while this one waits
        {
            const LmArgs &an = src.args(nxt);
            lm_fetch<N, E, LINES, MODE>(an, lm_where<N, E, LINES>(an, src.local(nxt), l, t), true, f);
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
            u[e] = f.p[e];
            pin_f2(u[e]);
        }
        if constexpr (MODE == LM_KIN) {
            m12 = scl(cmul(from_d2(f.f1), from_d2(f.f2)), src.args(nxt).scale);
            pin(m12);
        }
        if constexpr (MODE == LM_KERN) {
            q12 = f.q1 + f.q2;
            asm volatile("" : "+v"(q12));
        }
        tile = nxt;
    }
}

// ---------------------------------------------------------------- pipelined EM passes
// The density and phase passes in the same persistent, prefetching form: a
// block walks tiles of LINES row pairs; each row's loads for the next tile are
// issued as soon as that row's registers of the current tile have been
// converted, twiddles come from LDS, and rows past the end of the grid take
// the last row pair (identical loads, arithmetic and stores; they add nothing
// to the mass partial).  Loads with live = false read the tile's first point.
template <int N, int E, int LINES>
__device__ __forceinline__ int em_pair(const EmArgs &a, int tile, int l)
{
    return min(tile * LINES + l, a.nlines - 1);
}

// psi row r (0 or 1) of the pair `pair`: E float2 at positions t + TPL e
template <int N, int E>
__device__ __forceinline__ void em_fetch_row(const EmArgs &a, int pair, int r, int t, bool live, float2 (&p)[E])
{
    constexpr int TPL = N / E;
    const int pair0 = __builtin_amdgcn_readfirstlane(pair);
    const __amdgpu_buffer_rsrc_t rs = buf_rsrc(a.psi + (long long)pair0 * 2 * N);
    const unsigned vo = live ? (unsigned)(((pair - pair0) * 2 * N + r * N + t) * 8) : 0u;
#pragma unroll
    for (int e = 0; e < E; ++e) p[e] = buf_ld2(rs, vo, live ? e * TPL * 8 : 0);
}

template <int N, int E>
__device__ __forceinline__ void em_store_row(const EmArgs &a, int pair, int r, int t, const dc (&v)[E], double s)
{
    constexpr int TPL = N / E;
    const int pair0 = __builtin_amdgcn_readfirstlane(pair);
    const __amdgpu_buffer_rsrc_t rs = buf_rsrc(a.psi + (long long)pair0 * 2 * N);
    const unsigned vo = (unsigned)(((pair - pair0) * 2 * N + r * N + t) * 8);
#pragma unroll
    for (int e = 0; e < E; ++e) buf_st2(to_f2(scl(v[e], s)), rs, vo, e * TPL * 8);
}

// Half spectra of the two phi rows of a pair, as load_phi_pair reads them
// (bin k for e < E/2, bin N - k for e >= E/2; the Nyquist bin separately).
template <int N, int E> struct PhiRaw {
    float2 h0[E], h1[E];
    float2 n0, n1;
};

template <int N, int E>
__device__ __forceinline__ void em_fetch_raw(float2 *half, const float2 *nyq, int pair, int t, bool live,
                                             PhiRaw<N, E> &f)
{
    constexpr int TPL = N / E, H = N / 2;
    const int pair0 = __builtin_amdgcn_readfirstlane(pair);
    const __amdgpu_buffer_rsrc_t rs = buf_rsrc(half + (long long)pair0 * 2 * H);
    const int row = live ? (pair - pair0) * 2 * H : 0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        int idx;
        if (e < E / 2) idx = t + TPL * e;
        else if (e == E / 2) idx = t == 0 ? 0 : N - (t + TPL * e);
        else idx = N - (t + TPL * e);
        if (!live) idx = 0;
        const unsigned vo = (unsigned)((row + idx) * 8);
        f.h0[e] = buf_ld2(rs, vo, 0);
        f.h1[e] = buf_ld2(rs, vo, H * 8);
    }
    const long long r0 = live ? 2LL * pair : 2LL * pair0;
    f.n0 = gld(nyq, r0);
    f.n1 = gld(nyq, r0 + 1);
}

template <int N, int E>
__device__ __forceinline__ void em_fetch_phi(const EmArgs &a, int pair, int t, bool live, PhiRaw<N, E> &f)
{
    em_fetch_raw<N, E>(a.half, a.nyq, pair, t, live, f);
}

// A real field (static potential, coupling coefficients) at both rows of a
// pair, E floats each; live = false: the pair's first point, so the count of
// loads per iteration stays fixed.
template <int N, int E>
__device__ __forceinline__ void em_fetch_field(const float *f, int pair, int t, bool live, float (&v0)[E],
                                               float (&v1)[E])
{
    constexpr int TPL = N / E;
    const auto b = gmem(f) + (long long)pair * 2 * N + (live ? t : 0);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        v0[e] = b[live ? TPL * e : 0];
        v1[e] = b[live ? N + TPL * e : 0];
    }
}

// one row of a pair only
template <int N, int E>
__device__ __forceinline__ void em_fetch_field_row(const float *f, int pair, int r, int t, bool live, float (&v)[E])
{
    constexpr int TPL = N / E;
    const auto b = gmem(f) + (long long)pair * 2 * N + r * N + (live ? t : 0);
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = b[live ? TPL * e : 0];
}

template <int N, int E>
__device__ __forceinline__ void em_fetch_vext(const EmArgs &a, int pair, int t, bool live, float (&v0)[E],
                                              float (&v1)[E])
{
    em_fetch_field<N, E>(a.vext, pair, t, live, v0, v1);
}

// The full spectrum Z = X_0 + i X_1 of the pair (conjugate symmetry; DC and
// Nyquist real), the same operations as load_phi_pair.
template <int N, int E>
__device__ __forceinline__ void em_build_z(const PhiRaw<N, E> &f, int t, dc (&z)[E])
{
#pragma unroll
    for (int e = 0; e < E; ++e) {
        dc x0 = from_f2(f.h0[e]), x1 = from_f2(f.h1[e]);
        if (e < E / 2) {
            if (e == 0 && t == 0) { x0.y = 0.0; x1.y = 0.0; }
        } else if (e == E / 2 && t == 0) {
            x0 = mk((double)f.n0.x, 0.0);
            x1 = mk((double)f.n1.x, 0.0);
        } else {
            x0 = conj(x0);
            x1 = conj(x1);
        }
        z[e] = mk(x0.x - x1.y, x0.y + x1.x);
    }
}

template <int E, int... I>
__device__ __forceinline__ void pin_all(dc (&v)[E], std::integer_sequence<int, I...>)
{
    (pin(v[I]), ...);
}

template <int N, int E, int LINES>
__device__ __forceinline__ void copy_twiddles(const double2 *__restrict__ tw, double2 *twl)
{
    constexpr int NT = LINES * (N / E);
    for (int i = threadIdx.x; i < N; i += NT) twl[i] = gld(tw, i);
    __syncthreads();
}

// Phase pass (as phase_tile without ENERGY).
template <int N, int E, int LINES, bool REAL_IN, class LT, class Src>
__device__ __forceinline__ void phasep_body(const Src &src, LT *lds, double2 *twl, double2 *scl_tab)
{
    constexpr int TPL = N / E, NT = LINES * TPL;
    const int tid = threadIdx.x, t = tid % TPL, l = tid / TPL;
    for (int i = tid; i < kSinCosTable; i += NT) scl_tab[i] = gld(src.args(0).sct, i);
    copy_twiddles<N, E, LINES>(src.args(0).tw, twl);
    const int ntiles = src.ntiles();
    int tile = blockIdx.x;
    if (tile >= ntiles) return;
    const EmLayout<N, E> lay{l * EmLayout<N, E>::PITCH};
    const double inv_n = 1.0 / N;
    PhiRaw<N, E> fp;
    float2 p0[E], p1[E];
    int pair = em_pair<N, E, LINES>(src.args(tile), src.local(tile), l);
    em_fetch_phi<N, E>(src.args(tile), pair, t, true, fp);
    em_fetch_row<N, E>(src.args(tile), pair, 0, t, true, p0);
    em_fetch_row<N, E>(src.args(tile), pair, 1, t, true, p1);
    // nothing outstanding on entry to the loop: its waits then only count
    // the loop's own operations
    __builtin_amdgcn_s_waitcnt(0);
    dc z[E];
    em_build_z<N, E>(fp, t, z);
    for (;;) {
        const EmArgs &a = src.args(tile);
        const int nxt = tile + gridDim.x;
        const bool more = nxt < ntiles;
        const EmArgs &an = src.args(more ? nxt : tile);
        const int npair = more ? em_pair<N, E, LINES>(an, src.local(nxt), l) : pair;
        fft<N, E, 1>(z, t, lay, lds, twl);
        float phi0[E], phi1[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            phi0[e] = (float)(z[e].x * inv_n);
            phi1[e] = (float)(z[e].y * inv_n);
        }
        em_fetch_phi<N, E>(an, npair, t, more, fp);
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            dc v[E];
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] = from_f2(half ? p1[e] : p0[e]);
            // both rows of the next tile once both of this tile's are in
            // registers: fewer prefetch registers live at once
            if (half) {
                em_fetch_row<N, E>(an, npair, 0, t, more, p0);
                em_fetch_row<N, E>(an, npair, 1, t, more, p1);
            }
            if constexpr (!REAL_IN) fft<N, E, 1>(v, t, lay, lds, twl);
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const dc ps = REAL_IN ? v[e] : scl(v[e], inv_n);
                const double rho = norm2(ps);
                const double phi = (double)(half ? phi1[e] : phi0[e]);
                double sn, cs;
                sincos_tab(fma(a.g, rho, phi) * a.dz, scl_tab, &sn, &cs);
                v[e] = cmul(ps, mk(cs, sn));
            }
            fft<N, E, -1>(v, t, lay, lds, twl);
            em_store_row<N, E>(a, pair, half, t, v, 1.0);
        }
        if (!more) break;
        em_build_z<N, E>(fp, t, z);
        pin_all(z, std::make_integer_sequence<int, E>{});
        tile = nxt;
        pair = npair;
    }
}

// Phase pass with the local terms of Eq. (15) and the static potential, in
// the persistent prefetching form of phasep_body: the next tile's phi half
// spectra, lap(sqrt rho) half spectra (BOHM), psi rows and static potential
// (VEXT) are fetched while the current tile is transformed.
template <int N, int E, int LINES, bool REAL_IN, bool BOHM, bool VEXT, class LT, class Src>
__device__ __forceinline__ void phasep_local_body(const Src &src, LT *lds, double2 *twl, double2 *scl_tab,
                                                  float *stash)
{
    constexpr int TPL = N / E, NT = LINES * TPL;
    const int tid = threadIdx.x, t = tid % TPL, l = tid / TPL;
    for (int i = tid; i < kSinCosTable; i += NT) scl_tab[i] = gld(src.args(0).sct, i);
    copy_twiddles<N, E, LINES>(src.args(0).tw, twl);
    const int ntiles = src.ntiles();
    int tile = blockIdx.x;
    if (tile >= ntiles) return;
    const EmLayout<N, E> lay{l * EmLayout<N, E>::PITCH};
    const double inv_n = 1.0 / N;
    PhiRaw<N, E> fp, fl;
    float2 p0[E], p1[E];
    float vx0[E], vx1[E];
    int pair = em_pair<N, E, LINES>(src.args(tile), src.local(tile), l);
    em_fetch_phi<N, E>(src.args(tile), pair, t, true, fp);
    if constexpr (BOHM) em_fetch_raw<N, E>(src.args(tile).half2, src.args(tile).nyq2, pair, t, true, fl);
    em_fetch_row<N, E>(src.args(tile), pair, 0, t, true, p0);
    em_fetch_row<N, E>(src.args(tile), pair, 1, t, true, p1);
    if constexpr (VEXT) em_fetch_vext<N, E>(src.args(tile), pair, t, true, vx0, vx1);
    __builtin_amdgcn_s_waitcnt(0);
    dc z[E];
    em_build_z<N, E>(fp, t, z);
    for (;;) {
        const EmArgs &a = src.args(tile);
        const int nxt = tile + gridDim.x;
        const bool more = nxt < ntiles;
        const EmArgs &an = src.args(more ? nxt : tile);
        const int npair = more ? em_pair<N, E, LINES>(an, src.local(nxt), l) : pair;
        fft<N, E, 1>(z, t, lay, lds, twl);
        float phi0[E], phi1[E], lap0[E], lap1[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            phi0[e] = (float)(z[e].x * inv_n);
            phi1[e] = (float)(z[e].y * inv_n);
            lap0[e] = 0.0f;
            lap1[e] = 0.0f;
        }
        if constexpr (BOHM) {
            // phi waits in LDS (each thread its own slots) during the lap
            // transform and the rows: fewer live registers
#pragma unroll
            for (int e = 0; e < E; ++e) {
                stash[e * NT + tid] = phi0[e];
                stash[(E + e) * NT + tid] = phi1[e];
            }
        }
        em_fetch_phi<N, E>(an, npair, t, more, fp);
        if constexpr (BOHM) {
            em_build_z<N, E>(fl, t, z);
            fft<N, E, 1>(z, t, lay, lds, twl);
#pragma unroll
            for (int e = 0; e < E; ++e) {
                stash[(2 * E + e) * NT + tid] = (float)(z[e].x * inv_n);
                stash[(3 * E + e) * NT + tid] = (float)(z[e].y * inv_n);
            }
        }
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            if constexpr (BOHM) {
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    if (half) {
                        phi1[e] = stash[(E + e) * NT + tid];
                        lap1[e] = stash[(3 * E + e) * NT + tid];
                    } else {
                        phi0[e] = stash[e * NT + tid];
                        lap0[e] = stash[(2 * E + e) * NT + tid];
                    }
                }
            }
            dc v[E];
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] = from_f2(half ? p1[e] : p0[e]);
            if (half) {
                em_fetch_row<N, E>(an, npair, 0, t, more, p0);
                em_fetch_row<N, E>(an, npair, 1, t, more, p1);
            }
            if constexpr (!REAL_IN) fft<N, E, 1>(v, t, lay, lds, twl);
            double rho[E], U[E];
            float lp[E];
#pragma unroll
            for (int e = 0; e < E; ++e) {
                if constexpr (!REAL_IN) v[e] = scl(v[e], inv_n);
                rho[e] = norm2(v[e]);
                lp[e] = half ? lap1[e] : lap0[e];
            }
            local_potential<E>(a, rho, lp, U);
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const double vv = VEXT ? (double)(half ? vx1[e] : vx0[e]) : 0.0;
                const double th = (U[e] + vv + (double)(half ? phi1[e] : phi0[e])) * a.dz;
                double sn, cs;
                sincos_tab(th, scl_tab, &sn, &cs);
                v[e] = cmul(v[e], mk(cs, sn));
            }
            fft<N, E, -1>(v, t, lay, lds, twl);
            em_store_row<N, E>(a, pair, half, t, v, 1.0);
        }
        // the next tile's lap(sqrt rho) spectra and static potential, fetched
        // only now: their registers are free while the rows are worked on,
        // and the next tile's phi transform covers their latency
        if constexpr (BOHM) em_fetch_raw<N, E>(an.half2, an.nyq2, npair, t, more, fl);
        if constexpr (VEXT) em_fetch_vext<N, E>(an, npair, t, more, vx0, vx1);
        if (!more) break;
        em_build_z<N, E>(fp, t, z);
        pin_all(z, std::make_integer_sequence<int, E>{});
        tile = nxt;
        pair = npair;
    }
}

// Source pass (as source_tile) in the persistent prefetching form: the next
// tile's lap(rho) half spectra (LAP), psi rows and coefficient fields are
// fetched while the current tile is transformed; s's half spectra replace the
// current tile's in place.
template <int N, int E, int LINES, bool REAL_IN, bool LAP, bool GAM, class LT, class Src>
__device__ __forceinline__ void sourcep_body(const Src &src, LT *lds, double2 *twl)
{
    constexpr int TPL = N / E, H = N / 2;
    const int tid = threadIdx.x, t = tid % TPL, l = tid / TPL;
    copy_twiddles<N, E, LINES>(src.args(0).tw, twl);
    const int ntiles = src.ntiles();
    int tile = blockIdx.x;
    if (tile >= ntiles) return;
    const EmLayout<N, E> lay{l * EmLayout<N, E>::PITCH};
    const double inv_n = 1.0 / N;
    const double rs = REAL_IN ? 1.0 : inv_n * inv_n;
    PhiRaw<N, E> fl;
    float2 p0[E], p1[E];
    float g0[E], g1[E], b0[E], b1[E];
    int pair = em_pair<N, E, LINES>(src.args(tile), src.local(tile), l);
    if constexpr (LAP) em_fetch_raw<N, E>(src.args(tile).half, src.args(tile).nyq, pair, t, true, fl);
    em_fetch_row<N, E>(src.args(tile), pair, 0, t, true, p0);
    em_fetch_row<N, E>(src.args(tile), pair, 1, t, true, p1);
    if constexpr (GAM) em_fetch_field<N, E>(src.args(tile).gam, pair, t, true, g0, g1);
    if constexpr (LAP) em_fetch_field<N, E>(src.args(tile).bet, pair, t, true, b0, b1);
    __builtin_amdgcn_s_waitcnt(0);
    for (;;) {
        const EmArgs &a = src.args(tile);
        const int nxt = tile + gridDim.x;
        const bool more = nxt < ntiles;
        const EmArgs &an = src.args(more ? nxt : tile);
        const int npair = more ? em_pair<N, E, LINES>(an, src.local(nxt), l) : pair;
        dc z[E];
        float lap0[E], lap1[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            lap0[e] = 0.0f;
            lap1[e] = 0.0f;
        }
        if constexpr (LAP) {
            em_build_z<N, E>(fl, t, z);
            fft<N, E, 1>(z, t, lay, lds, twl);
#pragma unroll
            for (int e = 0; e < E; ++e) {
                lap0[e] = (float)(z[e].x * inv_n);
                lap1[e] = (float)(z[e].y * inv_n);
            }
            em_fetch_raw<N, E>(an.half, an.nyq, npair, t, more, fl);
        }
        double s0[E];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            dc v[E];
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] = from_f2(h ? p1[e] : p0[e]);
            em_fetch_row<N, E>(an, npair, h, t, more, h ? p1 : p0);
            if constexpr (!REAL_IN) fft<N, E, 1>(v, t, lay, lds, twl);
#pragma unroll
            for (int e = 0; e < E; ++e) {
                double sv = norm2(v[e]) * rs;
                if constexpr (GAM) sv *= (double)(h ? g1[e] : g0[e]);
                if constexpr (LAP) sv = fma((double)(h ? b1[e] : b0[e]), (double)(h ? lap1[e] : lap0[e]), sv);
                if (h) z[e] = mk(s0[e], sv);
                else s0[e] = sv;
            }
            if constexpr (GAM) em_fetch_field_row<N, E>(an.gam, npair, h, t, more, h ? g1 : g0);
            if constexpr (LAP) em_fetch_field_row<N, E>(an.bet, npair, h, t, more, h ? b1 : b0);
        }
        fft<N, E, -1>(z, t, lay, lds, twl);
#pragma unroll
        for (int e = 0; e < E; ++e) lds_put(lds, lay(t + TPL * e), z[e]);
        exchange_sync<EmLayout<N, E>::WAVE_LOCAL>();
        {
            const int pair0 = __builtin_amdgcn_readfirstlane(pair);
            const __amdgpu_buffer_rsrc_t rsr = buf_rsrc(a.half + (long long)pair0 * 2 * H);
            const unsigned vo = (unsigned)(((pair - pair0) * 2 * H + t) * 8);
#pragma unroll
            for (int e = 0; e < E / 2; ++e) {
                const int k = t + TPL * e;
                const dc zz = z[e];
                const dc zc = conj(lds_get(lds, lay((N - k) & (N - 1))));
                const dc sm = add(zz, zc), df = sub(zz, zc);
                buf_st2(to_f2(scl(sm, 0.5)), rsr, vo, e * TPL * 8);
                buf_st2(to_f2(mk(0.5 * df.y, -0.5 * df.x)), rsr, vo, H * 8 + e * TPL * 8);
            }
        }
        if (t == 0) {
            const dc zn = z[E / 2];
            gst(a.nyq, 2LL * pair, make_float2((float)zn.x, 0.0f));
            gst(a.nyq, 2LL * pair + 1, make_float2((float)zn.y, 0.0f));
        }
        // the LDS slots are rewritten by the next tile's first transform
        exchange_sync<EmLayout<N, E>::WAVE_LOCAL>();
        if (!more) break;
        tile = nxt;
        pair = npair;
    }
}

// Density pass (as density_tile).
template <int N, int E, int LINES, bool STORE_PSI, class LT, class Src, bool BOHM = false>
__device__ __forceinline__ void densityp_body(const Src &src, LT *lds, double2 *twl, double *sh)
{
    constexpr int TPL = N / E, NT = LINES * TPL, H = N / 2;
    const int tid = threadIdx.x, t = tid % TPL, l = tid / TPL;
    copy_twiddles<N, E, LINES>(src.args(0).tw, twl);
    const int ntiles = src.ntiles();
    int tile = blockIdx.x;
    if (tile >= ntiles) return;
    const EmLayout<N, E> lay{l * EmLayout<N, E>::PITCH};
    const double inv_n = 1.0 / N;
    float2 p0[E], p1[E];
    int pair = em_pair<N, E, LINES>(src.args(tile), src.local(tile), l);
    em_fetch_row<N, E>(src.args(tile), pair, 0, t, true, p0);
    em_fetch_row<N, E>(src.args(tile), pair, 1, t, true, p1);
    __builtin_amdgcn_s_waitcnt(0);
    dc v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = from_f2(p0[e]);
    for (;;) {
        const EmArgs &a = src.args(tile);
        const int loc = src.local(tile);
        const int nxt = tile + gridDim.x;
        const bool more = nxt < ntiles;
        const EmArgs &an = src.args(more ? nxt : tile);
        const int npair = more ? em_pair<N, E, LINES>(an, src.local(nxt), l) : pair;
        const bool real = loc * LINES + l < a.nlines;
        double rho0[E];
        em_fetch_row<N, E>(an, npair, 0, t, more, p0);
        fft<N, E, 1>(v, t, lay, lds, twl);
#pragma unroll
        for (int e = 0; e < E; ++e) rho0[e] = norm2(v[e]) * (inv_n * inv_n);
        if constexpr (STORE_PSI) em_store_row<N, E>(a, pair, 0, t, v, inv_n);
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = from_f2(p1[e]);
        em_fetch_row<N, E>(an, npair, 1, t, more, p1);
        fft<N, E, 1>(v, t, lay, lds, twl);
        if constexpr (STORE_PSI) em_store_row<N, E>(a, pair, 1, t, v, inv_n);
        double msum = 0.0;
        dc w[BOHM ? E : 1];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const double rho1 = norm2(v[e]) * (inv_n * inv_n);
            msum += rho0[e] + rho1;
            if constexpr (BOHM) w[e] = mk(sqrt(rho0[e]), sqrt(rho1));
            v[e] = mk(rho0[e], rho1);
        }
        fft<N, E, -1>(v, t, lay, lds, twl);
#pragma unroll
        for (int e = 0; e < E; ++e) lds_put(lds, lay(t + TPL * e), v[e]);
        exchange_sync<EmLayout<N, E>::WAVE_LOCAL>();
        {
            const int pair0 = __builtin_amdgcn_readfirstlane(pair);
            const __amdgpu_buffer_rsrc_t rs = buf_rsrc(a.half + (long long)pair0 * 2 * H);
            const unsigned vo = (unsigned)(((pair - pair0) * 2 * H + t) * 8);
#pragma unroll
            for (int e = 0; e < E / 2; ++e) {
                const int k = t + TPL * e;
                const dc zz = v[e];
                const dc zc = conj(lds_get(lds, lay((N - k) & (N - 1))));
                const dc sm = add(zz, zc), df = sub(zz, zc);
                buf_st2(to_f2(scl(sm, 0.5)), rs, vo, e * TPL * 8);
                buf_st2(to_f2(mk(0.5 * df.y, -0.5 * df.x)), rs, vo, H * 8 + e * TPL * 8);
            }
        }
        if (t == 0) {
            const dc zn = v[E / 2];   // bin N/2: both halves are real
            gst(a.nyq, 2LL * pair, make_float2((float)zn.x, 0.0f));
            gst(a.nyq, 2LL * pair + 1, make_float2((float)zn.y, 0.0f));
        }
        // the LDS slots are rewritten by the next tile's first transform
        exchange_sync<EmLayout<N, E>::WAVE_LOCAL>();
        if constexpr (BOHM) {
            // sqrt(rho) of both rows, the same split into half2 / nyq2
            fft<N, E, -1>(w, t, lay, lds, twl);
#pragma unroll
            for (int e = 0; e < E; ++e) lds_put(lds, lay(t + TPL * e), w[e]);
            exchange_sync<EmLayout<N, E>::WAVE_LOCAL>();
            const int pair0 = __builtin_amdgcn_readfirstlane(pair);
            const __amdgpu_buffer_rsrc_t rs = buf_rsrc(a.half2 + (long long)pair0 * 2 * H);
            const unsigned vo = (unsigned)(((pair - pair0) * 2 * H + t) * 8);
#pragma unroll
            for (int e = 0; e < E / 2; ++e) {
                const int k = t + TPL * e;
                const dc zz = w[e];
                const dc zc = conj(lds_get(lds, lay((N - k) & (N - 1))));
                const dc sm = add(zz, zc), df = sub(zz, zc);
                buf_st2(to_f2(scl(sm, 0.5)), rs, vo, e * TPL * 8);
                buf_st2(to_f2(mk(0.5 * df.y, -0.5 * df.x)), rs, vo, H * 8 + e * TPL * 8);
            }
            if (t == 0) {
                const dc zn = w[E / 2];
                gst(a.nyq2, 2LL * pair, make_float2((float)zn.x, 0.0f));
                gst(a.nyq2, 2LL * pair + 1, make_float2((float)zn.y, 0.0f));
            }
            exchange_sync<EmLayout<N, E>::WAVE_LOCAL>();
        }
        const double bs = block_sum<NT>(real ? msum : 0.0, sh);
        if (tid == 0) gmem(a.partials)[loc] = bs;
        if (!more) break;
        convert_pinned(v, p0, std::make_integer_sequence<int, E>{});
        tile = nxt;
        pair = npair;
    }
}

// ---------------------------------------------------------------- kernels
// One grid: block b is tile b.  Grouped: several instances of one shape in
// one launch; block b is tile (b mod tpi) of instance (b / tpi), whose
// arguments are read from a device array.
template <int N, int E, int LINES, int S, class ST = float2>
__global__ __launch_bounds__(LINES *(N / E)) void k_em_fft(EmArgs a)
{
    __shared__ ST lds[EmTile<N, E, LINES>::LDS];
    em_fft_tile<N, E, LINES, S>(a, blockIdx.x, lds);
}
template <int N, int E, int LINES, bool STORE_PSI, bool BOHM = false, class ST = float2>
__global__ __launch_bounds__(LINES *(N / E)) void k_density(EmArgs a)
{
    __shared__ ST lds[EmTile<N, E, LINES>::LDS];
    __shared__ double sh[EmTile<N, E, LINES>::NT / 64 + 1];
    density_tile<N, E, LINES, STORE_PSI, false, BOHM>(a, blockIdx.x, lds, sh);
}
template <int N, int E, int LINES, bool REAL_IN, bool LAP>
__global__ __launch_bounds__(LINES *(N / E)) void k_source(EmArgs a)
{
    __shared__ float2 lds[EmTile<N, E, LINES>::LDS];
    source_tile<N, E, LINES, REAL_IN, LAP>(a, blockIdx.x, lds);
}
template <int N, int E, int LINES, bool ENERGY, bool REAL_IN>
__global__ __launch_bounds__(LINES *(N / E)) void k_phase_local(EmArgs a)
{
    __shared__ float2 lds[EmTile<N, E, LINES>::LDS];
    __shared__ double sh[EmTile<N, E, LINES>::NT / 64 + 1];
    phase_local_tile<N, E, LINES, ENERGY, REAL_IN>(a, blockIdx.x, lds, sh);
}
template <int N, int E, int LINES>
__global__ __launch_bounds__(LINES *(N / E)) void k_density_real(EmArgs a)
{
    __shared__ float2 lds[EmTile<N, E, LINES>::LDS];
    __shared__ double sh[EmTile<N, E, LINES>::NT / 64 + 1];
    density_tile<N, E, LINES, false, true>(a, blockIdx.x, lds, sh);
}
template <int N, int E, int LINES, bool ENERGY, bool REAL_IN, class ST = float2>
__global__ __launch_bounds__(LINES *(N / E)) void k_phase(EmArgs a)
{
    __shared__ ST lds[EmTile<N, E, LINES>::LDS];
    __shared__ double sh[EmTile<N, E, LINES>::NT / 64 + 1];
    phase_tile<N, E, LINES, ENERGY, REAL_IN>(a, blockIdx.x, lds, sh);
}
template <int N, int E, int LINES>
__global__ __launch_bounds__(LINES *(N / E)) void k_potential(EmArgs a)
{
    __shared__ float2 lds[EmTile<N, E, LINES>::LDS];
    potential_tile<N, E, LINES>(a, blockIdx.x, lds);
}
template <int N, int E, int LINES, int MODE, class ST = float2>
__global__ __launch_bounds__(LINES *(N / E)) void k_lm(LmArgs a)
{
    __shared__ ST lds[LmTile<N, E, LINES>::LDS];
    __shared__ double sh[LmTile<N, E, LINES>::NT / 64 + 1];
    lm_tile<N, E, LINES, MODE>(a, blockIdx.x, lds, sh);
}

// Pipelined EM passes (persistent grid); LT: complex64 or complex128 LDS slots.
template <int N, int E, int LINES, bool REAL_IN, class LT = float2>
__global__ __launch_bounds__(LINES *(N / E)) void k_phasep(EmArgs a)
{
    __shared__ LT lds[EmTile<N, E, LINES>::LDS];
    __shared__ double2 twl[N];
    __shared__ double2 sct[kSinCosTable];
    const Src1<EmArgs> src{a, (a.nlines + LINES - 1) / LINES};
    phasep_body<N, E, LINES, REAL_IN, LT>(src, lds, twl, sct);
}
// Pipelined forms of the Eq. (15) density (also sqrt(rho)) and phase passes.
template <int N, int E, int LINES, bool STORE_PSI>
__global__ __launch_bounds__(LINES *(N / E)) void k_densityp_bohm(EmArgs a)
{
    __shared__ float2 lds[EmTile<N, E, LINES>::LDS];
    __shared__ double2 twl[N];
    __shared__ double sh[EmTile<N, E, LINES>::NT / 64 + 1];
    const Src1<EmArgs> src{a, (a.nlines + LINES - 1) / LINES};
    densityp_body<N, E, LINES, STORE_PSI, float2, Src1<EmArgs>, true>(src, lds, twl, sh);
}
template <int N, int E, int LINES, bool REAL_IN, bool LAP, bool GAM>
__global__ __launch_bounds__(LINES *(N / E)) void k_sourcep(EmArgs a)
{
    __shared__ float2 lds[EmTile<N, E, LINES>::LDS];
    __shared__ double2 twl[N];
    const Src1<EmArgs> src{a, (a.nlines + LINES - 1) / LINES};
    sourcep_body<N, E, LINES, REAL_IN, LAP, GAM, float2>(src, lds, twl);
}
template <int N, int E, int LINES, bool REAL_IN, bool BOHM, bool VEXT>
__global__ __launch_bounds__(LINES *(N / E)) void k_phasep_local(EmArgs a)
{
    __shared__ float2 lds[EmTile<N, E, LINES>::LDS];
    __shared__ double2 twl[N];
    __shared__ double2 sct[kSinCosTable];
    __shared__ float stash[BOHM ? 4 * E * LINES * (N / E) : 1];
    const Src1<EmArgs> src{a, (a.nlines + LINES - 1) / LINES};
    phasep_local_body<N, E, LINES, REAL_IN, BOHM, VEXT, float2>(src, lds, twl, sct, stash);
}
template <int N, int E, int LINES, bool STORE_PSI, class LT = float2>
__global__ __launch_bounds__(LINES *(N / E)) void k_densityp(EmArgs a)
{
    __shared__ LT lds[EmTile<N, E, LINES>::LDS];
    __shared__ double2 twl[N];
    __shared__ double sh[EmTile<N, E, LINES>::NT / 64 + 1];
    const Src1<EmArgs> src{a, (a.nlines + LINES - 1) / LINES};
    densityp_body<N, E, LINES, STORE_PSI, LT>(src, lds, twl, sh);
}
// Pipelined LM pass (persistent grid); LT: complex64 or complex128 LDS slots.
template <int N, int E, int LINES, int MODE, class LT>
__global__ __launch_bounds__(LINES *(N / E)) void k_lmp(LmArgs a)
{
    using B = LmpLds<N, E, LINES, MODE, LT>;
    __shared__ LT lds[LmTile<N, E, LINES>::LDS];
    __shared__ double2 twl[B::TW ? N : 1];
    __shared__ double2 kpl[MODE == LM_KIN && B::TB ? N : 1];
    __shared__ double k2l[MODE == LM_KERN && B::TB ? N : 1];
    __shared__ double sh[LmTile<N, E, LINES>::NT / 64 + 1];
    const auto src = lm_order<LINES>(Src1<LmArgs>{a, a.s0.ntiles + a.s1.ntiles});
    lmp_body<N, E, LINES, MODE, LT, decltype(src), B::TW, B::TB>(src, lds, B::TW ? twl : a.tw,
                                                                   B::TB ? kpl : a.kinp, B::TB ? k2l : a.k2_p, sh);
}

// Two-butterfly persistent LM pass (16 points per thread, 8-point plan): up
// to four waves per SIMD, so two 512-thread blocks share a CU.
template <int N, int LINES, int MODE>
__global__ __launch_bounds__(LINES *(N / 16), 4) void k_lmp2(LmArgs a)
{
    __shared__ float2 lds[LmTile<N, 16, LINES>::LDS];
    __shared__ double2 twl[R8<N>::TWN];
    __shared__ double2 kpl[MODE == LM_KIN ? N : 1];
    __shared__ double k2l[MODE == LM_KERN ? N : 1];
    __shared__ double sh[LmTile<N, 16, LINES>::NT / 64 + 1];
    const auto src = lm_order<LINES>(Src1<LmArgs>{a, a.s0.ntiles + a.s1.ntiles});
    lmp2_body<N, LINES, MODE>(src, lds, twl, kpl, k2l, sh);
}

template <int N, int E, int LINES, int S>
__global__ __launch_bounds__(LINES *(N / E)) void k_em_fft_g(const EmArgs *__restrict__ args, int tpi)
{
    __shared__ float2 lds[EmTile<N, E, LINES>::LDS];
    const EmArgs a = args[blockIdx.x / tpi];
    em_fft_tile<N, E, LINES, S>(a, blockIdx.x % tpi, lds);
}
template <int N, int E, int LINES, bool STORE_PSI>
__global__ __launch_bounds__(LINES *(N / E)) void k_density_g(const EmArgs *__restrict__ args, int tpi)
{
    __shared__ float2 lds[EmTile<N, E, LINES>::LDS];
    __shared__ double sh[EmTile<N, E, LINES>::NT / 64 + 1];
    const EmArgs a = args[blockIdx.x / tpi];
    density_tile<N, E, LINES, STORE_PSI>(a, blockIdx.x % tpi, lds, sh);
}
template <int N, int E, int LINES, bool REAL_IN>
__global__ __launch_bounds__(LINES *(N / E)) void k_phase_g(const EmArgs *__restrict__ args, int tpi)
{
    __shared__ float2 lds[EmTile<N, E, LINES>::LDS];
    __shared__ double sh[EmTile<N, E, LINES>::NT / 64 + 1];
    const EmArgs a = args[blockIdx.x / tpi];
    phase_tile<N, E, LINES, false, REAL_IN>(a, blockIdx.x % tpi, lds, sh);
}
template <int N, int E, int LINES, int MODE>
__global__ __launch_bounds__(LINES *(N / E)) void k_lm_g(const LmArgs *__restrict__ args, int tpi)
{
    __shared__ float2 lds[LmTile<N, E, LINES>::LDS];
    __shared__ double sh[LmTile<N, E, LINES>::NT / 64 + 1];
    const LmArgs a = args[blockIdx.x / tpi];
    lm_tile<N, E, LINES, MODE>(a, blockIdx.x % tpi, lds, sh);
}

// Grouped persistent prefetching passes: blocks walk the tiles of every
// instance of the group (instance-major numbering, tpi tiles per instance).
template <int N, int E, int LINES, int MODE>
__global__ __launch_bounds__(LINES *(N / E)) void k_lmp_g(const LmArgs *__restrict__ args, int tpi, int count)
{
    using B = LmpLds<N, E, LINES, MODE, float2>;
    __shared__ float2 lds[LmTile<N, E, LINES>::LDS];
    __shared__ double2 twl[B::TW ? N : 1];
    __shared__ double2 kpl[MODE == LM_KIN && B::TB ? N : 1];
    __shared__ double k2l[MODE == LM_KERN && B::TB ? N : 1];
    __shared__ double sh[LmTile<N, E, LINES>::NT / 64 + 1];
    const auto src = lm_order<LINES>(SrcG<LmArgs>{args, tpi, count});
    const LmArgs &a0 = src.args(0);
    lmp_body<N, E, LINES, MODE, float2, decltype(src), B::TW, B::TB>(src, lds, B::TW ? twl : a0.tw,
                                                                      B::TB ? kpl : a0.kinp, B::TB ? k2l : a0.k2_p, sh);
}
template <int N, int E, int LINES, bool STORE_PSI>
__global__ __launch_bounds__(LINES *(N / E)) void k_densityp_g(const EmArgs *__restrict__ args, int tpi, int count)
{
    __shared__ float2 lds[EmTile<N, E, LINES>::LDS];
    __shared__ double2 twl[N];
    __shared__ double sh[EmTile<N, E, LINES>::NT / 64 + 1];
    const SrcG<EmArgs> src{args, tpi, count};
    densityp_body<N, E, LINES, STORE_PSI, float2>(src, lds, twl, sh);
}
template <int N, int E, int LINES, bool REAL_IN>
__global__ __launch_bounds__(LINES *(N / E)) void k_phasep_g(const EmArgs *__restrict__ args, int tpi, int count)
{
    __shared__ float2 lds[EmTile<N, E, LINES>::LDS];
    __shared__ double2 twl[N];
    __shared__ double2 sct[kSinCosTable];
    const SrcG<EmArgs> src{args, tpi, count};
    phasep_body<N, E, LINES, REAL_IN, float2>(src, lds, twl, sct);
}

// ---------------------------------------------------------------- small kernels
template <int NT, class ST = float2>
__global__ __launch_bounds__(NT) void k_mass(const ST *__restrict__ psi, long long P, double *partials)
{
    __shared__ double sh[NT / 64 + 1];
    double s = 0.0;
    for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < P; i += (long long)gridDim.x * NT) {
        const dc v = ld_c(psi[i]);
        s += v.x * v.x + v.y * v.y;
    }
    s = block_sum<NT>(s, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// dst = src * exp(i theta) in FP64, to complex64 or complex128
template <bool C128, class ST = float2>
__global__ void k_readout(const ST *__restrict__ src, void *dst, long long P, const DevState *st)
{
    double s, c;
    sincos(st->theta, &s, &c);
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < P;
         i += (long long)gridDim.x * blockDim.x) {
        const dc v = ld_c(src[i]);
        const double re = c * v.x - s * v.y, im = s * v.x + c * v.y;
        if constexpr (C128) ((double2 *)dst)[i] = make_double2(re, im);
        else ((float2 *)dst)[i] = make_float2((float)re, (float)im);
    }
}

// complex64 input into a complex128-storage grid
static __global__ void k_from_c64(const float2 *__restrict__ src, double2 *dst, long long P)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < P;
         i += (long long)gridDim.x * blockDim.x) {
        const float2 v = src[i];
        dst[i] = make_double2((double)v.x, (double)v.y);
    }
}

static __global__ void k_from_c128(const double2 *__restrict__ src, float2 *dst, long long P)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < P;
         i += (long long)gridDim.x * blockDim.x) {
        const double2 v = src[i];
        dst[i] = make_float2((float)v.x, (float)v.y);
    }
}

// Relative difference of two states including their global phases:
// part[2b] = sum |a e^{i th_a} - b e^{i th_b}|^2, part[2b+1] = sum |b|^2.
static __global__ void k_state_diff(const float2 *__restrict__ a, const DevState *sa, const float2 *__restrict__ b,
                                    const DevState *sb, long long P, double *part)
{
    __shared__ double sh[5];
    double ca, sa_, cb, sb_;
    sincos(sa->theta, &sa_, &ca);
    sincos(sb->theta, &sb_, &cb);
    double d = 0.0, n = 0.0;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < P; i += (long long)gridDim.x * 256) {
        const float2 u = a[i], v = b[i];
        const double ur = ca * u.x - sa_ * u.y, ui = sa_ * u.x + ca * u.y;
        const double vr = cb * v.x - sb_ * v.y, vi = sb_ * v.x + cb * v.y;
        d += (ur - vr) * (ur - vr) + (ui - vi) * (ui - vi);
        n += vr * vr + vi * vi;
    }
    d = block_sum<256>(d, sh);
    n = block_sum<256>(n, sh);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = d;
        part[2 * blockIdx.x + 1] = n;
    }
}

static __global__ void k_reset_state(DevState *st)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->theta = 0.0;
        st->mass_sum = 0.0;
        st->steps = 0;
        st->nonfinite = 0;
        st->pad = 0;
    }
}

}  // namespace gsn
