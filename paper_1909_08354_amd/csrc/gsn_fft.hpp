// gsn_fft.hpp -- device FFT building blocks for gfx950.
//
// A line of N complex points is owned by TPL = N/E threads; thread t holds the
// E points at positions t + TPL*e (e = 0..E-1) in FP64 registers.  The
// transform is a Stockham (self-sorting) mixed-radix DFT: stage s with radix R
// takes butterfly j (t + TPL*m) from positions j + r*N/R, multiplies by the
// twiddles exp(+-2 pi i (j mod Ns) r / (Ns R)), does a length-R DFT in
// registers and sends the outputs to positions expand(j) + r*Ns, with
// expand(j) = (j / Ns) Ns R + (j mod Ns).  Between stages the data goes
// through LDS (complex64 or complex128 slots); the last stage's outputs land in the same
// registers in natural order (position t + TPL*e holds bin t + TPL*e), so a
// pointwise multiplier and an inverse transform can follow without another
// exchange.  Transforms are unnormalised in both directions.
#pragma once
#include <hip/hip_runtime.h>

namespace gsn {

struct dc { double x, y; };

__device__ __forceinline__ dc mk(double x, double y) { dc r; r.x = x; r.y = y; return r; }
__device__ __forceinline__ dc add(dc a, dc b) { return mk(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ dc sub(dc a, dc b) { return mk(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ dc scl(dc a, double s) { return mk(a.x * s, a.y * s); }
__device__ __forceinline__ dc conj(dc a) { return mk(a.x, -a.y); }
__device__ __forceinline__ dc cmul(dc a, dc b)
{
    return mk(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ double norm2(dc a) { return fma(a.x, a.x, a.y * a.y); }
__device__ __forceinline__ dc from_f2(float2 v) { return mk((double)v.x, (double)v.y); }
__device__ __forceinline__ float2 to_f2(dc v) { return make_float2((float)v.x, (float)v.y); }
__device__ __forceinline__ dc from_d2(double2 v) { return mk(v.x, v.y); }

// LDS exchange slots: complex64 (half the LDS footprint) or complex128 (no
// conversions, no intermediate rounding)
__device__ __forceinline__ void lds_put(float2 *p, int i, dc v) { p[i] = to_f2(v); }
__device__ __forceinline__ void lds_put(double2 *p, int i, dc v) { p[i] = make_double2(v.x, v.y); }
__device__ __forceinline__ dc lds_get(const float2 *p, int i) { return from_f2(p[i]); }
__device__ __forceinline__ dc lds_get(const double2 *p, int i) { return from_d2(p[i]); }

// multiply by S*i (S = -1 forward, +1 inverse)
template <int S> __device__ __forceinline__ dc mul_si(dc a)
{
    if constexpr (S > 0) return mk(-a.y, a.x);
    else return mk(a.y, -a.x);
}

// cos and sin of 2 pi m / 16 (exact mathematical constants)
constexpr double kC1 = 0.92387953251128675613;  // cos(pi/8)
constexpr double kS1 = 0.38268343236508977173;  // sin(pi/8)
constexpr double kR2 = 0.70710678118654752440;  // sqrt(1/2)

// a * exp(S 2 pi i m / 16) for a compile-time m in [0, 16)
template <int S, int M> __device__ __forceinline__ dc tw16(dc a)
{
    constexpr int m = M & 15;
    if constexpr (m == 0) return a;
    else if constexpr (m == 4) return mul_si<S>(a);
    else if constexpr (m == 8) return mk(-a.x, -a.y);
    else if constexpr (m == 12) return mul_si<-S>(a);
    else if constexpr (m == 2 || m == 6 || m == 10 || m == 14) {
        // (cx, S*sy) with |cx| = |sy| = sqrt(1/2)
        constexpr double cx = (m == 2 || m == 14) ? kR2 : -kR2;
        constexpr double sy = (m == 2 || m == 6) ? kR2 : -kR2;
        constexpr double ss = S > 0 ? sy : -sy;
        return mk(cx * a.x - ss * a.y, cx * a.y + ss * a.x);
    } else {
        constexpr double c = (m == 1 || m == 15) ? kC1 : (m == 3 || m == 13) ? kS1
                           : (m == 5 || m == 11) ? -kS1 : -kC1;
        constexpr double s0 = (m == 1 || m == 7) ? kS1 : (m == 3 || m == 5) ? kC1
                            : (m == 9 || m == 15) ? -kS1 : -kC1;
        constexpr double s = S > 0 ? s0 : -s0;
        return mk(fma(c, a.x, -s * a.y), fma(c, a.y, s * a.x));
    }
}

template <int S> __device__ __forceinline__ void dft2(dc *a)
{
    dc t = a[0];
    a[0] = add(t, a[1]);
    a[1] = sub(t, a[1]);
}

template <int S> __device__ __forceinline__ void dft4(dc &a0, dc &a1, dc &a2, dc &a3)
{
    dc s02 = add(a0, a2), d02 = sub(a0, a2);
    dc s13 = add(a1, a3), d13 = mul_si<S>(sub(a1, a3));
    a0 = add(s02, s13);
    a2 = sub(s02, s13);
    a1 = add(d02, d13);
    a3 = sub(d02, d13);
}

template <int S> __device__ __forceinline__ void dft4(dc *a) { dft4<S>(a[0], a[1], a[2], a[3]); }

// length-8 DFT: even/odd split into two length-4 DFTs
template <int S> __device__ __forceinline__ void dft8(dc *a)
{
    dc e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6];
    dc o0 = a[1], o1 = a[3], o2 = a[5], o3 = a[7];
    dft4<S>(e0, e1, e2, e3);
    dft4<S>(o0, o1, o2, o3);
    o1 = tw16<S, 2>(o1);
    o2 = tw16<S, 4>(o2);
    o3 = tw16<S, 6>(o3);
    a[0] = add(e0, o0); a[4] = sub(e0, o0);
    a[1] = add(e1, o1); a[5] = sub(e1, o1);
    a[2] = add(e2, o2); a[6] = sub(e2, o2);
    a[3] = add(e3, o3); a[7] = sub(e3, o3);
}

// length-16 DFT as 4 x 4: Y_q = DFT4(a_q, a_{q+4}, a_{q+8}, a_{q+12}),
// Y_q[k] *= w16^{q k}, X_{k + 4 j} = DFT4_q(Y_q[k])[j]
template <int S> __device__ __forceinline__ void dft16(dc *a)
{
    dc y[16];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        dc b0 = a[q], b1 = a[q + 4], b2 = a[q + 8], b3 = a[q + 12];
        dft4<S>(b0, b1, b2, b3);
        y[q * 4 + 0] = b0; y[q * 4 + 1] = b1; y[q * 4 + 2] = b2; y[q * 4 + 3] = b3;
    }
    // twiddles w16^{q k}
    y[1 * 4 + 1] = tw16<S, 1>(y[5]);
    y[1 * 4 + 2] = tw16<S, 2>(y[6]);
    y[1 * 4 + 3] = tw16<S, 3>(y[7]);
    y[2 * 4 + 1] = tw16<S, 2>(y[9]);
    y[2 * 4 + 2] = tw16<S, 4>(y[10]);
    y[2 * 4 + 3] = tw16<S, 6>(y[11]);
    y[3 * 4 + 1] = tw16<S, 3>(y[13]);
    y[3 * 4 + 2] = tw16<S, 6>(y[14]);
    y[3 * 4 + 3] = tw16<S, 9>(y[15]);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        dc b0 = y[k], b1 = y[4 + k], b2 = y[8 + k], b3 = y[12 + k];
        dft4<S>(b0, b1, b2, b3);
        a[k] = b0; a[k + 4] = b1; a[k + 8] = b2; a[k + 12] = b3;
    }
}

template <int R, int S> __device__ __forceinline__ void dft(dc *a)
{
    if constexpr (R == 2) dft2<S>(a);
    else if constexpr (R == 4) dft4<S>(a);
    else if constexpr (R == 8) dft8<S>(a);
    else if constexpr (R == 16) dft16<S>(a);
    else static_assert(R == 1, "unsupported radix");
}

// Stage plan: ceil(log_E N) stages, the first of radix N / E^(stages - 1)
// (the smallest), the others of radix E.  The short radix goes first because
// a short last stage, combining two halves that were just rounded to
// complex64 in the LDS exchange, biases the norm over long runs: 2000 steps
// of the 8-lump 512^3 state drift by -2.8e-6 with radices 16,16,2 and by
// -6.5e-8 with 2,16,16; 2000 steps at 128^3 by -8.8e-7 with 8,8,2 and by
// 3.8e-8 with 2,8,8.
template <int N, int E> struct Plan {
    static_assert(N >= E && N % E == 0, "E must divide N");
    static constexpr int TPL = N / E;
    static constexpr int nstages()
    {
        int s = 0;
        long p = 1;
        while (p < N) { p *= E; ++s; }
        return s;
    }
    static constexpr int radix(int s)
    {
        if (s > 0) return E;
        int r = N;
        for (int i = 1; i < nstages(); ++i) r /= E;
        return r;
    }
    static constexpr int ns(int s)
    {
        int p = 1;
        for (int i = 0; i < s; ++i) p *= radix(i);
        return p;
    }
};

// LDS addressing of one line.  Element-major lines (contiguous axis): one pad
// per 16 points plus a line pitch of 16 (mod 32) float2.  Line-major tiles
// (strided axes): position-major with the LINES lines of a tile adjacent.
// Synchronisation of an LDS exchange: a block barrier, or (when every line of
// the tile lives inside one wavefront) a wavefront-scope fence plus a wave
// barrier, which orders the wave's own LDS writes before its reads.
template <bool WAVE> __device__ __forceinline__ void exchange_sync()
{
    if constexpr (WAVE) {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    } else {
        __syncthreads();
    }
}

template <int N, int E = 16> struct EmLayout {
    // one pad slot per E points: the first-stage writes (E consecutive
    // positions per lane) then hit distinct banks across a wavefront
    static constexpr int PAD_SHIFT = E >= 16 ? 4 : E == 8 ? 3 : E == 4 ? 2 : 1;
    static constexpr int S0 = N + (N >> PAD_SHIFT);
    static constexpr int PITCH = (S0 % 32 == 0) ? S0 + 16 : S0;
    static constexpr int BYTES_PER_LINE = PITCH * 8;
    static constexpr bool WAVE_LOCAL = (N / E) <= 64;   // a row within one wavefront
    int base;
    __device__ __forceinline__ int operator()(int pos) const { return base + pos + (pos >> PAD_SHIFT); }
};
template <int LINES> struct LmLayout {
    static constexpr bool WAVE_LOCAL = false;
    int l;
    __device__ __forceinline__ int operator()(int pos) const { return pos * LINES + l; }
};

// One Stockham stage and the recursion over the remaining stages.
template <int N, int E, int S, int ST, class Lay, class LT>
__device__ __forceinline__ void fft_stages(dc (&v)[E], int t, const Lay &lay, LT *lds,
                                           const double2 *__restrict__ tw)
{
    using P = Plan<N, E>;
    if constexpr (ST < P::nstages()) {
        constexpr int R = P::radix(ST);
        constexpr int NS = P::ns(ST);
        constexpr bool LAST = (ST + 1 == P::nstages());
        constexpr int B = E / R;
        constexpr int TPL = P::TPL;
#pragma unroll
        for (int m = 0; m < B; ++m) {
            const int j = t + TPL * m;
            dc a[R];
#pragma unroll
            for (int r = 0; r < R; ++r) a[r] = v[m + r * B];
            if constexpr (NS > 1) {
                const int jm = j & (NS - 1);
                constexpr int STEP = N / (NS * R);
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    dc w = from_d2(tw[jm * r * STEP]);
                    if constexpr (S > 0) w.y = -w.y;
                    a[r] = cmul(a[r], w);
                }
            }
            dft<R, S>(a);
            if constexpr (LAST) {
#pragma unroll
                for (int r = 0; r < R; ++r) v[m + r * B] = a[r];
            } else {
                const int base = (j / NS) * NS * R + (j & (NS - 1));
#pragma unroll
                for (int r = 0; r < R; ++r) lds_put(lds, lay(base + r * NS), a[r]);
            }
        }
        if constexpr (!LAST) {
            exchange_sync<Lay::WAVE_LOCAL>();
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] = lds_get(lds, lay(t + TPL * e));
            exchange_sync<Lay::WAVE_LOCAL>();
            fft_stages<N, E, S, ST + 1>(v, t, lay, lds, tw);
        }
    }
}

// Unnormalised DFT of the line held in v (S = -1 forward, +1 inverse).
// tw[q] = exp(-2 pi i q / N), q < N, FP64 (global or LDS).  Every thread of the block must
// call this (it contains barriers when the plan has more than one stage).
template <int N, int E, int S, class Lay, class LT>
__device__ __forceinline__ void fft(dc (&v)[E], int t, const Lay &lay, LT *lds,
                                    const double2 *__restrict__ tw)
{
    fft_stages<N, E, S, 0>(v, t, lay, lds, tw);
}

// Deterministic FP64 block sum (result valid in thread 0).
template <int NT> __device__ __forceinline__ double block_sum(double v, double *sh)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int tid = threadIdx.x;
    if constexpr (NT > 64) {
        if ((tid & 63) == 0) sh[tid >> 6] = v;
        __syncthreads();
        if (tid == 0) {
            double s = 0.0;
#pragma unroll
            for (int w = 0; w < NT / 64; ++w) s += sh[w];
            v = s;
        }
        __syncthreads();
    }
    return v;
}

}  // namespace gsn
