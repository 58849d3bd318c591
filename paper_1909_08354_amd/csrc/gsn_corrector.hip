// gsn_corrector.hip -- learned corrector for coarse split steps on gfx950.
//
// A 4-layer 3x3 convolutional network (3 -> 32 -> 32 -> 32 -> 2 channels,
// ReLU after the first three, circular padding) reads (Re psi_c, Im psi_c,
// phi_c) of a coarse step and predicts the residual to the fine result.
// Activations and weights are bfloat16, every product accumulates in FP32 on
// the matrix cores (v_mfma_f32_16x16x16_bf16), the master weights and Adam
// moments are FP32.  Convolutions are implicit GEMMs over NHWC images:
//   forward        M = pixels, N = Cout, K = 9 * Cin   (A: input, B: weights)
//   backward data  M = pixels, N = Cin,  K = 9 * Cout  (A: dZ,    B: weights^T)
//   backward wts   M = Cout,   N = Cin,  K = pixels    (A: dZ^T,  B: input^T)
// MFMA 16x16x16 operand layout (64 lanes, l = lane): A[i = l%16][k = 4(l/16)+0..3],
// B[k = 4(l/16)+0..3][j = l%16], D[i = 4(l/16)+0..3][j = l%16].
// Weight gradients are reduced from per-block partials in a fixed order, so
// training is bitwise deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <type_traits>
#include <vector>

#include "gsn_host.hpp"
#include "gsn_corrector_internal.hpp"

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16;

constexpr int kNParams = 19970;
constexpr int kLayers = 4;
// per layer: real and padded channel counts
constexpr int kCin[kLayers] = {3, 32, 32, 32};
constexpr int kCout[kLayers] = {32, 32, 32, 2};
constexpr int kCinP[kLayers] = {4, 32, 32, 32};
constexpr int kCoutP[kLayers] = {32, 32, 32, 16};

__device__ inline u16 f2bf(float f)
{
    unsigned u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (u16)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (u16)(u >> 16);
}
__device__ inline float bf2f(u16 h) { return __uint_as_float(((unsigned)h) << 16); }

__device__ inline int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// (cos theta, sin theta) of a device FP64 phase (null: no rotation)
__device__ inline float2 phase_of(const double *theta)
{
    if (!theta) return make_float2(1.f, 0.f);
    double s, c;
    sincos_fp64(*theta, &s, &c);
    return make_float2((float)c, (float)s);
}
__device__ inline float2 rot(float2 v, float2 e) { return make_float2(v.x * e.x - v.y * e.y, v.x * e.y + v.y * e.x); }


// ---------------------------------------------------------------- forward conv
template <int CIN_P, int COUT_P, int COUT, bool RELU, bool OUT_F32>
__global__ __launch_bounds__(256) void k_conv_fwd(const u16 *__restrict__ X, const u16 *__restrict__ Wf,
                                                  const float *__restrict__ bias, void *__restrict__ Y,
                                                  int H, int W, long long npix)
{
    constexpr int KTOT = 9 * CIN_P, KCH = (KTOT + 15) / 16, NB = COUT_P / 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long long pix0 = ((long long)blockIdx.x * 4 + wave) * 16;
    if (pix0 >= npix) return;
    const long long HW = (long long)H * W;
    const long long pa = pix0 + (lane & 15);
    const long long img = pa / HW;
    const int rem = (int)(pa - img * HW), y = rem / W, x = rem - (rem / W) * W;
    const int kq = 4 * (lane >> 4);
    f32x4 acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[nb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
    for (int kc = 0; kc < KCH; ++kc) {
        const int k = kc * 16 + kq;
        const int tap = k / CIN_P, c0 = k - tap * CIN_P;
        bf16x4 av = {0, 0, 0, 0};
        if (tap < 9) {
            const int ys = wrap(y + tap / 3 - 1, H), xs = wrap(x + tap % 3 - 1, W);
            av = *(const bf16x4 *)(X + ((img * H + ys) * W + xs) * CIN_P + c0);
        }
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            bf16x4 bv = {0, 0, 0, 0};
            if (tap < 9) bv = *(const bf16x4 *)(Wf + ((long long)tap * COUT_P + nb * 16 + (lane & 15)) * CIN_P + c0);
            acc[nb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[nb], 0, 0, 0);
        }
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        const int ch = nb * 16 + (lane & 15);
        const float bch = bias[ch];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const long long p = pix0 + 4 * (lane >> 4) + r;
            float v = acc[nb][r] + bch;
            if (RELU) v = v > 0.f ? v : 0.f;
            if constexpr (OUT_F32) {
                if (ch < COUT) ((float *)Y)[p * COUT + ch] = v;
            } else {
                ((u16 *)Y)[p * COUT_P + ch] = f2bf(v);
            }
        }
    }
}

// ---------------------------------------------------------------- forward conv, LDS-tiled
// Layers with 32 input channels on images whose width is a multiple of 64
// and height a multiple of 4 (the 512^2 workload).  A block owns 4 rows x 64
// pixels; the 6 x 66 input halo (circular) is staged once in LDS, each wave
// computes one row (4 M-tiles of 16 pixels) against all output channels with
// v_mfma_f32_16x16x32_bf16 (one K chunk = the 32 channels of one tap), the
// weights live in registers for the block's lifetime (persistent blocks walk
// the tiles), and outputs go back through LDS so each lane stores 16 bytes.
// 16x16x32 operands (l = lane): A[i = l%16][k = 8(l/16)+0..7],
// B[k = 8(l/16)+0..7][j = l%16], D[i = 4(l/16)+0..3][j = l%16].
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned u32x4v __attribute__((ext_vector_type(4)));

constexpr int kTH = 4, kTW = 64;              // output tile
constexpr int kHP = kTH + 2, kWP = kTW + 2;   // staged input tile (halo 1)

// APPLY (last layer, inference): instead of storing the two FP32 outputs,
// write psi_o = psi_c + s (out0 + i out1) for the tile's pixels.
template <int COUT_P, int COUT, bool RELU, bool OUT_F32, bool APPLY = false>
__global__ __launch_bounds__(256) void k_conv_fwd_t(const u16 *__restrict__ X, const u16 *__restrict__ Wf,
                                                    const float *__restrict__ bias, void *__restrict__ Y,
                                                    int H, int W, int ntiles, const float2 *__restrict__ psi_c,
                                                    float2 *__restrict__ psi_o, float s_out, const double *theta)
{
    static_assert(!APPLY || (OUT_F32 && COUT == 2), "apply needs the two-channel FP32 output");
    constexpr int NB = COUT_P / 16;
    constexpr int OUT_B = OUT_F32 ? 4 * COUT : 2 * COUT_P;   // output bytes per pixel
    __shared__ u32x4v xin[kHP * kWP * 4];                      // 16-byte quarters of 64-byte pixels
    __shared__ u32x4v yst[4][kTW * OUT_B / 16];                // per-wave output staging
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int i16 = lane & 15, q = lane >> 4;
    // weights: B fragments of all 9 taps and NB column blocks
    bf16x8 wb[9][NB];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
            wb[t][nb] = *(const bf16x8 *)(Wf + ((long long)(t * COUT_P + nb * 16 + i16)) * 32 + 8 * q);
    float bch[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) bch[nb] = bias[nb * 16 + i16];
    const int tx = W / kTW, ty = H / kTH;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int img = tile / (tx * ty), r0 = tile - img * tx * ty;
        const int y0 = (r0 / tx) * kTH, x0 = (r0 % tx) * kTW;
        const u16 *Xi = X + (long long)img * H * W * 32;
        __syncthreads();   // the previous tile's readers are done with xin
        for (int c = tid; c < kHP * kWP * 4; c += 256) {
            const int pq = c & 3, pix = c >> 2, rr = pix / kWP, cc = pix - rr * kWP;
            int ys = y0 + rr - 1, xs = x0 + cc - 1;
            ys = ys < 0 ? ys + H : (ys >= H ? ys - H : ys);
            xs = xs < 0 ? xs + W : (xs >= W ? xs - W : xs);
            xin[c] = *(const u32x4v *)(Xi + ((long long)ys * W + xs) * 32 + pq * 8);
        }
        __syncthreads();
        f32x4 acc[4][NB];
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) acc[m][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int dy = t / 3, dx = t % 3;
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const u32x4v raw = xin[((wave + dy) * kWP + m * 16 + i16 + dx) * 4 + q];
                const bf16x8 av = __builtin_bit_cast(bf16x8, raw);
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    acc[m][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, wb[t][nb], acc[m][nb], 0, 0, 0);
            }
        }
        // bias, ReLU, convert, stage this wave's row in LDS
        u16 *ys16 = (u16 *)yst[wave];
        float *ysf = (float *)yst[wave];
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int px = m * 16 + 4 * q + r, ch = nb * 16 + i16;
                    float v = acc[m][nb][r] + bch[nb];
                    if (RELU) v = v > 0.f ? v : 0.f;
                    if constexpr (OUT_F32) {
                        if (ch < COUT) ysf[px * COUT + ch] = v;
                    } else {
                        ys16[px * COUT_P + ch] = f2bf(v);
                    }
                }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        // row (y0 + wave), pixels x0 .. x0 + 63: contiguous OUT_B * 64 bytes
        const long long p0 = ((long long)img * H + y0 + wave) * W + x0;
        if constexpr (APPLY) {
            const float2 e = phase_of(theta);
            const long long p = p0 + lane;
            const float2 c = psi_c[p];
            const float2 r = rot(make_float2(ysf[2 * lane], ysf[2 * lane + 1]), make_float2(e.x, -e.y));
            psi_o[p] = make_float2(c.x + s_out * r.x, c.y + s_out * r.y);
        } else {
            char *yrow = (char *)Y + p0 * OUT_B;
#pragma unroll
            for (int c = lane; c < kTW * OUT_B / 16; c += 64) ((u32x4v *)yrow)[c] = yst[wave][c];
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

// First layer (3 input channels padded to 4) in the same tiling.  K = 9 taps
// x 4 channels = 36 in two 16x16x32 chunks: taps 0-7, then tap 8 and zeros;
// lane (i, q) of a chunk holds taps 2q and 2q + 1 (4 channels each, 8 bytes
// apiece in LDS).  FROM_PSI (inference): the halo is built from
// (Re u, Im u, phi) times the input scales, u = e^{i theta} psi, instead of
// the packed image.
template <bool FROM_PSI>
__global__ __launch_bounds__(256) void k_conv1_t(const u16 *__restrict__ X, const float2 *__restrict__ psi,
                                                 const float *__restrict__ phi, float s0, float s1, float s2,
                                                 const u16 *__restrict__ Wf, const float *__restrict__ bias,
                                                 u16 *__restrict__ Y, int H, int W, int ntiles, const double *theta)
{
    typedef unsigned u32x2v __attribute__((ext_vector_type(2)));
    __shared__ u32x2v xin[kHP * kWP];           // 4 bf16 per pixel
    __shared__ u32x4v yst[4][kTW * 64 / 16];    // per-wave output staging, 64 bytes per pixel
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int i16 = lane & 15, q = lane >> 4;
    const u32x2v zero2 = {0u, 0u};
    bf16x8 wb[2][2];
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
        const int co = nb * 16 + i16;
        const u32x2v lo = *(const u32x2v *)(Wf + ((2 * q) * 32 + co) * 4);
        const u32x2v hi = *(const u32x2v *)(Wf + ((2 * q + 1) * 32 + co) * 4);
        wb[0][nb] = __builtin_bit_cast(bf16x8, u32x4v{lo.x, lo.y, hi.x, hi.y});
        const u32x2v l8 = q == 0 ? *(const u32x2v *)(Wf + (8 * 32 + co) * 4) : zero2;
        wb[1][nb] = __builtin_bit_cast(bf16x8, u32x4v{l8.x, l8.y, 0u, 0u});
    }
    const float bch[2] = {bias[i16], bias[16 + i16]};
    const float2 e = FROM_PSI ? phase_of(theta) : make_float2(1.f, 0.f);
    const int tx = W / kTW, ty = H / kTH;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int img = tile / (tx * ty), r0 = tile - img * tx * ty;
        const int y0 = (r0 / tx) * kTH, x0 = (r0 % tx) * kTW;
        const long long ib = (long long)img * H * W;
        __syncthreads();   // the previous tile's readers are done with xin
        for (int c = tid; c < kHP * kWP; c += 256) {
            const int rr = c / kWP, cc = c - rr * kWP;
            int ys = y0 + rr - 1, xs = x0 + cc - 1;
            ys = ys < 0 ? ys + H : (ys >= H ? ys - H : ys);
            xs = xs < 0 ? xs + W : (xs >= W ? xs - W : xs);
            const long long pix = ib + (long long)ys * W + xs;
            if constexpr (FROM_PSI) {
                const float2 v = rot(psi[pix], e);
                const float f = phi[pix];
                xin[c] = u32x2v{(unsigned)f2bf(v.x * s0) | ((unsigned)f2bf(v.y * s1) << 16), (unsigned)f2bf(f * s2)};
            } else {
                xin[c] = *(const u32x2v *)(X + pix * 4);
            }
        }
        __syncthreads();
        f32x4 acc[4][2];
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) acc[m][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
        const int t0 = 2 * q, t1 = 2 * q + 1;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int col = m * 16 + i16;
            const u32x2v a0 = xin[(wave + t0 / 3) * kWP + col + t0 % 3];
            const u32x2v a1 = xin[(wave + t1 / 3) * kWP + col + t1 % 3];
            const u32x2v a8 = q == 0 ? xin[(wave + 2) * kWP + col + 2] : zero2;
            const bf16x8 av0 = __builtin_bit_cast(bf16x8, u32x4v{a0.x, a0.y, a1.x, a1.y});
            const bf16x8 av1 = __builtin_bit_cast(bf16x8, u32x4v{a8.x, a8.y, 0u, 0u});
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) {
                acc[m][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av0, wb[0][nb], acc[m][nb], 0, 0, 0);
                acc[m][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av1, wb[1][nb], acc[m][nb], 0, 0, 0);
            }
        }
        u16 *ys16 = (u16 *)yst[wave];
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float v = acc[m][nb][r] + bch[nb];
                    ys16[(m * 16 + 4 * q + r) * 32 + nb * 16 + i16] = f2bf(v > 0.f ? v : 0.f);
                }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        char *yrow = (char *)Y + ((ib + (long long)(y0 + wave) * W + x0) * 64);
#pragma unroll
        for (int c = lane; c < kTW * 64 / 16; c += 64) ((u32x4v *)yrow)[c] = yst[wave][c];
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

// ---------------------------------------------------------------- fused inference
// The four layers of one corrected step in one kernel.  A block owns a
// segment of S output tiles (4 x 64 pixels each) stacked down one 64-column
// strip and walks it top to bottom.  Each layer keeps its last six rows in
// an LDS ring, so a step of 4 output rows computes 4 new rows per layer and
// reuses the two rows it shares with the step above.  With rows counted from
// the segment's first row, a warm-up fills the rings (features -4 .. 3,
// layer 1 -3 .. 2, layer 2 -2 .. 1, layer 3 -1 .. 0); step k then adds
// feature rows 4k+4 .. 4k+7, layer-1 rows 4k+3 .. 4k+6, layer-2 rows
// 4k+2 .. 4k+5 and layer-3 rows 4k+1 .. 4k+4, and writes output rows
// 4k .. 4k+3.  HBM sees (psi, phi) in and psi out: about 20 bytes per pixel
// instead of 4 layers' NHWC round trips.  Per pixel the arithmetic is that
// of k_conv1_t / k_conv_fwd_t / the last layer's APPLY (same MFMA sequence,
// same bf16 roundings), so results equal the layer-by-layer path.  The
// output goes to psi_out (other blocks still read psi for their halos).
// Columns relative to the strip origin x0: features -4 .. 79, layer l
// -(4 - l) .. 75 + (4 - l) (5 M-tiles of 16 per row).  A 3 x 3 window at the
// right edge of a row reads two pixels of the next ring row (of the next
// buffer after the last one); the columns past 67 - l it reaches feed only
// outputs that are never used, and ring rows not yet written feed only rows
// that are rewritten before they are read.  Activation pixels are 80 bytes
// apart (64 bytes of channels and 16 of padding): the 16-byte operand reads
// of 8 consecutive pixels hit 8 different bank groups, and the taps of one
// window row are fixed offsets from one address.  The weights sit in LDS for
// the block's lifetime (the last layer's only for its two live output
// channels), each wave runs two M-tiles at a time, and the next step's
// feature rows are loaded into registers while the current step computes.
constexpr int kFusedThreads = 512;
constexpr int kRing = 6, kFRing = 8;                 // activation / feature rows kept
constexpr int kFCols = kTW + 20;                     // 84 feature columns
constexpr int kACols = kTW + 16;                     // 80 activation columns
constexpr int kPixU = 5;                             // 16-byte units per activation pixel
constexpr int kMT = 5;                               // M-tiles per row, layers 1-3
constexpr int kRingU = kRing * kACols * kPixU;       // 16-byte units per activation ring
constexpr int kW1 = 9 * 32 * 4, kW23 = 9 * 32 * 32, kW4L = 9 * 2 * 32;   // bf16 weights in LDS per layer
constexpr int kFNew = 4 * kFCols;                    // feature pixels per step
constexpr int kLdsU = 3 * kRingU + (kW1 + 2 * kW23 + kW4L) / 8 + kFRing * kFCols / 2 + kTH * kTW / 2;
static_assert(kLdsU * 16 <= 163840, "fused inference LDS");
static_assert(kFNew <= kFusedThreads && kTH * kTW <= kFusedThreads, "one feature / output pixel per thread");

__device__ inline int wrapmod(int v, int n) { v %= n; return v < 0 ? v + n : v; }
// ring slots of row r (r >= -24)
__device__ inline int rslot(int r) { return (r + 4 * kRing) % kRing; }
__device__ inline int fslot(int r) { return (r + 3 * kFRing) & (kFRing - 1); }

// The weights' 64-byte rows (tap, output channel) in LDS: chunk c of row p
// sits at slot c ^ ((p >> 1) & 3), so the 16-byte reads of 16 consecutive
// rows spread over the LDS banks.
__device__ inline int w_slot(int p, int c) { return p * 4 + (c ^ ((p >> 1) & 3)); }
// 8-byte group g (channels 4g .. 4g + 3) of activation pixel p
__device__ inline int act_u2(int p, int g) { return p * (2 * kPixU) + g; }

// LDS barrier that leaves global loads in flight (the next step's prefetch)
__device__ inline void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// max(acc + b, 0) of 4 values to 4 bf16 (round to nearest even; the same
// rounding as f2bf), packed into 8 bytes
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
typedef float f32x2v __attribute__((ext_vector_type(2)));
__device__ inline uint2 relu_bf16x4(f32x4 acc, const float (&b)[4])
{
    const f32x2v lo = {fmaxf(acc[0] + b[0], 0.f), fmaxf(acc[1] + b[1], 0.f)};
    const f32x2v hi = {fmaxf(acc[2] + b[2], 0.f), fmaxf(acc[3] + b[3], 0.f)};
    return make_uint2(__builtin_bit_cast(unsigned, __builtin_convertvector(lo, bf16x2v)),
                      __builtin_bit_cast(unsigned, __builtin_convertvector(hi, bf16x2v)));
}

// Rows r0 .. r0 + NROWS - 1 of a hidden layer (32 -> 32, ReLU) from rows
// r0 - 1 .. r0 + NROWS of the input ring; two M-tiles (mt and mt + 8) per
// wave at a time.
template <int NROWS>
__device__ inline void ring_hidden(const u32x4v *__restrict__ in, uint2 *__restrict__ out, const u16 *Ws,
                                   const float *__restrict__ bias, int r0, int wave, int i16, int q)
{
    constexpr int NW = kFusedThreads / 64, NMT = NROWS * kMT;
    bf16x8 wb[9][2];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
            wb[t][nb] = __builtin_bit_cast(bf16x8, ((const u32x4v *)Ws)[w_slot(t * 32 + nb * 16 + i16, q)]);
    // D^T = W X^T: lane (i16, q) ends with pixel i16 of the M-tile and the 4
    // channels nb*16 + 4q .. +3, stored together as 8 bytes
    float bch[2][4];
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) bch[nb][rr] = bias[nb * 16 + 4 * q + rr];
    for (int mt0 = wave; mt0 < NMT; mt0 += 2 * NW) {
        const bool two = mt0 + NW < NMT;
        int ib[2][3], ob[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int mt = (u == 0 || two) ? mt0 + u * NW : mt0;
            const int rr = mt / kMT, px = (mt - rr * kMT) * 16 + i16, r = r0 + rr;
#pragma unroll
            for (int dy = 0; dy < 3; ++dy) ib[u][dy] = (rslot(r - 1 + dy) * kACols + px) * kPixU + q;
            ob[u] = rslot(r) * kACols + px;
        }
        f32x4 acc[2][2];
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) acc[u][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < 9; ++t) {
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const bf16x8 av = __builtin_bit_cast(bf16x8, in[ib[u][t / 3] + (t % 3) * kPixU]);
#pragma unroll
                for (int nb = 0; nb < 2; ++nb)
                    acc[u][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wb[t][nb], av, acc[u][nb], 0, 0, 0);
            }
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            if (u == 1 && !two) break;
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) out[act_u2(ob[u], nb * 4 + q)] = relu_bf16x4(acc[u][nb], bch[nb]);
        }
    }
}

__global__ __launch_bounds__(kFusedThreads) void k_corr_fused(
    const float2 *__restrict__ psi, const float *__restrict__ phi, float2 *__restrict__ psi_out, float s0, float s1,
    float s2, float s_out, const u16 *__restrict__ W1, const u16 *__restrict__ W2, const u16 *__restrict__ W3,
    const u16 *__restrict__ W4, const float *__restrict__ b1, const float *__restrict__ b2,
    const float *__restrict__ b3, const float *__restrict__ b4, int H, int W, int seg, int nseg, const double *theta)
{
    typedef unsigned u32x2v __attribute__((ext_vector_type(2)));
    // one LDS array: the three activation rings, the weights, the feature
    // ring (4 bf16 per pixel), the last layer's outputs
    __shared__ u32x4v lds[kLdsU];
    u32x4v *const ring1 = lds, *const ring2 = ring1 + kRingU, *const ring3 = ring2 + kRingU;
    u16 *const Ws1 = (u16 *)(ring3 + kRingU), *const Ws2 = Ws1 + kW1, *const Ws3 = Ws2 + kW23, *const Ws4 = Ws3 + kW23;
    u32x2v *const fin = (u32x2v *)(Ws4 + kW4L);
    float2 *const res = (float2 *)(fin + kFRing * kFCols);
    constexpr int NW = kFusedThreads / 64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int i16 = lane & 15, q = lane >> 4;
    const u32x2v zero2 = {0u, 0u};
    const float2 e = phase_of(theta);
    const int tx = W / kTW;
    for (int i = tid; i < kW1 / 8; i += kFusedThreads) ((u32x4v *)Ws1)[i] = ((const u32x4v *)W1)[i];
    for (int i = tid; i < kW23 / 8; i += kFusedThreads) {   // 64-byte rows (tap, output channel), swizzled
        ((u32x4v *)Ws2)[w_slot(i >> 2, i & 3)] = ((const u32x4v *)W2)[i];
        ((u32x4v *)Ws3)[w_slot(i >> 2, i & 3)] = ((const u32x4v *)W3)[i];
    }
    for (int i = tid; i < kW4L / 8; i += kFusedThreads)     // output channels 0 and 1 of each tap
        ((u32x4v *)Ws4)[i] = ((const u32x4v *)W4)[((i >> 3) * 16 + ((i >> 2) & 1)) * 4 + (i & 3)];

    // feature rows ra .. ra + 3 of the segment at (Y0, x0): one pixel per
    // thread, fetched into registers, then rotated, scaled and stored
    float2 fp = make_float2(0.f, 0.f);
    float ff = 0.f;
    auto fetch = [&](int Y0, int x0, int ra) {
        if (tid < kFNew) {
            const int rr = tid / kFCols, cc = tid - rr * kFCols;
            const long long pix = (long long)wrapmod(Y0 + ra + rr, H) * W + wrapmod(x0 - 4 + cc, W);
            fp = psi[pix];
            ff = phi[pix];
        }
    };
    auto stash = [&](int ra) {
        if (tid < kFNew) {
            const int rr = tid / kFCols, cc = tid - rr * kFCols;
            const float2 v = rot(fp, e);
            fin[fslot(ra + rr) * kFCols + cc] =
                u32x2v{(unsigned)f2bf(v.x * s0) | ((unsigned)f2bf(v.y * s1) << 16), (unsigned)f2bf(ff * s2)};
        }
    };
    // layer 1 (3 -> 32, ReLU), rows r0 .. r0 + nrows - 1: K = 9 taps x 4
    // channels in two chunks, taps 2q and 2q + 1 in the first, tap 8 (q = 0)
    // in the second; tap t reads feature row r - 1 + t / 3, column col + t % 3
    auto layer1 = [&](int r0, int nrows) {
        bf16x8 wb[2][2];
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
            const int co = nb * 16 + i16;
            const u32x2v lo = *(const u32x2v *)(Ws1 + ((2 * q) * 32 + co) * 4);
            const u32x2v hi = *(const u32x2v *)(Ws1 + ((2 * q + 1) * 32 + co) * 4);
            wb[0][nb] = __builtin_bit_cast(bf16x8, u32x4v{lo.x, lo.y, hi.x, hi.y});
            const u32x2v l8 = q == 0 ? *(const u32x2v *)(Ws1 + (8 * 32 + co) * 4) : zero2;
            wb[1][nb] = __builtin_bit_cast(bf16x8, u32x4v{l8.x, l8.y, 0u, 0u});
        }
        float bch[2][4];
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) bch[nb][rr] = b1[nb * 16 + 4 * q + rr];
        const int t0 = 2 * q, t1 = 2 * q + 1;
        uint2 *const out = (uint2 *)ring1;
        for (int mt = wave; mt < nrows * kMT; mt += NW) {
            const int rr = mt / kMT, col = (mt - rr * kMT) * 16 + i16, r = r0 + rr;
            const u32x2v a0 = fin[fslot(r - 1 + t0 / 3) * kFCols + col + t0 % 3];
            const u32x2v a1 = fin[fslot(r - 1 + t1 / 3) * kFCols + col + t1 % 3];
            const u32x2v a8 = q == 0 ? fin[fslot(r + 1) * kFCols + col + 2] : zero2;
            const bf16x8 av0 = __builtin_bit_cast(bf16x8, u32x4v{a0.x, a0.y, a1.x, a1.y});
            const bf16x8 av1 = __builtin_bit_cast(bf16x8, u32x4v{a8.x, a8.y, 0u, 0u});
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) {
                f32x4 acc = {0.f, 0.f, 0.f, 0.f};
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wb[0][nb], av0, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wb[1][nb], av1, acc, 0, 0, 0);
                out[act_u2(rslot(r) * kACols + col, nb * 4 + q)] = relu_bf16x4(acc, bch[nb]);
            }
        }
    };

    for (int sg = blockIdx.x; sg < nseg; sg += gridDim.x) {
        const int Y0 = (sg / tx) * seg * kTH, x0 = (sg % tx) * kTW;
        // warm-up
        fetch(Y0, x0, -4);
        stash(-4);
        fetch(Y0, x0, 0);
        stash(0);
        fetch(Y0, x0, 4);   // step 0's rows land while the warm-up computes
        lds_barrier();
        layer1(-3, 6);
        lds_barrier();
        ring_hidden<4>(ring1, (uint2 *)ring2, Ws2, b2, -2, wave, i16, q);
        lds_barrier();
        ring_hidden<2>(ring2, (uint2 *)ring3, Ws3, b3, -1, wave, i16, q);
        for (int k = 0; k < seg; ++k) {
            // the new feature rows overwrite rows that layer 1 has finished with
            stash(4 * k + 4);
            float2 pc = make_float2(0.f, 0.f);   // psi at this thread's output pixel
            if (tid < kTH * kTW) pc = psi[(long long)(Y0 + 4 * k + tid / kTW) * W + x0 + tid % kTW];
            lds_barrier();
            if (k + 1 < seg) fetch(Y0, x0, 4 * k + 8);
            layer1(4 * k + 3, 4);
            lds_barrier();
            ring_hidden<4>(ring1, (uint2 *)ring2, Ws2, b2, 4 * k + 2, wave, i16, q);
            lds_barrier();
            ring_hidden<4>(ring2, (uint2 *)ring3, Ws3, b3, 4 * k + 1, wave, i16, q);
            lds_barrier();
            // layer 4 (32 -> 2: output channels 0 and 1 of a 16-row A operand,
            // no ReLU); D^T: lanes with q = 0 hold channels 0 .. 3 of pixel i16
            {
                bf16x8 wb[9];
#pragma unroll
                for (int t = 0; t < 9; ++t)
                    wb[t] = i16 < 2 ? __builtin_bit_cast(bf16x8, ((const u32x4v *)Ws4)[(t * 2 + i16) * 4 + q])
                                    : bf16x8{};
                const float b40 = b4[0], b41 = b4[1];
                for (int mt = wave; mt < kTH * (kTW / 16); mt += NW) {
                    const int rr = mt / (kTW / 16), px = (mt - rr * (kTW / 16)) * 16 + i16, r = 4 * k + rr;
                    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int t = 0; t < 9; ++t) {
                        const bf16x8 av = __builtin_bit_cast(
                            bf16x8, ring3[(rslot(r - 1 + t / 3) * kACols + px + t % 3) * kPixU + q]);
                        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wb[t], av, acc, 0, 0, 0);
                    }
                    if (q == 0) res[rr * kTW + px] = make_float2(acc[0] + b40, acc[1] + b41);
                }
            }
            lds_barrier();
            // psi_out = psi + s e^{-i theta} (r0 + i r1) for the step's pixels
            if (tid < kTH * kTW) {
                const long long pix = (long long)(Y0 + 4 * k + tid / kTW) * W + x0 + tid % kTW;
                const float2 rv = rot(res[tid], make_float2(e.x, -e.y));
                psi_out[pix] = make_float2(pc.x + s_out * rv.x, pc.y + s_out * rv.y);
            }
        }
    }
}

// ---------------------------------------------------------------- backward data
// dX[q][ci] = sum_tap sum_co dZ[q - off(tap)][co] W[tap][co][ci], masked by the
// ReLU of the layer below (Aprev > 0), written as bf16.
template <int CIN_P, int COUT_P>
__global__ __launch_bounds__(256) void k_conv_bwd_data(const u16 *__restrict__ dZ, const u16 *__restrict__ Wb,
                                                       const u16 *__restrict__ Aprev, u16 *__restrict__ dX,
                                                       int H, int W, long long npix)
{
    constexpr int KTOT = 9 * COUT_P, KCH = KTOT / 16, NB = CIN_P / 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long long pix0 = ((long long)blockIdx.x * 4 + wave) * 16;
    if (pix0 >= npix) return;
    const long long HW = (long long)H * W;
    const long long pa = pix0 + (lane & 15);
    const long long img = pa / HW;
    const int rem = (int)(pa - img * HW), y = rem / W, x = rem - (rem / W) * W;
    const int kq = 4 * (lane >> 4);
    f32x4 acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[nb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
    for (int kc = 0; kc < KCH; ++kc) {
        const int k = kc * 16 + kq;
        const int tap = k / COUT_P, c0 = k - tap * COUT_P;
        const int ys = wrap(y - (tap / 3 - 1), H), xs = wrap(x - (tap % 3 - 1), W);
        const bf16x4 av = *(const bf16x4 *)(dZ + ((img * H + ys) * W + xs) * COUT_P + c0);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const bf16x4 bv = *(const bf16x4 *)(Wb + ((long long)tap * CIN_P + nb * 16 + (lane & 15)) * COUT_P + c0);
            acc[nb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[nb], 0, 0, 0);
        }
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        const int ch = nb * 16 + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const long long p = pix0 + 4 * (lane >> 4) + r;
            const float v = bf2f(Aprev[p * CIN_P + ch]) > 0.f ? acc[nb][r] : 0.f;
            dX[p * CIN_P + ch] = f2bf(v);
        }
    }
}

// Data gradients of a layer with 32 input channels on tiled shapes, in the
// forward kernel's tiling: dX[p][ci] = sum_tap sum_co dZ[p - off(tap)][co]
// W[tap][co][ci] is a forward convolution of dZ with the taps mirrored and
// the weights transposed.  D^T = W^T dZ^T: lane (i16, q) ends with pixel i16
// of an M-tile and the channels nb*16 + 4q .. +3, staged as 8 bytes in LDS;
// each wave then writes its row of 64 pixels as 16-byte pieces, zeroed where
// the layer below's ReLU was inactive (Aprev <= 0).  Taps accumulate in the
// order 0 .. 8, each one K chunk of the COUT output channels: 32 on
// v_mfma_f32_16x16x32_bf16 (8 channels per lane), 16 (the last layer's 2,
// padded) on v_mfma_f32_16x16x16_bf16 (4 per lane; same A, B and D lane
// layout with half the K).
template <int COUT>
__global__ __launch_bounds__(256) void k_conv_bwd_data_t(const u16 *__restrict__ dZ, const u16 *__restrict__ Wb,
                                                         const u16 *__restrict__ Aprev, u16 *__restrict__ dX,
                                                         int H, int W, int ntiles)
{
    static_assert(COUT == 32 || COUT == 16, "32 or 16 output channels");
    // one lane's K chunk of a pixel: 8 channels (16 bytes) or 4 (8 bytes)
    using Q = std::conditional_t<COUT == 32, u32x4v, uint2>;
    using KV = std::conditional_t<COUT == 32, bf16x8, bf16x4>;
    constexpr int KL = COUT / 4;   // channels per lane and K chunk
    __shared__ Q xin[kHP * kWP * 4];             // dZ halo, quarters of each pixel's channels
    __shared__ u32x4v yst[4][kTW * 64 / 16];     // per-wave output staging, 64 bytes per pixel
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int i16 = lane & 15, q = lane >> 4;
    // A fragments: rows ci = nb*16 + i16 of W[tap]^T, K = co KL q .. KL q + KL - 1
    KV wa[9][2];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
            wa[t][nb] = *(const KV *)(Wb + ((long long)(t * 32 + nb * 16 + i16)) * COUT + KL * q);
    const int tx = W / kTW, ty = H / kTH;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int img = tile / (tx * ty), r0 = tile - img * tx * ty;
        const int y0 = (r0 / tx) * kTH, x0 = (r0 % tx) * kTW;
        const u16 *Zi = dZ + (long long)img * H * W * COUT;
        __syncthreads();   // the previous tile's readers are done with xin
        for (int c = tid; c < kHP * kWP * 4; c += 256) {
            const int pq = c & 3, pix = c >> 2, rr = pix / kWP, cc = pix - rr * kWP;
            int ys = y0 + rr - 1, xs = x0 + cc - 1;
            ys = ys < 0 ? ys + H : (ys >= H ? ys - H : ys);
            xs = xs < 0 ? xs + W : (xs >= W ? xs - W : xs);
            xin[c] = *(const Q *)(Zi + ((long long)ys * W + xs) * COUT + pq * KL);
        }
        __syncthreads();
        f32x4 acc[4][2];
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) acc[m][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            // dZ at p - off(t): the staged halo at row offset 2 - t/3, column offset 2 - t%3
            const int dy = 2 - t / 3, dx = 2 - t % 3;
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const KV av = __builtin_bit_cast(KV, xin[((wave + dy) * kWP + m * 16 + i16 + dx) * 4 + q]);
#pragma unroll
                for (int nb = 0; nb < 2; ++nb) {
                    if constexpr (COUT == 32)
                        acc[m][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[t][nb], av, acc[m][nb], 0, 0, 0);
                    else
                        acc[m][nb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wa[t][nb], av, acc[m][nb], 0, 0, 0);
                }
            }
        }
        uint2 *ys = (uint2 *)yst[wave];
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) {
                const f32x2v lo = {acc[m][nb][0], acc[m][nb][1]}, hi = {acc[m][nb][2], acc[m][nb][3]};
                ys[(m * 16 + i16) * 8 + nb * 4 + q] =
                    make_uint2(__builtin_bit_cast(unsigned, __builtin_convertvector(lo, bf16x2v)),
                               __builtin_bit_cast(unsigned, __builtin_convertvector(hi, bf16x2v)));
            }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        // row (y0 + wave), pixels x0 .. x0 + 63: 4 KiB contiguous in dX and Aprev
        const long long p0 = ((long long)img * H + y0 + wave) * W + x0;
        const u32x4v *arow = (const u32x4v *)(Aprev + p0 * 32);
        u32x4v *drow = (u32x4v *)(dX + p0 * 32);
#pragma unroll
        for (int c = lane; c < kTW * 64 / 16; c += 64) {
            const u32x4v a = arow[c];
            u32x4v v = yst[wave][c];
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                const unsigned keep = (__uint_as_float(a[w] << 16) > 0.f ? 0xffffu : 0u) |
                                      (__uint_as_float(a[w] & 0xffff0000u) > 0.f ? 0xffff0000u : 0u);
                v[w] &= keep;
            }
            drow[c] = v;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

// ---------------------------------------------------------------- backward weights
// Per block, over its chunks of 64 flat pixels: dW[tap][co][ci] += dZ^T Xs and
// db[co] += sum dZ, staged through LDS transposed (channel-major) so every
// MFMA operand is one 8-byte read.  Partials go to part[block][...].
template <int CIN_P, int COUT_P>
__global__ __launch_bounds__(256) void k_conv_bwd_w(const u16 *__restrict__ X, const u16 *__restrict__ dZ,
                                                    float *__restrict__ part, int H, int W, long long npix)
{
    constexpr int CINN = CIN_P < 16 ? 16 : CIN_P;
    constexpr int MB = COUT_P / 16, NB = CINN / 16, NBLK = 9 * MB * NB;
    constexpr int PER_WAVE = (NBLK + 3) / 4;
    constexpr int PSTRIDE = 9 * COUT_P * CINN + COUT_P;
    __shared__ __align__(16) u16 xs[9 * CINN * 64];
    __shared__ __align__(16) u16 dz[COUT_P * 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const long long HW = (long long)H * W;
    const long long nchunks = npix / 64;
    f32x4 acc[PER_WAVE];
#pragma unroll
    for (int i = 0; i < PER_WAVE; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
    float dbias = 0.f;
    for (long long c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const long long p0 = c * 64;
        for (int e = tid; e < 9 * CINN * 64; e += 256) {
            const int px = e & 63, ci = (e >> 6) % CINN, tap = (e >> 6) / CINN;
            u16 v = 0;
            if (ci < CIN_P) {
                const long long p = p0 + px, img = p / HW;
                const int rem = (int)(p - img * HW), y = rem / W, x = rem - (rem / W) * W;
                const int ys = wrap(y + tap / 3 - 1, H), xx = wrap(x + tap % 3 - 1, W);
                v = X[((img * H + ys) * W + xx) * CIN_P + ci];
            }
            xs[e] = v;
        }
        for (int e = tid; e < COUT_P * 64; e += 256) {
            const int px = e & 63, co = e >> 6;
            dz[e] = dZ[(p0 + px) * COUT_P + co];
        }
        __syncthreads();
        if (tid < COUT_P) {
            float s = 0.f;
            for (int px = 0; px < 64; ++px) s += bf2f(dz[tid * 64 + px]);
            dbias += s;
        }
#pragma unroll
        for (int i = 0; i < PER_WAVE; ++i) {
            const int blk = wave + 4 * i;
            if (blk < NBLK) {
                const int tap = blk / (MB * NB), mb = (blk / NB) % MB, nb = blk % NB;
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const int pk = kk * 16 + 4 * (lane >> 4);
                    const bf16x4 av = *(const bf16x4 *)(dz + (mb * 16 + (lane & 15)) * 64 + pk);
                    const bf16x4 bv = *(const bf16x4 *)(xs + (tap * CINN + nb * 16 + (lane & 15)) * 64 + pk);
                    acc[i] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[i], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }
    float *out = part + (long long)blockIdx.x * PSTRIDE;
#pragma unroll
    for (int i = 0; i < PER_WAVE; ++i) {
        const int blk = wave + 4 * i;
        if (blk < NBLK) {
            const int tap = blk / (MB * NB), mb = (blk / NB) % MB, nb = blk % NB;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int co = mb * 16 + 4 * (lane >> 4) + r, ci = nb * 16 + (lane & 15);
                out[(tap * COUT_P + co) * CINN + ci] = acc[i][r];
            }
        }
    }
    if (tid < COUT_P) out[9 * COUT_P * CINN + tid] = dbias;
}

// Weight gradients on tiled shapes: dW[tap][co][ci] = sum_px dZ[px][co]
// X[px + off(tap)][ci] and db[co] = sum_px dZ[px][co] as implicit GEMMs with
// K = pixels on v_mfma_f32_16x16x32_bf16.  A block walks tiles of 4 x 64
// pixels (fixed tiles per block, fixed order: deterministic partials).  Per
// tile the 6 x 66 input halo (6 x 72 staged) and the tile's dZ arrive with
// coalesced 16-byte loads into pixel-major LDS (8 bytes of padding per
// pixel), then each lane turns 4 pixels x 4 channels around into 4 channel
// rows with 8-byte reads and writes: channel-major copies whose channel
// strides (880 and 528 bytes) put the 16-byte operand reads of 16 channels
// on distinct banks.  K is split over the waves: wave w owns pixels
// 32w .. 32w + 31 of every tile and accumulates all 9 x MB x NB output
// blocks.  Per window row one 16-byte read and the 4 bytes after it give the
// operands of all three tap columns (the shifted ones by a funnel shift),
// and the bias gradient is one more MFMA against ones.  The next tile's
// inputs are loaded into registers while the current one is computed; at
// the end the waves' sums are added in LDS in a fixed order and written as
// the block's partial.
template <int CIN_P, int COUT_P>
__global__ __launch_bounds__(512) void k_conv_bwd_w_t(const u16 *__restrict__ X, const u16 *__restrict__ dZ,
                                                      float *__restrict__ part, int H, int W, int ntiles)
{
    constexpr int CINN = CIN_P < 16 ? 16 : CIN_P;
    constexpr int MB = COUT_P / 16, NB = CINN / 16;
    constexpr int PSTRIDE = 9 * COUT_P * CINN + COUT_P;
    constexpr int XROW = 72, XCH = kHP * XROW + 8;   // u16: staged halo row (66 used), channel stride
    constexpr int ZCH = kTH * kTW + 8;               // u16: dZ channel stride
    constexpr int XPS = CIN_P == 4 ? 4 : CIN_P + 4;  // u16 per pixel, pixel-major halo
    constexpr int ZPS = COUT_P + 4;                  // u16 per pixel, pixel-major dZ
    constexpr int XQ = CIN_P / 4, ZQ = COUT_P / 4;   // 4-channel quads per pixel
    // coalesced loads: 16 bytes (two quads) where a pixel has them
    constexpr int XLQ = XQ >= 2 ? 2 : 1, XLOADS = kHP * XROW * XQ / XLQ, ZLOADS = kTH * kTW * ZQ / 2;
    constexpr int XLS = (XLOADS + 511) / 512, ZLS = (ZLOADS + 511) / 512;
    // turn-around items (quad p, row, 4-pixel group j): 16 lanes = JL groups x PL quads
    constexpr int XPL = XQ < 4 ? XQ : 4, XJL = 16 / XPL, XJH = (XROW / 4 + XJL - 1) / XJL;
    constexpr int XT = XQ * kHP * XJH * XJL, XTS = (XT + 511) / 512;
    constexpr int ZJH = (kTH * kTW / 4) / 4, ZT = ZQ * ZJH * 4, ZTS = (ZT + 511) / 512;
    constexpr int XRAW = kHP * XROW * XPS, ZRAW = kTH * kTW * ZPS;
    constexpr int SMU = XRAW + ZRAW + CIN_P * XCH + COUT_P * ZCH;
    static_assert(SMU * 2 >= 8 * NB * 256 * 4 && SMU * 2 >= 8 * COUT_P * 4, "reduction buffer");
    static_assert(ZQ % 4 == 0 && (XQ == 1 || XQ % 4 == 0), "quad layouts");
    typedef unsigned u32x2v __attribute__((ext_vector_type(2)));
    __shared__ __align__(16) u16 sm[SMU];
    u16 *const xraw = sm, *const zraw = xraw + XRAW, *const xt = zraw + ZRAW, *const dzt = xt + CIN_P * XCH;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int i16 = lane & 15, q = lane >> 4;
    f32x4 acc[9][MB][NB], accb[MB];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) acc[t][mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) accb[mb] = f32x4{0.f, 0.f, 0.f, 0.f};
    const bf16x8 ones = __builtin_bit_cast(bf16x8, u32x4v{0x3f803f80u, 0x3f803f80u, 0x3f803f80u, 0x3f803f80u});
    const int tx = W / kTW, ty = H / kTH;
    // the next tile's inputs in registers: load l of this thread is piece
    // (l * 512 + tid) of the pixel-major halo / dZ, XLQ or 2 quads each
    u32x4v xr[XLS], zr[ZLS];
    auto fetch = [&](int tile) {
        const int img = tile / (tx * ty), r0 = tile - img * tx * ty;
        const int y0 = (r0 / tx) * kTH, x0 = (r0 % tx) * kTW;
        const long long ib = (long long)img * H * W;
#pragma unroll
        for (int l = 0; l < XLS; ++l) {
            const int it = tid + l * 512;
            if (it < XLOADS) {
                const int pc = it % (XQ / XLQ), px = (it / (XQ / XLQ)) % XROW, rr = it / (XQ / XLQ * XROW);
                int ys = y0 + rr - 1, xs = x0 - 1 + px;
                ys = ys < 0 ? ys + H : (ys >= H ? ys - H : ys);
                xs = xs < 0 ? xs + W : (xs >= W ? xs - W : xs);
                const u16 *src = X + (ib + (long long)ys * W + xs) * CIN_P + 4 * XLQ * pc;
                if constexpr (XLQ == 2) {
                    xr[l] = *(const u32x4v *)src;
                } else {
                    const u32x2v v = *(const u32x2v *)src;
                    xr[l] = u32x4v{v.x, v.y, 0u, 0u};
                }
            }
        }
#pragma unroll
        for (int l = 0; l < ZLS; ++l) {
            const int it = tid + l * 512;
            if (it < ZLOADS) {
                const int pc = it % (ZQ / 2), px = it / (ZQ / 2), r = px / kTW, c = px - r * kTW;
                zr[l] = *(const u32x4v *)(dZ + (ib + (long long)(y0 + r) * W + x0 + c) * COUT_P + 8 * pc);
            }
        }
    };
    auto stash_raw = [&]() {
#pragma unroll
        for (int l = 0; l < XLS; ++l) {
            const int it = tid + l * 512;
            if (it < XLOADS) {
                const int pc = it % (XQ / XLQ), pix = it / (XQ / XLQ);
                u16 *dst = xraw + pix * XPS + 4 * XLQ * pc;
                *(u32x2v *)dst = u32x2v{xr[l].x, xr[l].y};
                if constexpr (XLQ == 2) *(u32x2v *)(dst + 4) = u32x2v{xr[l].z, xr[l].w};
            }
        }
#pragma unroll
        for (int l = 0; l < ZLS; ++l) {
            const int it = tid + l * 512;
            if (it < ZLOADS) {
                u16 *dst = zraw + (it / (ZQ / 2)) * ZPS + 8 * (it % (ZQ / 2));
                *(u32x2v *)dst = u32x2v{zr[l].x, zr[l].y};
                *(u32x2v *)(dst + 4) = u32x2v{zr[l].z, zr[l].w};
            }
        }
    };
    // 4 pixels x 4 channels (pixel-major, pixel stride ps) -> 4 channel rows
    // of 4 pixels (8 bytes each, channel stride cs)
    auto turn = [&](const u16 *src, int ps, u16 *dst, int cs) {
        u32x2v v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = *(const u32x2v *)(src + e * ps);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int wd = k >> 1;
            const unsigned a0 = wd ? v[0].y : v[0].x, a1 = wd ? v[1].y : v[1].x;
            const unsigned a2 = wd ? v[2].y : v[2].x, a3 = wd ? v[3].y : v[3].x;
            const unsigned lo = (k & 1) ? (a0 >> 16) | (a1 & 0xffff0000u) : (a0 & 0xffffu) | (a1 << 16);
            const unsigned hi = (k & 1) ? (a2 >> 16) | (a3 & 0xffff0000u) : (a2 & 0xffffu) | (a3 << 16);
            *(u32x2v *)(dst + k * cs) = u32x2v{lo, hi};
        }
    };
    auto transpose = [&]() {
#pragma unroll
        for (int s = 0; s < XTS; ++s) {
            const int it = tid + s * 512;
            if (it < XT) {
                const int pl = it % XPL, jl = (it / XPL) % XJL, jh = (it / 16) % XJH, rr = (it / (16 * XJH)) % kHP;
                const int p = (it / (16 * XJH * kHP)) * XPL + pl, j = jh * XJL + jl;
                if (j < XROW / 4) turn(xraw + (rr * XROW + 4 * j) * XPS + 4 * p, XPS, xt + 4 * p * XCH + rr * XROW + 4 * j, XCH);
            }
        }
#pragma unroll
        for (int s = 0; s < ZTS; ++s) {
            const int it = tid + s * 512;
            if (it < ZT) {
                const int pl = it % 4, jl = (it / 4) % 4, jh = (it / 16) % ZJH;
                const int p = (it / (16 * ZJH)) * 4 + pl, j = jh * 4 + jl;
                turn(zraw + 4 * j * ZPS + 4 * p, ZPS, dzt + 4 * p * ZCH + 4 * j, ZCH);
            }
        }
    };
    // this wave's K slice: tile pixels 32 wave + 8q .. +7, row r, column c
    const int px0 = 32 * wave + 8 * q, r = px0 / kTW, c = px0 - r * kTW;
    if (blockIdx.x < ntiles) fetch(blockIdx.x);
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        stash_raw();      // the previous tile's turn-around reads are done
        lds_barrier();    // ... and so are its MFMA operand reads
        transpose();
        lds_barrier();
        if (tile + (int)gridDim.x < ntiles) fetch(tile + gridDim.x);   // lands while this tile computes
        bf16x8 av[MB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            av[mb] = *(const bf16x8 *)(dzt + (mb * 16 + i16) * ZCH + px0);
            accb[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[mb], ones, accb[mb], 0, 0, 0);
        }
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const int ci = nb * 16 + i16;
                u32x4v w = {0u, 0u, 0u, 0u};
                unsigned w4 = 0u;
                if (ci < CIN_P) {
                    const u16 *src = xt + ci * XCH + (r + dy) * XROW + c;
                    w = *(const u32x4v *)src;
                    w4 = *(const unsigned *)(src + 8);
                }
                // halo columns c + dx .. c + dx + 7 for tap columns dx = 0, 1, 2
                const bf16x8 bv[3] = {
                    __builtin_bit_cast(bf16x8, w),
                    __builtin_bit_cast(bf16x8, u32x4v{__builtin_amdgcn_alignbit(w.y, w.x, 16),
                                                      __builtin_amdgcn_alignbit(w.z, w.y, 16),
                                                      __builtin_amdgcn_alignbit(w.w, w.z, 16),
                                                      __builtin_amdgcn_alignbit(w4, w.w, 16)}),
                    __builtin_bit_cast(bf16x8, u32x4v{w.y, w.z, w.w, w4})};
#pragma unroll
                for (int dx = 0; dx < 3; ++dx)
#pragma unroll
                    for (int mb = 0; mb < MB; ++mb)
                        acc[dy * 3 + dx][mb][nb] =
                            __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[mb], bv[dx], acc[dy * 3 + dx][mb][nb], 0, 0, 0);
            }
    }
    // the eight waves' sums, added in wave order, one (tap, mb) at a time
    float *const red = (float *)sm;
    float *out = part + (long long)blockIdx.x * PSTRIDE;
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
                *(f32x4 *)(red + ((wave * NB + nb) * 64 + lane) * 4) = acc[t][mb][nb];
            __syncthreads();
            if (tid < NB * 256) {
                const int nb = tid >> 8, e = tid & 255, ln = e >> 2, rr = e & 3;
                float s = 0.f;
                for (int w8 = 0; w8 < 8; ++w8) s += red[((w8 * NB + nb) * 64) * 4 + e];
                const int co = mb * 16 + 4 * (ln >> 4) + rr, ci = nb * 16 + (ln & 15);
                out[(t * COUT_P + co) * CINN + ci] = s;
            }
            __syncthreads();
        }
    // bias: column 0 of D holds sum_k dZ[k][co] for co = mb*16 + 4q + r
    if (i16 == 0) {
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) red[wave * COUT_P + mb * 16 + 4 * q + rr] = accb[mb][rr];
    }
    __syncthreads();
    if (tid < COUT_P) {
        float s = 0.f;
        for (int w8 = 0; w8 < 8; ++w8) s += red[w8 * COUT_P + tid];
        out[9 * COUT_P * CINN + tid] = s;
    }
}

// Sum the per-block partials of one layer into the flat gradient (fixed order).
__global__ void k_reduce_grad(const float *__restrict__ part, int nparts, int pstride, int cin, int cout,
                              int cinn, int coutp, float *__restrict__ gflat)
{
    const int nw = 9 * cout * cin;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nw + cout) return;
    int src;
    if (i < nw) {
        const int tap = i / (cout * cin), co = (i / cin) % cout, ci = i % cin;
        src = (tap * coutp + co) * cinn + ci;
    } else {
        src = 9 * coutp * cinn + (i - nw);
    }
    // 8 independent chains keep 8 loads in flight; combined in a fixed order
    float s8[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    int b = 0;
    for (; b + 8 <= nparts; b += 8)
#pragma unroll
        for (int k = 0; k < 8; ++k) s8[k] += part[(long long)(b + k) * pstride + src];
    for (; b < nparts; ++b) s8[0] += part[(long long)b * pstride + src];
    gflat[i] = ((s8[0] + s8[1]) + (s8[2] + s8[3])) + ((s8[4] + s8[5]) + (s8[6] + s8[7]));
}

// ---------------------------------------------------------------- loss, Adam, packing
// MSE over the two output channels; dZ4 = 2 (out - target) / count as bf16
// (16 padded channels), per-block FP32 partial of the squared error.
__global__ __launch_bounds__(256) void k_mse(const float *__restrict__ out, const float *__restrict__ tgt,
                                             u16 *__restrict__ dz4, float inv_count, long long npix,
                                             double *__restrict__ part)
{
    __shared__ double sh[5];
    double s = 0.0;
    for (long long p = (long long)blockIdx.x * 256 + threadIdx.x; p < npix; p += (long long)gridDim.x * 256) {
        const float d0 = out[2 * p] - tgt[2 * p], d1 = out[2 * p + 1] - tgt[2 * p + 1];
        s += (double)d0 * d0 + (double)d1 * d1;
        u16 *o = dz4 + p * 16;
        o[0] = f2bf(2.f * d0 * inv_count);
        o[1] = f2bf(2.f * d1 * inv_count);
#pragma unroll
        for (int c = 2; c < 16; ++c) o[c] = 0;
    }
    s = block_sum<256>(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_adam(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, int n, float lr, float b1, float b2, float eps, float c1,
                       float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Master FP32 flat weights -> bf16 forward [tap][coutp][cinp] and backward
// [tap][cinp][coutp] layouts (zero padded) and FP32 padded biases.
__global__ void k_refresh(const float *__restrict__ flat, int off, int cin, int cout, int cinp, int coutp,
                          u16 *__restrict__ wf, u16 *__restrict__ wb, float *__restrict__ bias)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = 9 * coutp * cinp;
    if (i < n) {
        const int tap = i / (coutp * cinp), co = (i / cinp) % coutp, ci = i % cinp;
        const float v = (co < cout && ci < cin) ? flat[off + (tap * cout + co) * cin + ci] : 0.f;
        const u16 h = f2bf(v);
        wf[(tap * coutp + co) * cinp + ci] = h;
        wb[(tap * cinp + ci) * coutp + co] = h;
    }
    if (i < coutp) bias[i] = i < cout ? flat[off + 9 * cout * cin + i] : 0.f;
}

// Input features of image b: (Re u, Im u, phi) times the input scales, bf16,
// with u = e^{i theta} psi.
__global__ void k_pack(const float2 *__restrict__ psi, const float *__restrict__ phi, u16 *__restrict__ x,
                       long long n, float s0, float s1, float s2, const double *theta)
{
    const float2 e = phase_of(theta);
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (long long)gridDim.x * blockDim.x) {
        const float2 v = rot(psi[p], e);
        u16 *o = x + p * 4;
        o[0] = f2bf(v.x * s0);
        o[1] = f2bf(v.y * s1);
        o[2] = f2bf(phi[p] * s2);
        o[3] = 0;
    }
}

// Target of image b: (psi_fine - psi_coarse) / s_out, FP32, two channels.
__global__ void k_pack_target(const float2 *__restrict__ fine, const float2 *__restrict__ coarse,
                              float *__restrict__ t, long long n, float inv_s)
{
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (long long)gridDim.x * blockDim.x) {
        const float2 f = fine[p], c = coarse[p];
        t[2 * p] = (f.x - c.x) * inv_s;
        t[2 * p + 1] = (f.y - c.y) * inv_s;
    }
}

// psi_out = psi_c + s_out e^{-i theta} (r0 + i r1)
__global__ void k_apply(const float2 *__restrict__ psi_c, const float *__restrict__ out, float2 *__restrict__ psi_o,
                        long long n, float s, const double *theta)
{
    const float2 e = phase_of(theta);
    const float2 eb = make_float2(e.x, -e.y);
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (long long)gridDim.x * blockDim.x) {
        const float2 c = psi_c[p];
        const float2 r = rot(make_float2(out[2 * p], out[2 * p + 1]), eb);
        psi_o[p] = make_float2(c.x + s * r.x, c.y + s * r.y);
    }
}

constexpr int kBwBlocks = 256;   // blocks of the weight-gradient kernels

}  // namespace

// ------------------------------------------------------------------ handle
struct gsn_corrector_ {
    int H, W, maxB;
    long long P;   // pixels per image
    hipStream_t stream;
    int device;
    // device buffers
    u16 *x0, *a[3], *dz4, *dza, *dzb;
    float *out, *tgt;
    float *wflat, *mom1, *mom2, *grad;
    u16 *wf[kLayers], *wb[kLayers];
    float *bias[kLayers];
    float *part;
    double *lpart;
    float *phi1;
    float2 *psic[2];
    int step;
    float in_scale[3], out_scale;
};

static size_t corrector_layout(int H, int W, int maxB, size_t *offs /* 16 entries or null */)
{
    const long long N = (long long)H * W * maxB;
    size_t o = 0, k = 0;
    auto take = [&](size_t bytes) {
        if (offs) offs[k] = o;
        ++k;
        o = align256(o + bytes);
    };
    take(8ull * N);        // x0: 4 bf16 channels
    take(64ull * N);       // a1
    take(64ull * N);       // a2
    take(64ull * N);       // a3
    take(32ull * N);       // dz4: 16 bf16 channels
    take(64ull * N);       // dza
    take(64ull * N);       // dzb
    take(8ull * N);        // out: 2 fp32
    take(8ull * N);        // target
    take(4ull * kNParams * 4);   // wflat, m, v, grad
    size_t wsz = 0;
    for (int l = 0; l < kLayers; ++l) wsz += 2 * align256(2ull * 9 * kCinP[l] * kCoutP[l]) + align256(4ull * kCoutP[l]);
    take(wsz);
    take(4ull * kBwBlocks * (9 * 32 * 32 + 32));   // weight-gradient partials
    take(8ull * 4096);                             // loss partials
    take(4ull * H * W);                            // phi of one image (corrected stepping)
    take(8ull * H * W);                            // psi copy 0
    take(8ull * H * W);                            // psi copy 1
    return o;
}

extern "C" gsn_status gsn_corrector_workspace_bytes(int H, int W, int max_batch, size_t *bytes)
{
    if (!bytes) return fail(GSN_EINVAL, "bytes is NULL");
    if (H < 8 || W < 8 || H > 4096 || W > 4096 || max_batch < 1 || max_batch > 256)
        return fail(GSN_EINVAL, "H, W must be in [8, 4096] and max_batch in [1, 256]");
    if (((long long)H * W) % 64 != 0) return fail(GSN_EUNSUPPORTED, "H * W must be a multiple of 64");
    *bytes = corrector_layout(H, W, max_batch, nullptr);
    return GSN_OK;
}

extern "C" gsn_status gsn_corrector_create(gsn_corrector *out, int H, int W, int max_batch, void *d_ws,
                                           size_t bytes, void *stream)
{
    if (!out) return fail(GSN_EINVAL, "out is NULL");
    *out = nullptr;
    size_t need = 0;
    gsn_status s = gsn_corrector_workspace_bytes(H, W, max_batch, &need);
    if (s) return s;
    if (!d_ws) return fail(GSN_EINVAL, "workspace is NULL");
    if (((uintptr_t)d_ws & 255) != 0) return fail(GSN_EWORKSPACE, "workspace must be 256-byte aligned");
    if (bytes < need) return fail(GSN_EWORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
    gsn_corrector c = new (std::nothrow) gsn_corrector_();
    if (!c) return fail(GSN_EINVAL, "out of host memory");
    c->H = H;
    c->W = W;
    c->maxB = max_batch;
    c->P = (long long)H * W;
    c->stream = (hipStream_t)stream;
    c->step = 0;
    c->in_scale[0] = c->in_scale[1] = c->in_scale[2] = 1.f;
    c->out_scale = 1.f;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return fail(GSN_EHIP, "hipGetDevice failed");
    }
    size_t off[16];
    corrector_layout(H, W, max_batch, off);
    char *ws = (char *)d_ws;
    c->x0 = (u16 *)(ws + off[0]);
    for (int i = 0; i < 3; ++i) c->a[i] = (u16 *)(ws + off[1 + i]);
    c->dz4 = (u16 *)(ws + off[4]);
    c->dza = (u16 *)(ws + off[5]);
    c->dzb = (u16 *)(ws + off[6]);
    c->out = (float *)(ws + off[7]);
    c->tgt = (float *)(ws + off[8]);
    c->wflat = (float *)(ws + off[9]);
    c->mom1 = c->wflat + kNParams;
    c->mom2 = c->mom1 + kNParams;
    c->grad = c->mom2 + kNParams;
    char *wp = ws + off[10];
    for (int l = 0; l < kLayers; ++l) {
        const size_t wsz = align256(2ull * 9 * kCinP[l] * kCoutP[l]);
        c->wf[l] = (u16 *)wp; wp += wsz;
        c->wb[l] = (u16 *)wp; wp += wsz;
        c->bias[l] = (float *)wp; wp += align256(4ull * kCoutP[l]);
    }
    c->part = (float *)(ws + off[11]);
    c->lpart = (double *)(ws + off[12]);
    c->phi1 = (float *)(ws + off[13]);
    c->psic[0] = (float2 *)(ws + off[14]);
    c->psic[1] = (float2 *)(ws + off[15]);
    // weights start at zero until set
    if (hipMemsetAsync(c->wflat, 0, 16ull * kNParams, c->stream) != hipSuccess) {
        delete c;
        return fail(GSN_EHIP, "hipMemsetAsync failed");
    }
    *out = c;
    return GSN_OK;
}

extern "C" gsn_status gsn_corrector_destroy(gsn_corrector c)
{
    if (!c) return fail(GSN_EINVAL, "corrector is NULL");
    (void)hipStreamSynchronize(c->stream);
    delete c;
    return GSN_OK;
}

static gsn_status refresh(gsn_corrector c)
{
    int off = 0;
    for (int l = 0; l < kLayers; ++l) {
        const int n = 9 * kCinP[l] * kCoutP[l];
        hipLaunchKernelGGL(k_refresh, dim3((n + 255) / 256), dim3(256), 0, c->stream, c->wflat, off, kCin[l],
                           kCout[l], kCinP[l], kCoutP[l], c->wf[l], c->wb[l], c->bias[l]);
        HIP_TRY(hipGetLastError());
        off += 9 * kCin[l] * kCout[l] + kCout[l];
    }
    return GSN_OK;
}

extern "C" gsn_status gsn_corrector_set_weights(gsn_corrector c, const float *w, size_t n)
{
    if (!c || !w) return fail(GSN_EINVAL, "NULL argument");
    if (n != (size_t)kNParams) return fail(GSN_EINVAL, "expected 19970 weights");
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(w[i])) return fail(GSN_EINVAL, "weights must be finite");
    HIP_TRY(hipSetDevice(c->device));
    HIP_TRY(hipMemcpyAsync(c->wflat, w, 4ull * n, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemsetAsync(c->mom1, 0, 8ull * n, c->stream));   // Adam moments m and v
    c->step = 0;
    gsn_status s = refresh(c);
    if (s) return s;
    HIP_TRY(hipStreamSynchronize(c->stream));
    return GSN_OK;
}

extern "C" gsn_status gsn_corrector_get_weights(gsn_corrector c, float *w, size_t n)
{
    if (!c || !w) return fail(GSN_EINVAL, "NULL argument");
    if (n != (size_t)kNParams) return fail(GSN_EINVAL, "expected 19970 weights");
    HIP_TRY(hipSetDevice(c->device));
    HIP_TRY(hipMemcpyAsync(w, c->wflat, 4ull * n, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return GSN_OK;
}

extern "C" gsn_status gsn_corrector_set_scales(gsn_corrector c, const float in_scale[3], float out_scale)
{
    if (!c || !in_scale) return fail(GSN_EINVAL, "NULL argument");
    for (int i = 0; i < 3; ++i)
        if (!std::isfinite(in_scale[i])) return fail(GSN_EINVAL, "scales must be finite");
    if (!(std::isfinite(out_scale) && out_scale != 0.f)) return fail(GSN_EINVAL, "out_scale must be finite and != 0");
    for (int i = 0; i < 3; ++i) c->in_scale[i] = in_scale[i];
    c->out_scale = out_scale;
    return GSN_OK;
}

static gsn_status check_slot(gsn_corrector c, int b)
{
    if (!c) return fail(GSN_EINVAL, "corrector is NULL");
    if (b < 0 || b >= c->maxB) return fail(GSN_EINVAL, "image slot out of range");
    return GSN_OK;
}

extern "C" gsn_status gsn_corrector_pack(gsn_corrector c, int b, const void *psi, const float *phi)
{
    gsn_status s = check_slot(c, b);
    if (s) return s;
    if (!psi || !phi) return fail(GSN_EINVAL, "NULL argument");
    HIP_TRY(hipSetDevice(c->device));
    hipLaunchKernelGGL(k_pack, dim3(512), dim3(256), 0, c->stream, (const float2 *)psi, phi, c->x0 + 4 * c->P * b,
                       c->P, c->in_scale[0], c->in_scale[1], c->in_scale[2], (const double *)nullptr);
    HIP_TRY(hipGetLastError());
    return GSN_OK;
}

extern "C" gsn_status gsn_corrector_pack_target(gsn_corrector c, int b, const void *psi_fine, const void *psi_coarse)
{
    gsn_status s = check_slot(c, b);
    if (s) return s;
    if (!psi_fine || !psi_coarse) return fail(GSN_EINVAL, "NULL argument");
    HIP_TRY(hipSetDevice(c->device));
    hipLaunchKernelGGL(k_pack_target, dim3(512), dim3(256), 0, c->stream, (const float2 *)psi_fine,
                       (const float2 *)psi_coarse, c->tgt + 2 * c->P * b, c->P, 1.f / c->out_scale);
    HIP_TRY(hipGetLastError());
    return GSN_OK;
}

// forward over B packed images: a1..a3 stashed, out (FP32, 2 channels)
static bool tiled(gsn_corrector c) { return c->W % kTW == 0 && c->H % kTH == 0; }

// persistent grid of the LDS-tiled layers: at most 3 blocks per CU
static dim3 tiled_grid(gsn_corrector c, int ntiles)
{
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess || cus < 1)
        cus = 256;
    return dim3((unsigned)std::min(ntiles, 3 * cus));
}

// the two hidden layers, tiled (a1 -> a2 -> a3)
static void hidden_tiled(gsn_corrector c, dim3 tg, int ntiles)
{
    const int H = c->H, W = c->W;
    hipLaunchKernelGGL((k_conv_fwd_t<32, 32, true, false>), tg, dim3(256), 0, c->stream, c->a[0], c->wf[1],
                       c->bias[1], (void *)c->a[1], H, W, ntiles, (const float2 *)nullptr, (float2 *)nullptr, 0.f,
                       (const double *)nullptr);
    hipLaunchKernelGGL((k_conv_fwd_t<32, 32, true, false>), tg, dim3(256), 0, c->stream, c->a[1], c->wf[2],
                       c->bias[2], (void *)c->a[2], H, W, ntiles, (const float2 *)nullptr, (float2 *)nullptr, 0.f,
                       (const double *)nullptr);
}

static gsn_status forward(gsn_corrector c, int B)
{
    const long long np = c->P * B;
    const dim3 grid((unsigned)(np / 64)), block(256);
    const int H = c->H, W = c->W;
    if (tiled(c)) {
        const int ntiles = (int)(np / (kTW * kTH));
        const dim3 tg = tiled_grid(c, ntiles);
        hipLaunchKernelGGL((k_conv1_t<false>), tg, block, 0, c->stream, c->x0, (const float2 *)nullptr,
                           (const float *)nullptr, 0.f, 0.f, 0.f, c->wf[0], c->bias[0], c->a[0], H, W, ntiles,
                           (const double *)nullptr);
        hidden_tiled(c, tg, ntiles);
        hipLaunchKernelGGL((k_conv_fwd_t<16, 2, false, true>), tg, block, 0, c->stream, c->a[2], c->wf[3],
                           c->bias[3], (void *)c->out, H, W, ntiles, (const float2 *)nullptr, (float2 *)nullptr, 0.f,
                           (const double *)nullptr);
    } else {
        hipLaunchKernelGGL((k_conv_fwd<4, 32, 32, true, false>), grid, block, 0, c->stream, c->x0, c->wf[0],
                           c->bias[0], (void *)c->a[0], H, W, np);
        hipLaunchKernelGGL((k_conv_fwd<32, 32, 32, true, false>), grid, block, 0, c->stream, c->a[0], c->wf[1],
                           c->bias[1], (void *)c->a[1], H, W, np);
        hipLaunchKernelGGL((k_conv_fwd<32, 32, 32, true, false>), grid, block, 0, c->stream, c->a[1], c->wf[2],
                           c->bias[2], (void *)c->a[2], H, W, np);
        hipLaunchKernelGGL((k_conv_fwd<32, 16, 2, false, true>), grid, block, 0, c->stream, c->a[2], c->wf[3],
                           c->bias[3], (void *)c->out, H, W, np);
    }
    HIP_TRY(hipGetLastError());
    return GSN_OK;
}

extern "C" gsn_status gsn_corrector_forward(gsn_corrector c, int B, float *out_dev)
{
    if (!c) return fail(GSN_EINVAL, "corrector is NULL");
    if (B < 1 || B > c->maxB) return fail(GSN_EINVAL, "batch size out of range");
    HIP_TRY(hipSetDevice(c->device));
    gsn_status s = forward(c, B);
    if (s) return s;
    if (out_dev)
        HIP_TRY(hipMemcpyAsync(out_dev, c->out, 8ull * c->P * B, hipMemcpyDeviceToDevice, c->stream));
    return GSN_OK;
}

// forward + loss + backward into c->grad (flat FP32); loss returned (synchronising)
static gsn_status gradients(gsn_corrector c, int B, float *loss)
{
    const long long np = c->P * B;
    const dim3 grid((unsigned)(np / 64)), block(256);
    const int H = c->H, W = c->W;
    gsn_status s = forward(c, B);
    if (s) return s;
    const int nlb = 1024;
    hipLaunchKernelGGL(k_mse, dim3(nlb), block, 0, c->stream, c->out, c->tgt, c->dz4, 1.f / (float)(2 * np), np,
                       c->lpart);
    // layer 4 (32 -> 2, padded 16): weight grads, then data grads into dza
    const int pstride_h = 9 * 32 * 32 + 32;
    int offs[kLayers], o = 0;
    for (int l = 0; l < kLayers; ++l) { offs[l] = o; o += 9 * kCin[l] * kCout[l] + kCout[l]; }
    const bool tl = tiled(c);
    const int ntl = (int)(np / (kTW * kTH));
    if (tl)
        hipLaunchKernelGGL((k_conv_bwd_w_t<32, 16>), dim3(kBwBlocks), dim3(512), 0, c->stream, c->a[2], c->dz4, c->part,
                           H, W, ntl);
    else
        hipLaunchKernelGGL((k_conv_bwd_w<32, 16>), dim3(kBwBlocks), block, 0, c->stream, c->a[2], c->dz4, c->part, H, W,
                           np);
    hipLaunchKernelGGL(k_reduce_grad, dim3((9 * 32 * 2 + 2 + 255) / 256), dim3(256), 0, c->stream, c->part,
                       kBwBlocks, 9 * 16 * 32 + 16, 32, 2, 32, 16, c->grad + offs[3]);
    if (tl)
        hipLaunchKernelGGL(k_conv_bwd_data_t<16>, tiled_grid(c, ntl), block, 0, c->stream, c->dz4, c->wb[3], c->a[2],
                           c->dza, H, W, ntl);
    else
        hipLaunchKernelGGL((k_conv_bwd_data<32, 16>), grid, block, 0, c->stream, c->dz4, c->wb[3], c->a[2], c->dza, H,
                           W, np);
    // layer 3
    if (tl)
        hipLaunchKernelGGL((k_conv_bwd_w_t<32, 32>), dim3(kBwBlocks), dim3(512), 0, c->stream, c->a[1], c->dza, c->part,
                           H, W, ntl);
    else
        hipLaunchKernelGGL((k_conv_bwd_w<32, 32>), dim3(kBwBlocks), block, 0, c->stream, c->a[1], c->dza, c->part, H, W,
                           np);
    hipLaunchKernelGGL(k_reduce_grad, dim3((9 * 32 * 32 + 32 + 255) / 256), dim3(256), 0, c->stream, c->part,
                       kBwBlocks, pstride_h, 32, 32, 32, 32, c->grad + offs[2]);
    if (tl)
        hipLaunchKernelGGL(k_conv_bwd_data_t<32>, tiled_grid(c, ntl), block, 0, c->stream, c->dza, c->wb[2], c->a[1], c->dzb,
                           H, W, ntl);
    else
        hipLaunchKernelGGL((k_conv_bwd_data<32, 32>), grid, block, 0, c->stream, c->dza, c->wb[2], c->a[1], c->dzb, H, W,
                           np);
    // layer 2
    if (tl)
        hipLaunchKernelGGL((k_conv_bwd_w_t<32, 32>), dim3(kBwBlocks), dim3(512), 0, c->stream, c->a[0], c->dzb, c->part,
                           H, W, ntl);
    else
        hipLaunchKernelGGL((k_conv_bwd_w<32, 32>), dim3(kBwBlocks), block, 0, c->stream, c->a[0], c->dzb, c->part, H, W,
                           np);
    hipLaunchKernelGGL(k_reduce_grad, dim3((9 * 32 * 32 + 32 + 255) / 256), dim3(256), 0, c->stream, c->part,
                       kBwBlocks, pstride_h, 32, 32, 32, 32, c->grad + offs[1]);
    if (tl)
        hipLaunchKernelGGL(k_conv_bwd_data_t<32>, tiled_grid(c, ntl), block, 0, c->stream, c->dzb, c->wb[1], c->a[0], c->dza,
                           H, W, ntl);
    else
        hipLaunchKernelGGL((k_conv_bwd_data<32, 32>), grid, block, 0, c->stream, c->dzb, c->wb[1], c->a[0], c->dza, H, W,
                           np);
    // layer 1 (3 -> 32, input padded to 4 channels; no data gradient needed)
    if (tl)
        hipLaunchKernelGGL((k_conv_bwd_w_t<4, 32>), dim3(kBwBlocks), dim3(512), 0, c->stream, c->x0, c->dza, c->part, H,
                           W, ntl);
    else
        hipLaunchKernelGGL((k_conv_bwd_w<4, 32>), dim3(kBwBlocks), block, 0, c->stream, c->x0, c->dza, c->part, H, W, np);
    hipLaunchKernelGGL(k_reduce_grad, dim3((9 * 3 * 32 + 32 + 255) / 256), dim3(256), 0, c->stream, c->part,
                       kBwBlocks, 9 * 32 * 16 + 32, 3, 32, 16, 32, c->grad + offs[0]);
    HIP_TRY(hipGetLastError());
    std::vector<double> h(nlb);
    HIP_TRY(hipMemcpyAsync(h.data(), c->lpart, 8ull * nlb, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    double sum = 0.0;
    for (double v : h) sum += v;
    if (loss) *loss = (float)(sum / (double)(2 * np));
    return GSN_OK;
}

extern "C" gsn_status gsn_corrector_gradients(gsn_corrector c, int B, float *grad_host, float *loss)
{
    if (!c) return fail(GSN_EINVAL, "corrector is NULL");
    if (B < 1 || B > c->maxB) return fail(GSN_EINVAL, "batch size out of range");
    HIP_TRY(hipSetDevice(c->device));
    gsn_status s = gradients(c, B, loss);
    if (s) return s;
    if (grad_host) {
        HIP_TRY(hipMemcpyAsync(grad_host, c->grad, 4ull * kNParams, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
    }
    return GSN_OK;
}

extern "C" gsn_status gsn_corrector_train_step(gsn_corrector c, int B, float lr, float *loss)
{
    if (!c) return fail(GSN_EINVAL, "corrector is NULL");
    if (B < 1 || B > c->maxB) return fail(GSN_EINVAL, "batch size out of range");
    if (!(std::isfinite(lr) && lr > 0.f)) return fail(GSN_EINVAL, "lr must be finite and > 0");
    HIP_TRY(hipSetDevice(c->device));
    gsn_status s = gradients(c, B, loss);
    if (s) return s;
    if (loss && !std::isfinite(*loss)) return fail(GSN_ENONFINITE, "training loss is not finite");
    c->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, (float)c->step), c2 = 1.f - std::pow(b2, (float)c->step);
    hipLaunchKernelGGL(k_adam, dim3((kNParams + 255) / 256), dim3(256), 0, c->stream, c->wflat, c->mom1, c->mom2,
                       c->grad, kNParams, lr, b1, b2, 1e-8f, c1, c2);
    HIP_TRY(hipGetLastError());
    return refresh(c);
}

extern "C" gsn_status gsn_corrector_apply(gsn_corrector c, int b, const void *psi_c, void *psi_out)
{
    gsn_status s = check_slot(c, b);
    if (s) return s;
    if (!psi_c || !psi_out) return fail(GSN_EINVAL, "NULL argument");
    HIP_TRY(hipSetDevice(c->device));
    hipLaunchKernelGGL(k_apply, dim3(512), dim3(256), 0, c->stream, (const float2 *)psi_c, c->out + 2 * c->P * b,
                       (float2 *)psi_out, c->P, c->out_scale, (const double *)nullptr);
    HIP_TRY(hipGetLastError());
    return GSN_OK;
}

// ------------------------------------------------------------------ internal hooks for corrected stepping
gsn_status corrector_correct_inplace(gsn_corrector c, float2 *psi, const float *phi, const double *theta,
                                     hipStream_t s)
{
    // the corrector runs on the caller's stream for this call only; the guard
    // puts its own stream back on every return path
    struct StreamGuard {
        gsn_corrector c;
        hipStream_t keep;
        ~StreamGuard() { c->stream = keep; }
    } guard{c, c->stream};
    c->stream = s;
    gsn_status st = GSN_OK;
    if (tiled(c)) {
        // the four layers fused: features from (psi, phi), the corrected
        // state into the output buffer (other tiles still read psi for their
        // halos), then copied back over psi
        HIP_TRY(hipSetDevice(c->device));
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess || cus < 1)
            cus = 256;
        // segments of seg tiles down a 64-column strip, about one per CU
        // (longer segments amortise the warm-up, more segments fill the chip)
        const int th = c->H / kTH, tw = c->W / kTW;
        int seg = std::max(1, th * tw / cus);
        while (th % seg) --seg;
        const int nseg = th / seg * tw;
        float2 *tmp = (float2 *)c->out;   // 8 bytes per pixel, unused by inference
        hipLaunchKernelGGL(k_corr_fused, dim3((unsigned)std::min(nseg, cus)), dim3(kFusedThreads), 0, c->stream,
                           (const float2 *)psi, phi, tmp, c->in_scale[0], c->in_scale[1], c->in_scale[2],
                           c->out_scale, c->wf[0], c->wf[1], c->wf[2], c->wf[3], c->bias[0], c->bias[1], c->bias[2],
                           c->bias[3], c->H, c->W, seg, nseg, theta);
        if (hipGetLastError() != hipSuccess) return fail(GSN_EHIP, "corrector inference launch failed");
        HIP_TRY(hipMemcpyAsync(psi, tmp, 8ull * c->P, hipMemcpyDeviceToDevice, c->stream));
    } else {
        HIP_TRY(hipSetDevice(c->device));
        hipLaunchKernelGGL(k_pack, dim3(512), dim3(256), 0, c->stream, (const float2 *)psi, phi, c->x0, c->P,
                           c->in_scale[0], c->in_scale[1], c->in_scale[2], theta);
        st = forward(c, 1);
        if (!st) {
            hipLaunchKernelGGL(k_apply, dim3(512), dim3(256), 0, c->stream, (const float2 *)psi, c->out, psi, c->P,
                               c->out_scale, theta);
            if (hipGetLastError() != hipSuccess) st = fail(GSN_EHIP, "corrector apply launch failed");
        }
    }
    return st;
}

int corrector_height(gsn_corrector c) { return c->H; }
float *corrector_phi_buffer(gsn_corrector c) { return c->phi1; }
float2 *corrector_psi_buffer(gsn_corrector c, int which) { return c->psic[which & 1]; }
int corrector_width(gsn_corrector c) { return c->W; }
