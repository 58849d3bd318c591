/*
 * gsn_oracle.c -- plain FP64 CPU oracle for the generalised Schroedinger-Newton
 * split-step solver of Ferreira, Silva, Bertolami, Gomes & Guerreiro,
 * "Using numerical methods from nonlocal optics to simulate the dynamics of
 * N-body systems in alternative theories of gravity" (arXiv:1909.08354).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct reference
 * the HIP solver is checked against.  Only the test-suite, the smoke check and
 * the benchmark's CPU-baseline leg may load it; the product path never does.
 * It shares no code, header, table or constant generator with the GPU library.
 *
 * What is computed (paper Sec. II, Eq. (1)-(2) and the optics form Eq. (3);
 * Sec. III for the method: symmetric split-step Fourier for Eq. (1) and a
 * spectral solve for Eq. (2)):
 *
 *     i d(psi)/dz = -a lap(psi) - (g |psi|^2 + phi) psi,
 *     phi_hat(k)  = K(k) rho_hat(k),   rho = |psi|^2,
 *     K(k)        = c_N/|k|^2 [k != 0] + c_Y/(|k|^2 + m_Y^2) + c_0.
 *
 * This is Eq. (1) with A = -a, B = -1, G(rho) = -g rho, i.e. Eq. (3) with
 * k = k0 = 1 and Delta n = g rho + phi.  The kernel family is the Fourier form
 * of Eq. (2), Eq. (4), Eq. (5), and the constant-coefficient Fourier form of the
 * modified Poisson equation Eq. (8) / Eq. (12) (Newtonian 1/k^2 plus a Yukawa
 * correction plus a contact term).  The k = 0 Newtonian term is dropped (a
 * periodic Poisson problem needs a neutral source); the Yukawa and contact
 * k = 0 terms are kept.
 *
 * Discretisation: C-order grid [n0][n1][n2] (last axis contiguous), periodic,
 * x_j = -L/2 + j L/N, k_j = 2 pi j'/L with j' = j for j < N/2 else j - N.
 * Forward DFT  X_k = sum_x x_x exp(-i k.x)   (unnormalised);
 * inverse DFT  x_x = (1/P) sum_k X_k exp(+i k.x).
 *
 * One symmetric step (Strang):  psi <- L(dz/2) N(dz) L(dz/2) psi with
 *   L(h): psi <- IDFT[ exp(-i a |k|^2 h) DFT psi ]
 *   N(h): rho = |psi|^2; phi = Re IDFT[ K DFT rho ]; psi <- psi exp(i (g rho + phi) h)
 * The nonlinear sub-step is exact because rho is unchanged by a pointwise phase.
 *
 * Local terms of Eq. (15) (Sec. II C), optional: the Kerr term g rho generalises
 * to the local potential
 *   U = g rho + c_p f_n(max(rho, rho_f)) + c_B lap(s) / (2 max(s, sqrt(rho_f))),
 *   s = sqrt(rho),  f_1(rho) = ln rho,  f_n(rho) = n/(n-1) rho^(n-1) (n > 1 or n < 0),
 * the polytropic pressure potential and the Bohm potential lap(sqrt rho)/(2 sqrt rho),
 * with lap(s) = Re IDFT[-|k|^2 DFT s] and rho_f > 0 a floor that keeps ln rho,
 * negative powers and the division finite where the density vanishes.  Then
 *   N(h): psi <- psi exp(i (U + phi) h).
 * Eq. (15) divided by nu is this form with a = nu/2, c_B = -nu, c_p = -w/nu and
 * phi = -(phi_N + phi_C)/nu.
 *
 * Position-dependent source and static potential (Eq. (9)-(12)), optional:
 * the kernel acts on s = gamma(x) rho + beta(x) lap(rho) instead of rho, and a
 * static field V(x) joins the phase:  N(h): psi <- psi exp(i (U + phi + V) h).
 * The pure non-minimal coupling of Eq. (12), lap phi_N = beta lap rho + gamma rho,
 * with Eq. (9)-(11) for gamma(r), beta(r) and phi_C(r), is this with
 * K = (1/nu)/|k|^2 and V = -phi_C/nu.
 *
 * The FFT is an iterative radix-2 transform with twiddles from direct FP64
 * cos/sin of 2 pi m / n (never a recurrence).  Multi-dimensional transforms are
 * applied axis by axis.  OpenMP threads run independent 1-D lines in parallel;
 * results do not depend on the thread count.
 */
#define _GNU_SOURCE
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef double _Complex cx;

#define ORC_OK 0
#define ORC_EINVAL 1
#define ORC_ENOMEM 2

typedef struct {
    int ndim;
    int n[3];
    double L[3];
    long long P;      /* total number of points */
    long long stride[3];
} grid_t;

static int is_pow2(int v) { return v >= 1 && (v & (v - 1)) == 0; }

static int grid_init(grid_t *g, int ndim, const int *n, const double *L)
{
    if (ndim < 1 || ndim > 3 || !n) return ORC_EINVAL;
    g->ndim = ndim;
    g->P = 1;
    for (int d = 0; d < ndim; d++) {
        if (!is_pow2(n[d])) return ORC_EINVAL;
        if (L && !(L[d] > 0.0)) return ORC_EINVAL;
        g->n[d] = n[d];
        g->L[d] = L ? L[d] : 1.0;
        g->P *= n[d];
    }
    long long s = 1;
    for (int d = ndim - 1; d >= 0; d--) { g->stride[d] = s; s *= n[d]; }
    return ORC_OK;
}

static int nthreads_or_default(int nthreads)
{
    return nthreads > 0 ? nthreads : omp_get_max_threads();
}

/* wavenumber of DFT index j on an axis with N points and length L */
static double wavenumber(int j, int N, double L)
{
    int jj = (j < N / 2) ? j : j - N;
    return 2.0 * M_PI * (double)jj / L;
}

/* |k|^2 of the point with flat index q */
static double k_squared(const grid_t *g, long long q)
{
    double k2 = 0.0;
    for (int d = 0; d < g->ndim; d++) {
        int j = (int)((q / g->stride[d]) % g->n[d]);
        double k = wavenumber(j, g->n[d], g->L[d]);
        k2 += k * k;
    }
    return k2;
}

/* K(k) of Eq. (2) in Fourier form, kp = {c_N, c_Y, m_Y, c_0} */
static double kernel_value(double k2, const double *kp)
{
    double K = kp[3];
    if (kp[1] != 0.0) K += kp[1] / (k2 + kp[2] * kp[2]);
    if (k2 > 0.0) K += kp[0] / k2;
    return K;
}

/*
 * The multiplier K(k) of phi_hat = K rho_hat, from either the kernel family
 * (kp) or Eq. (1)-(2) with their own constants: lap phi + C phi = D rho gives
 * phi_hat = D rho_hat / (C - |k|^2), and Eq. (1)'s term B phi enters the phase
 * with the opposite sign of this file's phi, so K = B D / (|k|^2 - C).  With
 * C = 0 the k = 0 mode of the Poisson problem is dropped; with C > 0 (a
 * Helmholtz operator) a grid wavenumber with |k|^2 = C has no solution and is
 * rejected.
 */
typedef struct {
    int eq;              /* 0: kp; 1: (B, C, D) */
    const double *kp;
    double B, C, D;
} kspec_t;

static int kspec_check(const kspec_t *ks)
{
    if (!ks->eq) return ks->kp && !(ks->kp[1] != 0.0 && !(ks->kp[2] > 0.0)) ? ORC_OK : ORC_EINVAL;
    return isfinite(ks->B) && isfinite(ks->C) && isfinite(ks->D) ? ORC_OK : ORC_EINVAL;
}

static int kspec_value(const kspec_t *ks, double k2, double *K)
{
    if (!ks->eq) {
        *K = kernel_value(k2, ks->kp);
        return ORC_OK;
    }
    if (ks->C == 0.0 && k2 == 0.0) {
        *K = 0.0;
        return ORC_OK;
    }
    double den = k2 - ks->C;
    if (fabs(den) <= 1e-12 * fmax(1.0, fabs(ks->C))) return ORC_EINVAL;
    *K = ks->B * ks->D / den;
    return ORC_OK;
}

static int kspec_table(double *Kk, const kspec_t *ks, const grid_t *g)
{
    int bad = 0;
    for (long long q = 0; q < g->P; q++)
        if (kspec_value(ks, k_squared(g, q), &Kk[q])) bad = 1;
    return bad ? ORC_EINVAL : ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* 1-D radix-2 FFT                                                          */
/* ------------------------------------------------------------------------ */

/* tw[m] = exp(sign * 2 pi i m / n), m < n/2, each from cos/sin directly */
static cx *make_twiddles(int n, int sign)
{
    int h = n / 2 > 0 ? n / 2 : 1;
    cx *tw = (cx *)malloc(sizeof(cx) * (size_t)h);
    if (!tw) return NULL;
    for (int m = 0; m < h; m++) {
        double ang = 2.0 * M_PI * (double)m / (double)n;
        tw[m] = cos(ang) + (double)sign * sin(ang) * I;
    }
    return tw;
}

/* in-place unnormalised DFT of one contiguous line: bit reversal, then
   log2(n) butterfly stages of growing length */
static void fft_line(cx *a, int n, const cx *tw)
{
    for (int i = 1, j = 0; i < n; i++) {
        int bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) { cx t = a[i]; a[i] = a[j]; a[j] = t; }
    }
    for (int len = 2; len <= n; len <<= 1) {
        int half = len / 2, step = n / len;
        for (int i = 0; i < n; i += len) {
            for (int j = 0; j < half; j++) {
                cx u = a[i + j];
                cx v = a[i + j + half] * tw[j * step];
                a[i + j] = u + v;
                a[i + j + half] = u - v;
            }
        }
    }
}

/* transform every line along axis d; sign -1 forward, +1 inverse (no scale) */
static int fft_axis(cx *data, const grid_t *g, int d, int sign, int nthreads)
{
    int n = g->n[d];
    if (n == 1) return ORC_OK;
    long long stride = g->stride[d];
    long long nlines = g->P / n;
    cx *tw = make_twiddles(n, sign);
    if (!tw) return ORC_ENOMEM;
    int err = 0;
#pragma omp parallel num_threads(nthreads)
    {
        cx *line = (cx *)malloc(sizeof(cx) * (size_t)n);
        if (!line) {
#pragma omp atomic write
            err = 1;
        } else {
#pragma omp for schedule(static)
            for (long long q = 0; q < nlines; q++) {
                long long outer = q / stride, inner = q % stride;
                cx *base = data + outer * stride * n + inner;
                for (int j = 0; j < n; j++) line[j] = base[(long long)j * stride];
                fft_line(line, n, tw);
                for (int j = 0; j < n; j++) base[(long long)j * stride] = line[j];
            }
            free(line);
        }
    }
    free(tw);
    return err ? ORC_ENOMEM : ORC_OK;
}

/* full N-D transform; sign -1: unnormalised forward, +1: inverse with 1/P */
static int fft_nd(cx *data, const grid_t *g, int sign, int nthreads)
{
    for (int d = 0; d < g->ndim; d++) {
        int e = fft_axis(data, g, d, sign, nthreads);
        if (e) return e;
    }
    if (sign > 0) {
        double s = 1.0 / (double)g->P;
#pragma omp parallel for num_threads(nthreads) schedule(static)
        for (long long q = 0; q < g->P; q++) data[q] *= s;
    }
    return ORC_OK;
}

int orc_fft(double *data, int ndim, const int *n, int sign, int nthreads)
{
    grid_t g;
    if (!data || (sign != -1 && sign != 1) || grid_init(&g, ndim, n, NULL)) return ORC_EINVAL;
    return fft_nd((cx *)data, &g, sign, nthreads_or_default(nthreads));
}

/* brute-force O(P^2) DFT, same normalisation as orc_fft; for pinning only.
   The phase sum_d k_d x_d / n_d is reduced exactly in integers modulo P. */
int orc_dft_brute(const double *in, double *out, int ndim, const int *n, int sign)
{
    grid_t g;
    if (!in || !out || (sign != -1 && sign != 1) || grid_init(&g, ndim, n, NULL)) return ORC_EINVAL;
    const cx *a = (const cx *)in;
    cx *b = (cx *)out;
    long long P = g.P;
    for (long long kq = 0; kq < P; kq++) {
        cx acc = 0.0;
        for (long long xq = 0; xq < P; xq++) {
            long long m = 0;
            for (int d = 0; d < ndim; d++) {
                long long kd = (kq / g.stride[d]) % g.n[d];
                long long xd = (xq / g.stride[d]) % g.n[d];
                m += ((kd * xd) % g.n[d]) * (P / g.n[d]);
            }
            m %= P;
            double ang = 2.0 * M_PI * (double)m / (double)P;
            acc += a[xq] * (cos(ang) + (double)sign * sin(ang) * I);
        }
        b[kq] = (sign > 0) ? acc / (double)P : acc;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* local terms of Eq. (15)                                                  */
/* ------------------------------------------------------------------------ */

/* lp = {c_p, n_p, c_B, rho_f}; lp == NULL: Kerr term only */
typedef struct {
    int on;
    double cp, np, cb, floor;
} local_t;

static int local_init(local_t *lt, const double *lp)
{
    memset(lt, 0, sizeof(*lt));
    if (!lp) return ORC_OK;
    for (int i = 0; i < 4; i++)
        if (!isfinite(lp[i])) return ORC_EINVAL;
    lt->cp = lp[0];
    lt->np = lp[1];
    lt->cb = lp[2];
    lt->floor = lp[3];
    if (lt->floor < 0.0) return ORC_EINVAL;
    /* the pressure law is given for n = 1, n > 1 and n < 0 */
    if (lt->cp != 0.0 && lt->np >= 0.0 && lt->np < 1.0) return ORC_EINVAL;
    /* ln rho, rho^(n-1) with n < 1 and 1/sqrt(rho) need a positive floor */
    if (((lt->cp != 0.0 && lt->np <= 1.0) || lt->cb != 0.0) && !(lt->floor > 0.0)) return ORC_EINVAL;
    lt->on = lt->cp != 0.0 || lt->cb != 0.0;
    return ORC_OK;
}

/* polytropic pressure potential f_n of Eq. (15) */
static double poly_f(double rho, double n)
{
    return n == 1.0 ? log(rho) : n / (n - 1.0) * pow(rho, n - 1.0);
}

/* its antiderivative F_n (F_n' = f_n): the pressure energy density */
static double poly_F(double rho, double n)
{
    return n == 1.0 ? rho * log(rho) - rho : pow(rho, n) / (n - 1.0);
}

/* antiderivative of the floored potential f_n(max(rho, rho_f)) */
static double poly_G(double rho, double n, double rho_f)
{
    if (rho >= rho_f) return poly_F(rho, n);
    return poly_F(rho_f, n) + (rho - rho_f) * poly_f(rho_f, n);
}

/* lap(sqrt rho) = Re IDFT[-|k|^2 DFT sqrt(rho)] into lap (real), tmp scratch */
static int laplacian_of_sqrt(double *lap, const double *rho, cx *tmp, const grid_t *g, int nt)
{
#pragma omp parallel for num_threads(nt) schedule(static)
    for (long long q = 0; q < g->P; q++) tmp[q] = sqrt(rho[q]);
    int e = fft_nd(tmp, g, -1, nt);
    if (e) return e;
#pragma omp parallel for num_threads(nt) schedule(static)
    for (long long q = 0; q < g->P; q++) tmp[q] *= -k_squared(g, q);
    e = fft_nd(tmp, g, +1, nt);
    if (e) return e;
#pragma omp parallel for num_threads(nt) schedule(static)
    for (long long q = 0; q < g->P; q++) lap[q] = creal(tmp[q]);
    return ORC_OK;
}

/* lap(f) = Re IDFT[-|k|^2 DFT f] of a real field into lap, tmp scratch */
static int laplacian_into(double *lap, const double *f, cx *tmp, const grid_t *g, int nt)
{
#pragma omp parallel for num_threads(nt) schedule(static)
    for (long long q = 0; q < g->P; q++) tmp[q] = f[q];
    int e = fft_nd(tmp, g, -1, nt);
    if (e) return e;
#pragma omp parallel for num_threads(nt) schedule(static)
    for (long long q = 0; q < g->P; q++) tmp[q] *= -k_squared(g, q);
    e = fft_nd(tmp, g, +1, nt);
    if (e) return e;
#pragma omp parallel for num_threads(nt) schedule(static)
    for (long long q = 0; q < g->P; q++) lap[q] = creal(tmp[q]);
    return ORC_OK;
}

/* Position-dependent source coefficients and static potential (NULL: absent;
   gamma absent means gamma = 1, beta absent beta = 0, V absent V = 0). */
typedef struct {
    const double *gamma, *beta, *V;
} fields_t;

/* s = gamma rho + beta lap(rho) into s; tmp scratch */
static int source_into(double *s_out, const double *rho, cx *tmp, const fields_t *fl, const grid_t *g, int nt)
{
    if (fl->beta) {
        int e = laplacian_into(s_out, rho, tmp, g, nt);
        if (e) return e;
#pragma omp parallel for num_threads(nt) schedule(static)
        for (long long q = 0; q < g->P; q++) s_out[q] *= fl->beta[q];
    } else {
#pragma omp parallel for num_threads(nt) schedule(static)
        for (long long q = 0; q < g->P; q++) s_out[q] = 0.0;
    }
#pragma omp parallel for num_threads(nt) schedule(static)
    for (long long q = 0; q < g->P; q++) s_out[q] += (fl->gamma ? fl->gamma[q] : 1.0) * rho[q];
    return ORC_OK;
}

/* U = g rho + polytropic + Bohm terms (see the header); tmp scratch */
static int local_potential_into(double *U, const double *rho, cx *tmp, double gloc,
                                const local_t *lt, const grid_t *g, int nt)
{
#pragma omp parallel for num_threads(nt) schedule(static)
    for (long long q = 0; q < g->P; q++) U[q] = gloc * rho[q];
    if (!lt->on) return ORC_OK;
    if (lt->cp != 0.0) {
#pragma omp parallel for num_threads(nt) schedule(static)
        for (long long q = 0; q < g->P; q++) U[q] += lt->cp * poly_f(fmax(rho[q], lt->floor), lt->np);
    }
    if (lt->cb != 0.0) {
        double *lap = (double *)malloc(sizeof(double) * (size_t)g->P);
        if (!lap) return ORC_ENOMEM;
        int e = laplacian_of_sqrt(lap, rho, tmp, g, nt);
        if (!e) {
            const double sf = sqrt(lt->floor);
#pragma omp parallel for num_threads(nt) schedule(static)
            for (long long q = 0; q < g->P; q++)
                U[q] += lt->cb * lap[q] / (2.0 * fmax(sqrt(rho[q]), sf));
        }
        free(lap);
        return e;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* potential, sub-steps, evolution                                          */
/* ------------------------------------------------------------------------ */

/* phi = Re IDFT[ K DFT rho ] into tmp (complex scratch of P entries) */
static int potential_into(cx *tmp, const double *rho, const double *Kk,
                          const grid_t *g, int nt)
{
#pragma omp parallel for num_threads(nt) schedule(static)
    for (long long q = 0; q < g->P; q++) tmp[q] = rho[q];
    int e = fft_nd(tmp, g, -1, nt);
    if (e) return e;
#pragma omp parallel for num_threads(nt) schedule(static)
    for (long long q = 0; q < g->P; q++) tmp[q] *= Kk[q];
    return fft_nd(tmp, g, +1, nt);
}

static int potential_spec(const double *rho, double *phi, int ndim, const int *n,
                          const double *L, const kspec_t *ks, int nthreads)
{
    grid_t g;
    if (!rho || !phi || grid_init(&g, ndim, n, L) || kspec_check(ks)) return ORC_EINVAL;
    int nt = nthreads_or_default(nthreads);
    cx *tmp = (cx *)malloc(sizeof(cx) * (size_t)g.P);
    double *Kk = (double *)malloc(sizeof(double) * (size_t)g.P);
    int e = ORC_ENOMEM;
    if (tmp && Kk && !(e = kspec_table(Kk, ks, &g))) {
        e = potential_into(tmp, rho, Kk, &g, nt);
        if (!e)
            for (long long q = 0; q < g.P; q++) phi[q] = creal(tmp[q]);
    }
    free(tmp);
    free(Kk);
    return e;
}

int orc_potential(const double *rho, double *phi, int ndim, const int *n,
                  const double *L, const double *kp, int nthreads)
{
    kspec_t ks = {0, kp, 0.0, 0.0, 0.0};
    return potential_spec(rho, phi, ndim, n, L, &ks, nthreads);
}

/* phi of Eq. (2) with Eq. (1)'s coupling: Re IDFT[B D / (|k|^2 - C) DFT rho] */
int orc_potential_equation(const double *rho, double *phi, int ndim, const int *n,
                           const double *L, double B, double C, double D, int nthreads)
{
    kspec_t ks = {1, NULL, B, C, D};
    return potential_spec(rho, phi, ndim, n, L, &ks, nthreads);
}

/* kinetic sub-step L(h) with a precomputed propagator table prop[q] */
static int kinetic_step(cx *psi, const cx *prop, const grid_t *g, int nt)
{
    int e = fft_nd(psi, g, -1, nt);
    if (e) return e;
#pragma omp parallel for num_threads(nt) schedule(static)
    for (long long q = 0; q < g->P; q++) psi[q] *= prop[q];
    return fft_nd(psi, g, +1, nt);
}

/* nonlinear sub-step N(h): psi <- psi exp(i (U + phi + V) h), U the local
   potential, phi the potential of rho (or of the source s when source fields
   are given); src is scratch for s */
static int nonlinear_step(cx *psi, cx *tmp, double *rho, double *U, double *src, const double *Kk,
                          double gloc, const local_t *lt, const fields_t *fl, double h,
                          const grid_t *g, int nt)
{
#pragma omp parallel for num_threads(nt) schedule(static)
    for (long long q = 0; q < g->P; q++) {
        double re = creal(psi[q]), im = cimag(psi[q]);
        rho[q] = re * re + im * im;
    }
    int e = local_potential_into(U, rho, tmp, gloc, lt, g, nt);
    if (e) return e;
    const double *s = rho;
    if (fl && (fl->gamma || fl->beta)) {
        if ((e = source_into(src, rho, tmp, fl, g, nt))) return e;
        s = src;
    }
    e = potential_into(tmp, s, Kk, g, nt);
    if (e) return e;
#pragma omp parallel for num_threads(nt) schedule(static)
    for (long long q = 0; q < g->P; q++) {
        double th = (U[q] + creal(tmp[q]) + (fl && fl->V ? fl->V[q] : 0.0)) * h;
        psi[q] *= cos(th) + sin(th) * I;
    }
    return ORC_OK;
}

/*
 * Evolve psi (interleaved complex128, C-order) by nsteps symmetric steps.
 *   kp = {c_N, c_Y, m_Y, c_0};  a = kinetic coefficient; g = local coefficient.
 *   merged = 0: each step is literally L(dz/2) N(dz) L(dz/2).
 *   merged = 1: L(dz/2) [N(dz) L(dz)]^(n-1) N(dz) L(dz/2), algebraically the
 *               same product of operators (L(h1) L(h2) = L(h1 + h2) exactly).
 * Returns 0 on success.
 */
static int evolve_spec(double *psi_io, int ndim, const int *n, const double *L,
                       const kspec_t *ks, double a, double gloc, const double *lp,
                       const fields_t *fl, double dz, long long nsteps, int merged, int nthreads)
{
    grid_t g;
    local_t lt;
    if (!psi_io || grid_init(&g, ndim, n, L) || nsteps < 0) return ORC_EINVAL;
    if (local_init(&lt, lp) || kspec_check(ks)) return ORC_EINVAL;
    if (!isfinite(dz) || !isfinite(a) || !isfinite(gloc)) return ORC_EINVAL;
    if (nsteps == 0) return ORC_OK;
    int nt = nthreads_or_default(nthreads);
    cx *psi = (cx *)psi_io;
    size_t P = (size_t)g.P;
    cx *half = (cx *)malloc(sizeof(cx) * P);
    cx *full = (cx *)malloc(sizeof(cx) * P);
    cx *tmp = (cx *)malloc(sizeof(cx) * P);
    double *Kk = (double *)malloc(sizeof(double) * P);
    double *rho = (double *)malloc(sizeof(double) * P);
    double *U = (double *)malloc(sizeof(double) * P);
    double *src = (double *)malloc(sizeof(double) * P);
    int e = ORC_ENOMEM;
    if (!half || !full || !tmp || !Kk || !rho || !U || !src) goto done;
    if ((e = kspec_table(Kk, ks, &g))) goto done;
#pragma omp parallel for num_threads(nt) schedule(static)
    for (long long q = 0; q < g.P; q++) {
        double k2 = k_squared(&g, q);
        double th_h = -a * k2 * dz * 0.5, th_f = -a * k2 * dz;
        half[q] = cos(th_h) + sin(th_h) * I;
        full[q] = cos(th_f) + sin(th_f) * I;
    }
    if (!merged) {
        for (long long s = 0; s < nsteps; s++) {
            if ((e = kinetic_step(psi, half, &g, nt))) goto done;
            if ((e = nonlinear_step(psi, tmp, rho, U, src, Kk, gloc, &lt, fl, dz, &g, nt))) goto done;
            if ((e = kinetic_step(psi, half, &g, nt))) goto done;
        }
    } else {
        if ((e = kinetic_step(psi, half, &g, nt))) goto done;
        for (long long s = 0; s < nsteps; s++) {
            if ((e = nonlinear_step(psi, tmp, rho, U, src, Kk, gloc, &lt, fl, dz, &g, nt))) goto done;
            if ((e = kinetic_step(psi, s + 1 < nsteps ? full : half, &g, nt))) goto done;
        }
    }
    e = ORC_OK;
done:
    free(half);
    free(full);
    free(tmp);
    free(Kk);
    free(rho);
    free(U);
    free(src);
    return e;
}

int orc_evolve_local(double *psi_io, int ndim, const int *n, const double *L,
                     const double *kp, double a, double gloc, const double *lp, double dz,
                     long long nsteps, int merged, int nthreads)
{
    kspec_t ks = {0, kp, 0.0, 0.0, 0.0};
    return evolve_spec(psi_io, ndim, n, L, &ks, a, gloc, lp, NULL, dz, nsteps, merged, nthreads);
}

/* orc_evolve_local with position-dependent source fields and a static
   potential (any of gamma, beta, V may be NULL) */
int orc_evolve_fields(double *psi_io, int ndim, const int *n, const double *L,
                      const double *kp, double a, double gloc, const double *lp,
                      const double *gamma, const double *beta, const double *V, double dz,
                      long long nsteps, int merged, int nthreads)
{
    kspec_t ks = {0, kp, 0.0, 0.0, 0.0};
    fields_t fl = {gamma, beta, V};
    return evolve_spec(psi_io, ndim, n, L, &ks, a, gloc, lp, &fl, dz, nsteps, merged, nthreads);
}

/* phi = Re IDFT[K DFT s], s = gamma rho + beta lap(rho) */
int orc_potential_fields(const double *rho, double *phi, int ndim, const int *n, const double *L,
                         const double *kp, const double *gamma, const double *beta, int nthreads)
{
    grid_t g;
    kspec_t ks = {0, kp, 0.0, 0.0, 0.0};
    if (!rho || !phi || grid_init(&g, ndim, n, L) || kspec_check(&ks)) return ORC_EINVAL;
    int nt = nthreads_or_default(nthreads);
    fields_t fl = {gamma, beta, NULL};
    cx *tmp = (cx *)malloc(sizeof(cx) * (size_t)g.P);
    double *Kk = (double *)malloc(sizeof(double) * (size_t)g.P);
    double *s = (double *)malloc(sizeof(double) * (size_t)g.P);
    int e = ORC_ENOMEM;
    if (tmp && Kk && s && !(e = kspec_table(Kk, &ks, &g)) && !(e = source_into(s, rho, tmp, &fl, &g, nt)) &&
        !(e = potential_into(tmp, s, Kk, &g, nt)))
        for (long long q = 0; q < g.P; q++) phi[q] = creal(tmp[q]);
    free(tmp);
    free(Kk);
    free(s);
    return e;
}

/*
 * Fields of the pure non-minimal coupling, Eq. (9)-(11), on the grid: with
 * r the (minimum-image) distance from the centre c and u = (r0/(r + r0))^lambda,
 *   gamma = (1 - u)/2,   beta = lambda u / (r + r0),   phi_C = ln(1 - u),
 * and V = -phi_C / nu (this file's sign and scale); phi_C diverges at r = 0, so
 * it takes r = max(r, r_min).
 */
int orc_nmc_fields(int ndim, const int *n, const double *L, double lambda, double r0, double nu,
                   const double *center, double r_min, double *gamma, double *beta, double *V)
{
    grid_t g;
    if (grid_init(&g, ndim, n, L) || !center || !gamma || !beta || !V) return ORC_EINVAL;
    if (!(lambda > 0.0) || !(r0 > 0.0) || !(nu != 0.0) || !(r_min > 0.0)) return ORC_EINVAL;
    for (long long q = 0; q < g.P; q++) {
        double r2 = 0.0;
        for (int d = 0; d < g.ndim; d++) {
            int j = (int)((q / g.stride[d]) % g.n[d]);
            double x = -0.5 * g.L[d] + j * g.L[d] / g.n[d] - center[d];
            x -= g.L[d] * floor(x / g.L[d] + 0.5);   /* minimum image */
            r2 += x * x;
        }
        double r = sqrt(r2);
        double u = pow(r0 / (r + r0), lambda);
        gamma[q] = 0.5 * (1.0 - u);
        beta[q] = lambda * u / (r + r0);
        double rc = fmax(r, r_min);
        V[q] = -log(1.0 - pow(r0 / (rc + r0), lambda)) / nu;
    }
    return ORC_OK;
}

/*
 * Eq. (1)-(2) with their own constants: i psi_t = A lap psi + B phi psi
 * + G psi, lap phi + C phi = D rho, with G = -(g rho + local terms), i.e.
 * a = -A and K = B D / (|k|^2 - C) in this file's form.
 */
int orc_evolve_equation(double *psi_io, int ndim, const int *n, const double *L,
                        double A, double B, double C, double D, double gloc, const double *lp,
                        double dz, long long nsteps, int merged, int nthreads)
{
    kspec_t ks = {1, NULL, B, C, D};
    return evolve_spec(psi_io, ndim, n, L, &ks, -A, gloc, lp, NULL, dz, nsteps, merged, nthreads);
}

/* orc_evolve_local with the Kerr term only */
int orc_evolve(double *psi_io, int ndim, const int *n, const double *L,
               const double *kp, double a, double gloc, double dz,
               long long nsteps, int merged, int nthreads)
{
    return orc_evolve_local(psi_io, ndim, n, L, kp, a, gloc, NULL, dz, nsteps, merged, nthreads);
}

/* The local potential U of psi (see the header) into U_out (P doubles). */
int orc_local_potential(const double *psi_in, int ndim, const int *n, const double *L,
                        double gloc, const double *lp, double *U_out, int nthreads)
{
    grid_t g;
    local_t lt;
    if (!psi_in || !U_out || grid_init(&g, ndim, n, L) || local_init(&lt, lp)) return ORC_EINVAL;
    int nt = nthreads_or_default(nthreads);
    const cx *psi = (const cx *)psi_in;
    cx *tmp = (cx *)malloc(sizeof(cx) * (size_t)g.P);
    double *rho = (double *)malloc(sizeof(double) * (size_t)g.P);
    int e = ORC_ENOMEM;
    if (tmp && rho) {
        for (long long q = 0; q < g.P; q++) {
            double re = creal(psi[q]), im = cimag(psi[q]);
            rho[q] = re * re + im * im;
        }
        e = local_potential_into(U_out, rho, tmp, gloc, &lt, &g, nt);
    }
    free(tmp);
    free(rho);
    return e;
}

/*
 * Observables of psi: out = {M, E_kin, E_loc, E_nl, E_total, E_p, E_B} with
 *   M     = dV sum |psi|^2
 *   E_kin = a dV / P sum_k |k|^2 |psi_hat_k|^2      (= a dV sum |grad psi|^2)
 *   E_loc = -(g/2) dV sum rho^2 + E_p + E_B
 *   E_p   = -c_p dV sum G_n(rho),  G_n' = f_n(max(rho, rho_f))
 *   E_B   = (c_B/2) dV sum |grad s|^2 = -(c_B/2) dV sum s lap(s),  s = sqrt(rho)
 *   E_nl  = -(1/2) dV sum rho phi
 * (with a static potential V, E_loc also holds -dV sum V rho)
 * E_total is the Hamiltonian of the equation above: its variation with
 * respect to conj(psi) is -a lap(psi) - U psi - phi psi (for the Bohm part
 * where rho >= rho_f, since the variation of sum |grad s|^2 with respect to rho
 * is -lap(s)/s).  lp == NULL: E_p = E_B = 0.
 */
static int observables_spec(const double *psi_in, int ndim, const int *n, const double *L,
                            const kspec_t *ks, double a, double gloc, const double *lp,
                            const double *V, double *out, int nthreads)
{
    grid_t g;
    local_t lt;
    if (!psi_in || !out || grid_init(&g, ndim, n, L)) return ORC_EINVAL;
    if (local_init(&lt, lp) || kspec_check(ks)) return ORC_EINVAL;
    int nt = nthreads_or_default(nthreads);
    const cx *psi = (const cx *)psi_in;
    size_t P = (size_t)g.P;
    double dV = 1.0;
    for (int d = 0; d < g.ndim; d++) dV *= g.L[d] / g.n[d];
    cx *tmp = (cx *)malloc(sizeof(cx) * P);
    double *Kk = (double *)malloc(sizeof(double) * P);
    double *rho = (double *)malloc(sizeof(double) * P);
    double *lap = NULL;
    int e = ORC_ENOMEM;
    if (!tmp || !Kk || !rho) goto done;
    double mass = 0.0, ekin = 0.0, eloc = 0.0, enl = 0.0;
    if ((e = kspec_table(Kk, ks, &g))) goto done;
    for (long long q = 0; q < g.P; q++) {
        double re = creal(psi[q]), im = cimag(psi[q]);
        rho[q] = re * re + im * im;
        mass += rho[q];
        eloc += rho[q] * rho[q];
        tmp[q] = psi[q];
    }
    if ((e = fft_nd(tmp, &g, -1, nt))) goto done;
    for (long long q = 0; q < g.P; q++) {
        double re = creal(tmp[q]), im = cimag(tmp[q]);
        ekin += k_squared(&g, q) * (re * re + im * im);
    }
    if ((e = potential_into(tmp, rho, Kk, &g, nt))) goto done;
    for (long long q = 0; q < g.P; q++) enl += rho[q] * creal(tmp[q]);
    double ep = 0.0, eb = 0.0;
    if (lt.cp != 0.0) {
        for (long long q = 0; q < g.P; q++) ep += poly_G(rho[q], lt.np, lt.floor);
        ep *= -lt.cp * dV;
    }
    if (lt.cb != 0.0) {
        lap = (double *)malloc(sizeof(double) * P);
        e = ORC_ENOMEM;
        if (!lap) goto done;
        if ((e = laplacian_of_sqrt(lap, rho, tmp, &g, nt))) goto done;
        for (long long q = 0; q < g.P; q++) eb += sqrt(rho[q]) * lap[q];
        eb *= -0.5 * lt.cb * dV;
    }
    out[0] = dV * mass;
    out[1] = a * dV / (double)g.P * ekin;
    double ev = 0.0;   /* static potential: -dV sum V rho */
    if (V) {
        for (long long q = 0; q < g.P; q++) ev += V[q] * rho[q];
        ev *= -dV;
    }
    out[2] = -0.5 * gloc * dV * eloc + ep + eb + ev;
    out[3] = -0.5 * dV * enl;
    out[4] = out[1] + out[2] + out[3];
    out[5] = ep;
    out[6] = eb;
    e = ORC_OK;
done:
    free(tmp);
    free(Kk);
    free(rho);
    free(lap);
    return e;
}

int orc_observables_local(const double *psi_in, int ndim, const int *n, const double *L,
                          const double *kp, double a, double gloc, const double *lp,
                          double *out, int nthreads)
{
    kspec_t ks = {0, kp, 0.0, 0.0, 0.0};
    return observables_spec(psi_in, ndim, n, L, &ks, a, gloc, lp, NULL, out, nthreads);
}

/* orc_observables_local with a static potential V (the local energy then
   includes -dV sum V rho); V == NULL: none */
int orc_observables_vext(const double *psi_in, int ndim, const int *n, const double *L,
                         const double *kp, double a, double gloc, const double *lp, const double *V,
                         double *out, int nthreads)
{
    kspec_t ks = {0, kp, 0.0, 0.0, 0.0};
    return observables_spec(psi_in, ndim, n, L, &ks, a, gloc, lp, V, out, nthreads);
}

/* observables of Eq. (1)-(2) with their own constants (a = -A) */
int orc_observables_equation(const double *psi_in, int ndim, const int *n, const double *L,
                             double A, double B, double C, double D, double gloc, const double *lp,
                             double *out, int nthreads)
{
    kspec_t ks = {1, NULL, B, C, D};
    return observables_spec(psi_in, ndim, n, L, &ks, -A, gloc, lp, NULL, out, nthreads);
}

/* orc_observables_local with the Kerr term only; out has 5 entries */
int orc_observables(const double *psi_in, int ndim, const int *n, const double *L,
                    const double *kp, double a, double gloc, double *out, int nthreads)
{
    double o[7];
    int e = orc_observables_local(psi_in, ndim, n, L, kp, a, gloc, NULL, o, nthreads);
    if (!e)
        for (int i = 0; i < 5; i++) out[i] = o[i];
    return e;
}

int orc_max_threads(void) { return omp_get_max_threads(); }
