/* Sanitizer run of the FP64 oracle (built with -fsanitize=address,undefined
   by tests/test_sanitizers.py): every entry point on small 1-D..3-D grids,
   with the options that take other code paths (literal and merged steps,
   local terms, Eq. (1)-(2) constants, source fields, observables).  Any
   invalid access or undefined behaviour aborts the run; the printed sums let
   the test check that the calls did their work. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

int orc_fft(double *data, int ndim, const int *n, int sign, int nthreads);
int orc_dft_brute(const double *in, double *out, int ndim, const int *n, int sign);
int orc_potential(const double *rho, double *phi, int ndim, const int *n, const double *L, const double *kp,
                  int nthreads);
int orc_evolve(double *psi_io, int ndim, const int *n, const double *L, const double *kp, double a, double gloc,
               double dz, long long nsteps, int merged, int nthreads);
int orc_evolve_local(double *psi_io, int ndim, const int *n, const double *L, const double *kp, double a,
                     double gloc, const double *lp, double dz, long long nsteps, int merged, int nthreads);
int orc_evolve_fields(double *psi_io, int ndim, const int *n, const double *L, const double *kp, double a,
                      double gloc, const double *lp, const double *gamma, const double *beta, const double *V,
                      double dz, long long nsteps, int merged, int nthreads);
int orc_evolve_equation(double *psi_io, int ndim, const int *n, const double *L, double A, double B, double C,
                        double D, double gloc, const double *lp, double dz, long long nsteps, int merged,
                        int nthreads);
int orc_observables_local(const double *psi_in, int ndim, const int *n, const double *L, const double *kp,
                          double a, double gloc, const double *lp, double *out, int nthreads);
int orc_nmc_fields(int ndim, const int *n, const double *L, double lambda, double r0, double nu,
                   const double *center, double r_min, double *gamma, double *beta, double *V);

static void lump(double *psi, int ndim, const int *n, const double *L)
{
    long long P = 1;
    for (int d = 0; d < ndim; ++d) P *= n[d];
    for (long long q = 0; q < P; ++q) {
        long long rem = q;
        double r2 = 0.0, ph = 0.0;
        for (int d = ndim - 1; d >= 0; --d) {
            const int j = (int)(rem % n[d]);
            rem /= n[d];
            const double x = -0.5 * L[d] + j * L[d] / n[d];
            r2 += x * x;
            ph += 0.3 * (d + 1) * x;
        }
        const double a = exp(-r2 / (0.04 * L[0] * L[0]));
        psi[2 * q] = a * cos(ph);
        psi[2 * q + 1] = a * sin(ph);
    }
}

int main(void)
{
    int fails = 0;
    double sum = 0.0;
    const int shapes[4][3] = {{16, 1, 1}, {8, 16, 1}, {4, 8, 16}, {32, 8, 1}};
    const int dims[4] = {1, 2, 3, 2};
    for (int s = 0; s < 4; ++s) {
        const int nd = dims[s];
        const int *n = shapes[s];
        long long P = 1;
        double L[3];
        for (int d = 0; d < nd; ++d) {
            P *= n[d];
            L[d] = 2.0 * n[d];
        }
        double *a = malloc(sizeof(double) * 2 * P), *b = malloc(sizeof(double) * 2 * P);
        double *c = malloc(sizeof(double) * 2 * P), *rho = malloc(sizeof(double) * P);
        double *phi = malloc(sizeof(double) * P), *g = malloc(sizeof(double) * P);
        double *be = malloc(sizeof(double) * P), *V = malloc(sizeof(double) * P);
        lump(a, nd, n, L);
        for (long long q = 0; q < 2 * P; ++q) c[q] = a[q];
        fails += orc_dft_brute(a, b, nd, n, -1) != 0;
        fails += orc_fft(c, nd, n, -1, 2) != 0;
        for (long long q = 0; q < 2 * P; ++q) fails += fabs(b[q] - c[q]) > 1e-10;
        fails += orc_fft(c, nd, n, 1, 1) != 0;
        for (long long q = 0; q < P; ++q) rho[q] = a[2 * q] * a[2 * q] + a[2 * q + 1] * a[2 * q + 1];
        const double kp[4] = {1.0, 0.3, 0.2, 0.1};
        fails += orc_potential(rho, phi, nd, n, L, kp, 2) != 0;
        for (int merged = 0; merged < 2; ++merged) {
            for (long long q = 0; q < 2 * P; ++q) b[q] = a[q];
            fails += orc_evolve(b, nd, n, L, kp, 0.5, -0.5, 1e-3, 3, merged, 2) != 0;
            sum += b[0] + b[2 * P - 1];
        }
        const double lp[4] = {-1.02, 1.0, -1.0, 1e-10}, lp2[4] = {-0.5, 2.5, -1.0, 1e-8};
        for (long long q = 0; q < 2 * P; ++q) b[q] = a[q] + 1e-3;
        fails += orc_evolve_local(b, nd, n, L, kp, 0.5, 0.0, lp, 1e-3, 2, 1, 2) != 0;
        fails += orc_evolve_local(b, nd, n, L, kp, 0.5, 0.0, lp2, 1e-3, 2, 0, 1) != 0;
        const double ctr[3] = {0.0, 0.0, 0.0};
        fails += orc_nmc_fields(nd, n, L, 1.0, 2.0, 1.0, ctr, 0.5, g, be, V) != 0;
        const double kn[4] = {1.0, 0.0, 0.0, 0.0};
        fails += orc_evolve_fields(b, nd, n, L, kn, 0.5, 0.0, lp, g, be, V, 1e-3, 2, 1, 2) != 0;
        fails += orc_evolve_fields(b, nd, n, L, kn, 0.5, 0.0, NULL, NULL, NULL, V, 1e-3, 2, 0, 1) != 0;
        fails += orc_evolve_equation(b, nd, n, L, -0.5, -1.0, -0.2, -0.4, 0.1, NULL, 1e-3, 2, 1, 2) != 0;
        double obs[7];
        fails += orc_observables_local(b, nd, n, L, kp, 0.5, -0.5, lp, obs, 2) != 0;
        for (int i = 0; i < 7; ++i) sum += obs[i];
        free(a); free(b); free(c); free(rho); free(phi); free(g); free(be); free(V);
    }
    printf("fails %d sum %.6e\n", fails, sum);
    return fails != 0 || !isfinite(sum);
}
