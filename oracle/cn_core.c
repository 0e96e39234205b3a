/*
 * FP64 reference core: Crank-Nicolson time stepping of the decoupled per-mode
 * systems of the semi-discrete SE(2,N) diffusion.
 *
 * TEST INFRASTRUCTURE ONLY.  This file belongs to the oracle: it is compiled
 * and called by the tests, the smoke check and the benchmark's CPU-baseline
 * leg, never by the library it checks, and shares no code with it.
 *
 * What it computes (paper, Sec. "Numerical treatment of the diffusion
 * equation", Theorem 2 and the remark that follows it): after the FFT over
 * (Z/MZ)^2 every spatial frequency (k,l) carries an N-vector that obeys
 *     d psi/dt = A psi,   A = beta*L - diag(pot_r),
 * where L is the cyclic second difference over Z_N (-2 on the diagonal, +1 at
 * r-1 and r+1 modulo N; the jump generator of Sec. "The semi-discrete
 * diffusion operator") and pot_r = M*(cos(e_r) s_k + sin(e_r) s_l)^2 is the
 * diagonal potential.  Each Crank-Nicolson step with tau = T/n forms
 *     b = (I + tau/2 A) x
 * and solves (I - tau/2 A) x' = b.  The system matrix is tridiagonal plus two
 * corner entries (the periodic coupling in r), so it is solved as a
 * tridiagonal system plus a rank-one Sherman-Morrison correction, the kind of
 * cyclic solver the paper recommends.  The matrix is strictly diagonally
 * dominant, so the tridiagonal elimination needs no pivoting.
 *
 * Real and imaginary parts are independent real right-hand sides because A
 * is real.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* Solve the cyclic tridiagonal system with constant off-diagonal `off`
 * (including both corners) and diagonal `diag` for one right-hand side.
 * Work arrays cp and work have length n.  Returns 0, or -1 if a pivot vanishes.
 *
 * Sherman-Morrison: B = T + u v^T with u = (g,0,..,0,off), v = (1,0,..,0,off/g),
 * g = -diag[0].  T is B with T[0][0] = diag[0]-g, T[n-1][n-1] = diag[n-1]-off^2/g
 * and no corners.  x = y - (v.y / (1 + v.z)) z with T y = rhs, T z = u. */
static int tri_solve(int n, const double *diag, double off, double g,
                     const double *rhs, double *x, double *cp, double *work)
{
    /* Thomas elimination for T (constant sub/super diagonal `off`). */
    double d0 = diag[0] - g;
    if (d0 == 0.0) return -1;
    cp[0] = off / d0;
    work[0] = rhs[0] / d0;
    for (int i = 1; i < n; ++i) {
        double di = diag[i];
        if (i == n - 1) di -= off * off / g;
        double den = di - off * cp[i - 1];
        if (den == 0.0) return -1;
        cp[i] = off / den;
        work[i] = (rhs[i] - off * work[i - 1]) / den;
    }
    x[n - 1] = work[n - 1];
    for (int i = n - 2; i >= 0; --i) x[i] = work[i] - cp[i] * x[i + 1];
    return 0;
}

/* One cyclic solve, exposed for the oracle's own checks. */
int oracle_cyclic_solve(int n, const double *diag, double off, const double *rhs,
                        double *x)
{
    if (n < 3) return -1;
    double *buf = (double *)malloc(sizeof(double) * 5 * (size_t)n);
    if (!buf) return -2;
    double *cp = buf, *work = buf + n, *u = buf + 2 * n, *z = buf + 3 * n, *y = buf + 4 * n;
    double g = -diag[0];
    memset(u, 0, sizeof(double) * n);
    u[0] = g;
    u[n - 1] = off;
    int rc = tri_solve(n, diag, off, g, u, z, cp, work);
    if (rc == 0) rc = tri_solve(n, diag, off, g, rhs, y, cp, work);
    if (rc == 0) {
        double vz = z[0] + (off / g) * z[n - 1];
        double vy = y[0] + (off / g) * y[n - 1];
        double fac = vy / (1.0 + vz);
        for (int i = 0; i < n; ++i) x[i] = y[i] - fac * z[i];
    }
    free(buf);
    return rc;
}

/* Crank-Nicolson over `nsteps` steps for `nmodes` independent modes.
 * pot : [nmodes][N] potentials M*a_r^2 for each mode
 * re, im : [nmodes][N] spectra, overwritten with the result at T = nsteps*tau.
 * Returns 0 on success, -1 on a vanishing pivot, -2 on allocation failure. */
int oracle_cn_modes(int N, long nmodes, const double *pot, double beta, double tau,
                    int nsteps, double *re, double *im)
{
    if (N < 3 || nsteps < 0) return -1;
    int status = 0;
#pragma omp parallel
    {
        double *buf = (double *)malloc(sizeof(double) * 9 * (size_t)N);
        if (!buf) {
#pragma omp atomic write
            status = -2;
        }
#pragma omp for schedule(static)
        for (long m = 0; m < nmodes; ++m) {
            if (!buf) continue;
            double *diag = buf, *cp = buf + N, *work = buf + 2 * N, *u = buf + 3 * N;
            double *z = buf + 4 * N, *rhs = buf + 5 * N, *y = buf + 6 * N, *xr = buf + 7 * N,
                   *xi = buf + 8 * N;
            const double *p = pot + (size_t)m * N;
            const double off = -0.5 * tau * beta;
            for (int r = 0; r < N; ++r) diag[r] = 1.0 + tau * beta + 0.5 * tau * p[r];
            const double g = -diag[0];
            for (int r = 0; r < N; ++r) u[r] = 0.0;
            u[0] = g;
            u[N - 1] = off;
            if (tri_solve(N, diag, off, g, u, z, cp, work) != 0) {
#pragma omp atomic write
                status = -1;
                continue;
            }
            const double vz = z[0] + (off / g) * z[N - 1];
            for (int r = 0; r < N; ++r) {
                xr[r] = re[(size_t)m * N + r];
                xi[r] = im[(size_t)m * N + r];
            }
            for (int s = 0; s < nsteps; ++s) {
                for (int part = 0; part < 2; ++part) {
                    double *x = part ? xi : xr;
                    /* b = (I + tau/2 A) x */
                    for (int r = 0; r < N; ++r) {
                        int rm = (r + N - 1) % N, rp = (r + 1) % N;
                        double ax = beta * (x[rm] - 2.0 * x[r] + x[rp]) - p[r] * x[r];
                        rhs[r] = x[r] + 0.5 * tau * ax;
                    }
                    tri_solve(N, diag, off, g, rhs, y, cp, work);
                    double vy = y[0] + (off / g) * y[N - 1];
                    double fac = vy / (1.0 + vz);
                    for (int r = 0; r < N; ++r) x[r] = y[r] - fac * z[r];
                }
            }
            for (int r = 0; r < N; ++r) {
                re[(size_t)m * N + r] = xr[r];
                im[(size_t)m * N + r] = xi[r];
            }
        }
        free(buf);
    }
    return status;
}

#ifdef _OPENMP
#include <omp.h>
#endif
/* Number of OpenMP threads the mode loop uses (1 without OpenMP). */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Set the number of OpenMP threads of the mode loop (no effect without OpenMP). */
void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
