/* Host driver for the sanitizer build of the oracle's C core: cyclic solves
 * of every size the oracle accepts and a Crank-Nicolson run over many modes,
 * checked against the dense definitions (residuals). */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_cyclic_solve(int n, const double *diag, double off, const double *rhs, double *x);
int oracle_cn_modes(int N, long nmodes, const double *pot, double beta, double tau, int nsteps, double *re,
                    double *im);

int main(void)
{
    double worst = 0.0;
    for (int n = 3; n <= 70; ++n) {
        double *d = malloc(sizeof(double) * n), *b = malloc(sizeof(double) * n), *x = malloc(sizeof(double) * n);
        for (int i = 0; i < n; ++i) {
            d[i] = 3.0 + 0.1 * i;
            b[i] = sin(1.0 + i);
        }
        const double off = -0.7;
        if (oracle_cyclic_solve(n, d, off, b, x) != 0) return 1;
        for (int i = 0; i < n; ++i) {
            const double r = d[i] * x[i] + off * (x[(i + 1) % n] + x[(i + n - 1) % n]) - b[i];
            worst = fmax(worst, fabs(r));
        }
        free(d);
        free(b);
        free(x);
    }
    const int N = 17;
    const long nm = 300;
    double *pot = malloc(sizeof(double) * N * nm), *re = malloc(sizeof(double) * N * nm),
           *im = malloc(sizeof(double) * N * nm);
    for (long i = 0; i < N * nm; ++i) {
        pot[i] = 5.0 * fabs(sin(0.3 * i));
        re[i] = cos(0.1 * i);
        im[i] = sin(0.2 * i);
    }
    if (oracle_cn_modes(N, nm, pot, 1.5, 0.01, 25, re, im) != 0) return 2;
    printf("oracle core: worst cyclic residual %.3e, CN ran on %ld modes\n", worst, nm);
    free(pot);
    free(re);
    free(im);
    return worst < 1e-12 ? 0 : 3;
}
