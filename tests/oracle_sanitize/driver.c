/*
 * Sanitizer driver for the CPU oracle (test harness; never part of the
 * library).  Built with gcc -fsanitize=address,undefined together with the
 * oracle's C sources, it runs the oracle's entry points on the cells of an
 * input file and prints every result at full precision, so that the test can
 * compare them with the regular build.
 *
 * usage: driver MECH CELLS DT RTOL
 * CELLS: first line "n ns", then per cell "T p Y_0 ... Y_{ns-1}".
 * Output: per cell "T_final status" then the ns final mass fractions, and the
 * RHS and Jacobian of the first cell at its initial state.
 */
#include <stdio.h>
#include <stdlib.h>

const char *oracle_last_error(void);
void *oracle_load(const char *path);
void oracle_free(void *h);
void oracle_info(void *h, int *ns, int *nr, int *ne);
void oracle_state_from_TPY(void *h, long n, const double *T, const double *p, const double *Y,
                           double *rho, double *e);
int oracle_T_from_e(void *h, double e, const double *Y, double Tguess, double *T);
void oracle_rhs(void *h, double rho, const double *y, double *f);
void oracle_jac(void *h, double rho, const double *y, double *J);
long oracle_integrate(void *h, long ncell, const double *rho, const double *e, double *Y, long ldY,
                      double *T, double dt, double rtol, double atol, long max_steps, int nthreads,
                      unsigned char *status, long *cstats);

int main(int argc, char **argv) {
    if (argc != 5) {
        fprintf(stderr, "usage: driver MECH CELLS DT RTOL\n");
        return 2;
    }
    void *h = oracle_load(argv[1]);
    if (!h) {
        fprintf(stderr, "load: %s\n", oracle_last_error());
        return 2;
    }
    int ns, nr, ne;
    oracle_info(h, &ns, &nr, &ne);
    FILE *f = fopen(argv[2], "r");
    long n;
    int nsf;
    if (!f || fscanf(f, "%ld %d", &n, &nsf) != 2 || nsf != ns || n <= 0) {
        fprintf(stderr, "bad cell file\n");
        return 2;
    }
    double *T = malloc(sizeof(double) * n), *p = malloc(sizeof(double) * n);
    double *Y = malloc(sizeof(double) * n * ns), *rho = malloc(sizeof(double) * n);
    double *e = malloc(sizeof(double) * n), *T0 = malloc(sizeof(double) * n);
    for (long i = 0; i < n; i++) {
        if (fscanf(f, "%lf %lf", &T[i], &p[i]) != 2) return 2;
        for (int k = 0; k < ns; k++)
            if (fscanf(f, "%lf", &Y[(size_t)k * n + i]) != 1) return 2;
    }
    fclose(f);
    const double dt = atof(argv[3]), rtol = atof(argv[4]);
    oracle_state_from_TPY(h, n, T, p, Y, rho, e);
    /* temperature inversion from a guess 300 K off */
    double *y = malloc(sizeof(double) * (ns + 1));
    for (long i = 0; i < n; i++) {
        for (int k = 0; k < ns; k++) y[k] = Y[(size_t)k * n + i];
        if (oracle_T_from_e(h, e[i], y, T[i] + 300.0, &T0[i]) != 0) return 3;
    }
    /* RHS and Jacobian of the first cell */
    double *rhs = malloc(sizeof(double) * (ns + 1)), *J = malloc(sizeof(double) * (ns + 1) * (ns + 1));
    for (int k = 0; k < ns; k++) y[k] = Y[k * n];
    y[ns] = T0[0];
    oracle_rhs(h, rho[0], y, rhs);
    oracle_jac(h, rho[0], y, J);
    unsigned char *st = malloc(n);
    long *cs = malloc(sizeof(long) * 5 * n);
    oracle_integrate(h, n, rho, e, Y, n, T0, dt, rtol, 1e-20, 200000, 1, st, cs);
    for (long i = 0; i < n; i++) {
        printf("%.17g %d", T0[i], (int)st[i]);
        for (int k = 0; k < ns; k++) printf(" %.17g", Y[(size_t)k * n + i]);
        printf("\n");
    }
    for (int k = 0; k <= ns; k++) printf("%.17g ", rhs[k]);
    printf("\n");
    for (int k = 0; k < (ns + 1) * (ns + 1); k++) printf("%.17g ", J[k]);
    printf("\n");
    free(T); free(p); free(Y); free(rho); free(e); free(T0); free(y); free(rhs); free(J); free(st); free(cs);
    oracle_free(h);
    return 0;
}
