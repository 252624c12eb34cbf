/*
 * Oracle driver and exported entry points (test infrastructure; see
 * oracle.h).  Every cell is integrated independently over [0, dt] with
 * rho and e constant (Strang-split chemistry substep, Sec. 2.1); OpenMP
 * spreads cells over host threads.  The oracle has no skip rule: cold
 * cells are integrated like any other.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    const omech_t *m;
    double rho;
} cell_ctx_t;

static void cell_rhs(void *c, double t, const double *y, double *f) {
    (void)t;
    cell_ctx_t *cc = (cell_ctx_t *)c;
    o_rhs(cc->m, cc->rho, y, f);
}
static void cell_jac(void *c, double t, const double *y, double *J) {
    (void)t;
    cell_ctx_t *cc = (cell_ctx_t *)c;
    o_jac(cc->m, cc->rho, y, J);
}

static char g_err[512];

const char *oracle_last_error(void) { return g_err; }

void *oracle_load(const char *path) {
    omech_t *m = NULL;
    if (omech_load(path, &m, g_err, sizeof g_err) != 0) return NULL;
    return m;
}

void oracle_free(void *h) { omech_free((omech_t *)h); }

void oracle_info(void *h, int *ns, int *nr, int *ne) {
    omech_t *m = (omech_t *)h;
    *ns = m->ns;
    *nr = m->nr;
    *ne = m->ne;
}

const char *oracle_species_name(void *h, int k) { return ((omech_t *)h)->sp[k]; }
const char *oracle_element_name(void *h, int e) { return ((omech_t *)h)->elem[e]; }

void oracle_species_data(void *h, double *W, int *comp) {
    omech_t *m = (omech_t *)h;
    memcpy(W, m->W, sizeof(double) * m->ns);
    memcpy(comp, m->comp, sizeof(int) * m->ns * m->ne);
}

void oracle_thermo(void *h, int k, double T, double *out4) {
    o_nasa((omech_t *)h, k, T, &out4[0], &out4[1], &out4[2], &out4[3]);
}

double oracle_e_mass(void *h, double T, const double *Y) { return o_e_mass((omech_t *)h, T, Y); }
double oracle_cv_mass(void *h, double T, const double *Y) { return o_cv_mass((omech_t *)h, T, Y); }

int oracle_T_from_e(void *h, double e, const double *Y, double Tguess, double *T) {
    return o_T_from_e((omech_t *)h, e, Y, Tguess, T);
}

/* (T, p, Y) -> (rho, e) for n cells; Y column-major [ns][n]. */
void oracle_state_from_TPY(void *h, long n, const double *T, const double *p, const double *Y,
                           double *rho, double *e) {
    omech_t *m = (omech_t *)h;
    double *y = malloc(sizeof(double) * m->ns);
    for (long i = 0; i < n; i++) {
        double sw = 0.0;
        for (int k = 0; k < m->ns; k++) {
            y[k] = Y[(size_t)k * n + i];
            sw += y[k] / m->W[k];
        }
        rho[i] = p[i] / (OR_RGAS * T[i] * sw);
        e[i] = o_e_mass(m, T[i], y);
    }
    free(y);
}

void oracle_rates(void *h, double T, const double *C, double *kf, double *kr, double *qf,
                  double *qr) {
    o_rates((omech_t *)h, T, C, kf, kr, qf, qr);
}

void oracle_rhs(void *h, double rho, const double *y, double *f) { o_rhs((omech_t *)h, rho, y, f); }
void oracle_jac(void *h, double rho, const double *y, double *J) { o_jac((omech_t *)h, rho, y, J); }

/* Integrate ncell cells over [0, dt].  Y is column-major, Y[k*ldY + i], in/out.
 * T: in = guess (non-finite or NULL -> 1500 K), out = final temperature.
 * status (may be NULL): per-cell status.  cstats (may be NULL): per-cell
 * [steps, attempts, rhs, jac, lu] as 5 longs.  Returns the number of cells
 * that did not reach dt. */
long oracle_integrate(void *h, long ncell, const double *rho, const double *e, double *Y, long ldY,
                      double *T, double dt, double rtol, double atol, long max_steps, int nthreads,
                      unsigned char *status, long *cstats) {
    omech_t *m = (omech_t *)h;
    const int ns = m->ns, n = ns + 1;
    long bad = 0;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads) reduction(+ : bad)
#endif
    for (long i = 0; i < ncell; i++) {
        double y[256];
        double *yy = n <= 256 ? y : malloc(sizeof(double) * n);
        for (int k = 0; k < ns; k++) yy[k] = Y[(size_t)k * ldY + i];
        double Tg = T ? T[i] : NAN, T0;
        int st;
        o_bdf_stats bs;
        memset(&bs, 0, sizeof bs);
        if (o_T_from_e(m, e[i], yy, Tg, &T0) != 0) {
            st = OR_ST_TINV;
        } else {
            yy[ns] = T0;
            cell_ctx_t cc = {m, rho[i]};
            st = o_bdf(n, 0.0, dt, yy, rtol, atol, max_steps, cell_rhs, cell_jac, &cc, NULL, 0, NULL,
                       &bs);
            for (int k = 0; k < ns; k++) Y[(size_t)k * ldY + i] = yy[k];
            if (T) T[i] = yy[ns];
        }
        if (status) status[i] = (unsigned char)st;
        if (cstats) {
            cstats[5 * i + 0] = bs.steps;
            cstats[5 * i + 1] = bs.attempts;
            cstats[5 * i + 2] = bs.rhs;
            cstats[5 * i + 3] = bs.jac;
            cstats[5 * i + 4] = bs.lu;
        }
        if (st != OR_ST_DONE) bad++;
        if (yy != y) free(yy);
    }
    return bad;
}

/* One cell with dense output at nout times (sorted); yout is [nout][ns+1]
 * holding (Y, T).  Returns the status. */
int oracle_trajectory(void *h, double rho, double e, const double *Y0, double Tguess, double t1,
                      const double *tout, int nout, double *yout, double rtol, double atol,
                      long max_steps) {
    omech_t *m = (omech_t *)h;
    const int ns = m->ns, n = ns + 1;
    double *y = malloc(sizeof(double) * n);
    memcpy(y, Y0, sizeof(double) * ns);
    double T0;
    if (o_T_from_e(m, e, y, Tguess, &T0) != 0) {
        free(y);
        return OR_ST_TINV;
    }
    y[ns] = T0;
    cell_ctx_t cc = {m, rho};
    int st = o_bdf(n, 0.0, t1, y, rtol, atol, max_steps, cell_rhs, cell_jac, &cc, tout, nout, yout,
                   NULL);
    free(y);
    return st;
}

/* Linear constant-coefficient test system y' = A y (A row-major n x n). */
typedef struct {
    int n;
    const double *A;
} lin_ctx_t;

static void lin_rhs(void *c, double t, const double *y, double *f) {
    (void)t;
    lin_ctx_t *l = (lin_ctx_t *)c;
    for (int i = 0; i < l->n; i++) {
        double s = 0.0;
        for (int j = 0; j < l->n; j++) s += l->A[i * l->n + j] * y[j];
        f[i] = s;
    }
}
static void lin_jac(void *c, double t, const double *y, double *J) {
    (void)t;
    (void)y;
    lin_ctx_t *l = (lin_ctx_t *)c;
    memcpy(J, l->A, sizeof(double) * l->n * l->n);
}

int oracle_bdf_linear(int n, const double *A, double *y, double t1, double rtol, double atol,
                      long max_steps, const double *tout, int nout, double *yout, long *stats7) {
    lin_ctx_t l = {n, A};
    o_bdf_stats st;
    int s = o_bdf(n, 0.0, t1, y, rtol, atol, max_steps, lin_rhs, lin_jac, &l, tout, nout, yout, &st);
    if (stats7) {
        stats7[0] = st.steps; stats7[1] = st.attempts; stats7[2] = st.rhs; stats7[3] = st.jac;
        stats7[4] = st.lu; stats7[5] = st.rej; stats7[6] = st.nfail;
    }
    return s;
}
