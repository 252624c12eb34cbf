/*
 * CPU FP64 oracle for constant-volume (constant rho, constant e) ideal-gas
 * reactor chemistry.  TEST INFRASTRUCTURE ONLY: it is used by tests/, by the
 * smoke check and by the benchmark's CPU-baseline leg; the product library
 * never links, loads or calls it, and it shares no code with the product.
 *
 * What it computes (per cell, independently): the solution at t = dt of
 *   dY_k/dt = W_k omega_k / rho                                  (Eq. 5)
 *   dT/dt   = -sum_k u_k omega_k / (rho c_v)                     (Eq. 6, read
 *             with the mass-based mixture c_v and molar u_k, which is the
 *             form that keeps e constant; the printed Eq. 6 is garbled)
 * starting from T0 = T(e, Y0) (the Newton temperature inversion at constant
 * e and rho described with Eq. 5-6), with plain mass-action kinetics:
 * Arrhenius, third-body, Lindemann/Troe falloff, reverse rates from the
 * equilibrium constant, NASA-7 thermo.  Rates use integer powers of the
 * concentrations (no logarithms, no floors).  The integrator is a
 * variable-order (1-5) variable-step BDF in backward-difference form
 * (Shampine & Reichelt 1997, quasi-constant step size, kappa = 0) with a
 * modified Newton iteration on the analytic Jacobian and a WRMS error test
 * with weights 1/(rtol |y| + atol).
 *
 * Units: SI (kg, m, s, mol, J, K).  e is the mass-specific internal energy
 * including formation energy (absolute NASA-7 basis).  Reference pressure
 * for the equilibrium constant: 101325 Pa.
 */
#ifndef ORACLE_H
#define ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define OR_RGAS 8.314462618
#define OR_PREF 101325.0
#define OR_CAL 4.184
#define OR_MAXPART 6

enum { OR_ELEM = 0, OR_THREEBODY = 1, OR_FALLOFF = 2 };

typedef struct {
    char name[128];
    int ns, nr, ne;
    char (*elem)[8];
    char (*sp)[32];
    double *W;      /* kg/mol, [ns] */
    int *comp;      /* [ns*ne] atoms of element e in species k */
    double *Tlo, *Tmid, *Thi; /* [ns] */
    double *alo, *ahi;        /* [ns*7] NASA-7 for T < Tmid and T >= Tmid */
    int *type, *rev;          /* [nr] */
    int *nre, *npr;           /* [nr] */
    int *rsp, *rnu, *psp, *pnu; /* [nr*OR_MAXPART] */
    double *A, *b, *Ea;       /* SI; Ea in J/mol */
    double *eff;              /* [nr*ns], default 1 */
    double *A0, *b0, *Ea0;    /* falloff low-pressure limit, SI */
    int *troe_n;              /* 0 (Lindemann), 3 or 4 */
    double *troe;             /* [nr*4]: a, T***, T*, T** */
} omech_t;

/* statuses, same meaning as the product's */
enum { OR_ST_DONE = 0, OR_ST_SKIPPED = 1, OR_ST_KMAX = 2, OR_ST_FAIL = 3, OR_ST_TINV = 4 };

typedef struct { long steps, attempts, rhs, jac, lu, rej, nfail; } o_bdf_stats;
typedef void (*o_rhs_fn)(void *ctx, double t, const double *y, double *f);
typedef void (*o_jac_fn)(void *ctx, double t, const double *y, double *J);

/* mechanism */
int omech_load(const char *path, omech_t **out, char *err, int errlen);
void omech_free(omech_t *m);

/* thermo (molar, dimensionless) */
void o_nasa(const omech_t *m, int k, double T, double *cp_R, double *h_RT, double *s_R,
            double *dcp_R_dT);
double o_e_mass(const omech_t *m, double T, const double *Y);
double o_cv_mass(const omech_t *m, double T, const double *Y);
int o_T_from_e(const omech_t *m, double e, const double *Y, double Tguess, double *T);

/* kinetics */
void o_rates(const omech_t *m, double T, const double *C, double *kf, double *kr,
             double *qf, double *qr);
void o_rhs(const omech_t *m, double rho, const double *y, double *f);
void o_jac(const omech_t *m, double rho, const double *y, double *J);

/* integrator */
int o_bdf(int n, double t0, double t1, double *y, double rtol, double atol, long max_steps,
          o_rhs_fn rhs, o_jac_fn jac, void *ctx, const double *tout, int nout, double *yout,
          o_bdf_stats *st);

#ifdef __cplusplus
}
#endif
#endif
