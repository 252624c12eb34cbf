/*
 * Oracle thermo, kinetics, right-hand side and analytic Jacobian
 * (test infrastructure; see oracle.h).
 *
 * Problem statement: each cell is a constant-volume ideal-gas reactor with
 * rho and e fixed over the flow step (Sec. 2.1, Eq. 5-6).  State
 * y = (Y_1..Y_ns, T).  Everything is written out from the textbook
 * definitions; no step uses logarithms of concentrations.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* NASA-7 polynomials: cp/R, h/RT, s/R and d(cp/R)/dT; the low set is used
 * iff T < Tmid, and the polynomials are evaluated as they are outside
 * [Tlow, Thigh] (no clamping). */
void o_nasa(const omech_t *m, int k, double T, double *cp_R, double *h_RT, double *s_R,
            double *dcp_R_dT) {
    const double *a = (T < m->Tmid[k]) ? &m->alo[k * 7] : &m->ahi[k * 7];
    double T2 = T * T, T3 = T2 * T, T4 = T3 * T;
    if (cp_R) *cp_R = a[0] + a[1] * T + a[2] * T2 + a[3] * T3 + a[4] * T4;
    if (h_RT)
        *h_RT = a[0] + a[1] * T / 2.0 + a[2] * T2 / 3.0 + a[3] * T3 / 4.0 + a[4] * T4 / 5.0 + a[5] / T;
    if (s_R)
        *s_R = a[0] * log(T) + a[1] * T + a[2] * T2 / 2.0 + a[3] * T3 / 3.0 + a[4] * T4 / 4.0 + a[6];
    if (dcp_R_dT) *dcp_R_dT = a[1] + 2.0 * a[2] * T + 3.0 * a[3] * T2 + 4.0 * a[4] * T3;
}

/* mass-specific internal energy e = sum_k Y_k u_k / W_k, u_k = h_k - R T */
double o_e_mass(const omech_t *m, double T, const double *Y) {
    double e = 0.0;
    for (int k = 0; k < m->ns; k++) {
        double h_RT;
        o_nasa(m, k, T, NULL, &h_RT, NULL, NULL);
        e += Y[k] * (h_RT - 1.0) * OR_RGAS * T / m->W[k];
    }
    return e;
}

/* mass-specific constant-volume heat capacity c_v = sum_k Y_k (cp_k - R) / W_k */
double o_cv_mass(const omech_t *m, double T, const double *Y) {
    double cv = 0.0;
    for (int k = 0; k < m->ns; k++) {
        double cp_R;
        o_nasa(m, k, T, &cp_R, NULL, NULL, NULL);
        cv += Y[k] * (cp_R - 1.0) * OR_RGAS / m->W[k];
    }
    return cv;
}

/* Temperature from (e, Y) at constant rho: Newton on e(T) - e = 0, guarded by
 * bisection inside [100, 6000] K.  Returns 0 on success. */
int o_T_from_e(const omech_t *m, double e, const double *Y, double Tguess, double *Tout) {
    double lo = 100.0, hi = 6000.0;
    double flo = o_e_mass(m, lo, Y) - e, fhi = o_e_mass(m, hi, Y) - e;
    if (!(flo <= 0.0 && fhi >= 0.0)) return -1;
    double T = (isfinite(Tguess) && Tguess > lo && Tguess < hi) ? Tguess : 1500.0;
    for (int it = 0; it < 100; it++) {
        double f = o_e_mass(m, T, Y) - e;
        if (f == 0.0) break;
        if (f < 0.0) lo = T;
        else hi = T;
        double cv = o_cv_mass(m, T, Y);
        double Tn = T - f / cv;
        if (!(Tn > lo && Tn < hi)) Tn = 0.5 * (lo + hi);
        double dT = fabs(Tn - T);
        T = Tn;
        if (dT <= 1e-12 * T || hi - lo <= 1e-12 * T) break;
    }
    *Tout = T;
    return 0;
}

static double ipow(double x, int n) {
    double r = 1.0;
    for (int i = 0; i < n; i++) r *= x;
    return r;
}

/* Per-reaction quantities shared by the rates, the RHS and the Jacobian. */
typedef struct {
    double kf, kr, Kc;
    double Pf, Pr_;        /* prod C^nu' and prod C^nu'' */
    double M;              /* third-body concentration (THREEBODY, FALLOFF) */
    double dlnkf_dT;       /* total d ln kf / dT at fixed concentrations */
    double dlnKc_dT;
    double dkf_dM;         /* falloff: d kf / d[M] */
} rxn_eval_t;

static void eval_reaction(const omech_t *m, int j, double T, const double *C,
                          const double *g_RT, const double *h_RT, rxn_eval_t *r) {
    const int ns = m->ns;
    const int *rsp = &m->rsp[j * OR_MAXPART], *rnu = &m->rnu[j * OR_MAXPART];
    const int *psp = &m->psp[j * OR_MAXPART], *pnu = &m->pnu[j * OR_MAXPART];
    double RT = OR_RGAS * T;
    /* Arrhenius */
    double kinf = m->A[j] * pow(T, m->b[j]) * exp(-m->Ea[j] / RT);
    double dlnkinf = m->b[j] / T + m->Ea[j] / (RT * T);
    r->M = 0.0;
    if (m->type[j] != OR_ELEM) {
        for (int k = 0; k < ns; k++) r->M += m->eff[(size_t)j * ns + k] * C[k];
    }
    r->dkf_dM = 0.0;
    if (m->type[j] == OR_FALLOFF) {
        double k0 = m->A0[j] * pow(T, m->b0[j]) * exp(-m->Ea0[j] / RT);
        double dlnk0 = m->b0[j] / T + m->Ea0[j] / (RT * T);
        double Pr = k0 * r->M / kinf;
        double F = 1.0, dlog10F_dx = 0.0, dlnF_dT = 0.0;
        if (m->troe_n[j] > 0) {
            const double *tp = &m->troe[j * 4];
            double a = tp[0], T3 = tp[1], T1 = tp[2];
            double Fc = (1.0 - a) * exp(-T / T3) + a * exp(-T / T1);
            double dFc = -(1.0 - a) / T3 * exp(-T / T3) - a / T1 * exp(-T / T1);
            if (m->troe_n[j] == 4) {
                double T2 = tp[3];
                Fc += exp(-T2 / T);
                dFc += T2 / (T * T) * exp(-T2 / T);
            }
            double phi = log10(Fc);
            double c = -0.4 - 0.67 * phi, nn = 0.75 - 1.27 * phi;
            double x = log10(Pr > 1e-300 ? Pr : 1e-300);
            double u = x + c, den = nn - 0.14 * u;
            double f1 = u / den;
            double q = 1.0 + f1 * f1;
            double log10F = phi / q;
            F = pow(10.0, log10F);
            double df1_dx = nn / (den * den);
            double df1_dphi = (-0.67 * den - u * (-1.27 + 0.14 * 0.67)) / (den * den);
            dlog10F_dx = -phi * 2.0 * f1 * df1_dx / (q * q);
            double dlog10F_dphi = 1.0 / q - phi * 2.0 * f1 * df1_dphi / (q * q);
            dlnF_dT = dlog10F_dphi * dFc / Fc; /* ln10 factors cancel */
        }
        double dlnPr_dT = dlnk0 - dlnkinf;
        r->kf = kinf * (Pr / (1.0 + Pr)) * F;
        r->dlnkf_dT = dlnkinf + dlnPr_dT / (1.0 + Pr) + dlnF_dT + dlog10F_dx * dlnPr_dT;
        /* d kf/d[M] = k0 F (1/(1+Pr)^2 + (dlnF/dlnPr)/(1+Pr)) */
        r->dkf_dM = k0 * F * (1.0 / ((1.0 + Pr) * (1.0 + Pr)) + dlog10F_dx / (1.0 + Pr));
    } else {
        r->kf = kinf;
        r->dlnkf_dT = dlnkinf;
    }
    /* equilibrium constant Kc = exp(-sum nu g/RT) (Pref/RT)^dnu */
    double sg = 0.0, sh = 0.0;
    int dnu = 0;
    for (int i = 0; i < m->nre[j]; i++) {
        sg -= rnu[i] * g_RT[rsp[i]];
        sh -= rnu[i] * h_RT[rsp[i]];
        dnu -= rnu[i];
    }
    for (int i = 0; i < m->npr[j]; i++) {
        sg += pnu[i] * g_RT[psp[i]];
        sh += pnu[i] * h_RT[psp[i]];
        dnu += pnu[i];
    }
    r->Kc = exp(-sg) * pow(OR_PREF / RT, (double)dnu);
    r->dlnKc_dT = sh / T - (double)dnu / T; /* d(g/RT)/dT = -h/(R T^2) */
    r->kr = m->rev[j] ? r->kf / r->Kc : 0.0;
    r->Pf = 1.0;
    for (int i = 0; i < m->nre[j]; i++) r->Pf *= ipow(C[rsp[i]], rnu[i]);
    r->Pr_ = 1.0;
    for (int i = 0; i < m->npr[j]; i++) r->Pr_ *= ipow(C[psp[i]], pnu[i]);
}

static void species_thermo(const omech_t *m, double T, double *g_RT, double *h_RT) {
    for (int k = 0; k < m->ns; k++) {
        double h, s;
        o_nasa(m, k, T, NULL, &h, &s, NULL);
        h_RT[k] = h;
        g_RT[k] = h - s;
    }
}

/* Rate constants and rates of progress.  qf and qr include the third-body
 * concentration of THREEBODY reactions, so the net rate is qf - qr. */
void o_rates(const omech_t *m, double T, const double *C, double *kf, double *kr,
             double *qf, double *qr) {
    double *g = malloc(2 * m->ns * sizeof(double)), *h = g + m->ns;
    species_thermo(m, T, g, h);
    for (int j = 0; j < m->nr; j++) {
        rxn_eval_t r;
        eval_reaction(m, j, T, C, g, h, &r);
        double mul = (m->type[j] == OR_THREEBODY) ? r.M : 1.0;
        if (kf) kf[j] = r.kf;
        if (kr) kr[j] = r.kr;
        if (qf) qf[j] = mul * r.kf * r.Pf;
        if (qr) qr[j] = mul * r.kr * r.Pr_;
    }
    free(g);
}

/* Right-hand side: f_k = W_k omega_k / rho, f_T = -sum u_k omega_k/(rho c_v). */
void o_rhs(const omech_t *m, double rho, const double *y, double *f) {
    const int ns = m->ns;
    const double T = y[ns];
    double *C = malloc(4 * ns * sizeof(double)), *g = C + ns, *h = g + ns, *om = h + ns;
    for (int k = 0; k < ns; k++) {
        C[k] = rho * y[k] / m->W[k];
        om[k] = 0.0;
    }
    species_thermo(m, T, g, h);
    for (int j = 0; j < m->nr; j++) {
        rxn_eval_t r;
        eval_reaction(m, j, T, C, g, h, &r);
        double mul = (m->type[j] == OR_THREEBODY) ? r.M : 1.0;
        double q = mul * (r.kf * r.Pf - r.kr * r.Pr_);
        for (int i = 0; i < m->nre[j]; i++) om[m->rsp[j * OR_MAXPART + i]] -= m->rnu[j * OR_MAXPART + i] * q;
        for (int i = 0; i < m->npr[j]; i++) om[m->psp[j * OR_MAXPART + i]] += m->pnu[j * OR_MAXPART + i] * q;
    }
    double cv = o_cv_mass(m, T, y), S = 0.0;
    for (int k = 0; k < ns; k++) {
        f[k] = m->W[k] * om[k] / rho;
        S += (h[k] - 1.0) * OR_RGAS * T * om[k];
    }
    f[ns] = -S / (rho * cv);
    free(C);
}

/* d(prod_l C_l^nu_l)/dC_m without dividing by C_m */
static double dprod(const double *C, const int *sp, const int *nu, int cnt, int m) {
    double p = 1.0;
    int found = 0;
    for (int i = 0; i < cnt; i++) {
        if (sp[i] == m) {
            p *= nu[i] * ipow(C[sp[i]], nu[i] - 1);
            found = 1;
        } else {
            p *= ipow(C[sp[i]], nu[i]);
        }
    }
    return found ? p : 0.0;
}

/* Analytic Jacobian J[i*n + j] = d f_i / d y_j, n = ns + 1. */
void o_jac(const omech_t *m, double rho, const double *y, double *J) {
    const int ns = m->ns, n = ns + 1;
    const double T = y[ns];
    double *C = malloc((5 * ns + 2 * ns * ns + ns) * sizeof(double));
    double *g = C + ns, *h = g + ns, *om = h + ns, *dwdT = om + ns;
    double *dwdC = dwdT + ns; /* [ns][ns]: d omega_k / d C_m */
    double *dqdC = dwdC + ns * ns;
    for (int k = 0; k < ns; k++) {
        C[k] = rho * y[k] / m->W[k];
        om[k] = dwdT[k] = 0.0;
    }
    memset(dwdC, 0, sizeof(double) * ns * ns);
    species_thermo(m, T, g, h);
    for (int j = 0; j < m->nr; j++) {
        const int *rsp = &m->rsp[j * OR_MAXPART], *rnu = &m->rnu[j * OR_MAXPART];
        const int *psp = &m->psp[j * OR_MAXPART], *pnu = &m->pnu[j * OR_MAXPART];
        rxn_eval_t r;
        eval_reaction(m, j, T, C, g, h, &r);
        double mul = (m->type[j] == OR_THREEBODY) ? r.M : 1.0;
        double net = r.kf * r.Pf - r.kr * r.Pr_;
        double q = mul * net;
        /* d q / d C_m */
        for (int mm = 0; mm < ns; mm++) {
            double d = mul * (r.kf * dprod(C, rsp, rnu, m->nre[j], mm) -
                              r.kr * dprod(C, psp, pnu, m->npr[j], mm));
            if (m->type[j] == OR_THREEBODY) d += m->eff[(size_t)j * ns + mm] * net;
            if (m->type[j] == OR_FALLOFF) {
                /* kf and kr = kf/Kc both depend on [M] */
                double dkf = r.dkf_dM * m->eff[(size_t)j * ns + mm];
                double dkr = m->rev[j] ? dkf / r.Kc : 0.0;
                d += dkf * r.Pf - dkr * r.Pr_;
            }
            dqdC[mm] = d;
        }
        /* d q / d T: kf' = kf dlnkf, kr' = kr (dlnkf - dlnKc) */
        double dqdT = mul * (r.kf * r.dlnkf_dT * r.Pf -
                             r.kr * (r.dlnkf_dT - r.dlnKc_dT) * r.Pr_);
        for (int i = 0; i < m->nre[j]; i++) {
            int k = rsp[i];
            om[k] -= rnu[i] * q;
            dwdT[k] -= rnu[i] * dqdT;
            for (int mm = 0; mm < ns; mm++) dwdC[k * ns + mm] -= rnu[i] * dqdC[mm];
        }
        for (int i = 0; i < m->npr[j]; i++) {
            int k = psp[i];
            om[k] += pnu[i] * q;
            dwdT[k] += pnu[i] * dqdT;
            for (int mm = 0; mm < ns; mm++) dwdC[k * ns + mm] += pnu[i] * dqdC[mm];
        }
    }
    double cv = 0.0, dcv = 0.0, S = 0.0;
    double *u = malloc(2 * ns * sizeof(double)), *cvk = u + ns;
    for (int k = 0; k < ns; k++) {
        double cp_R, dcp;
        o_nasa(m, k, T, &cp_R, NULL, NULL, &dcp);
        cvk[k] = (cp_R - 1.0) * OR_RGAS;
        u[k] = (h[k] - 1.0) * OR_RGAS * T;
        cv += y[k] * cvk[k] / m->W[k];
        dcv += y[k] * dcp * OR_RGAS / m->W[k];
        S += u[k] * om[k];
    }
    double fT = -S / (rho * cv);
    for (int k = 0; k < ns; k++) {
        for (int mm = 0; mm < ns; mm++) J[k * n + mm] = m->W[k] / m->W[mm] * dwdC[k * ns + mm];
        J[k * n + ns] = m->W[k] / rho * dwdT[k];
    }
    for (int mm = 0; mm < ns; mm++) {
        double dS = 0.0; /* d S / d Y_m */
        for (int k = 0; k < ns; k++) dS += u[k] * dwdC[k * ns + mm] * rho / m->W[mm];
        J[ns * n + mm] = -dS / (rho * cv) - fT * (cvk[mm] / m->W[mm]) / cv;
    }
    {
        double dS = 0.0;
        for (int k = 0; k < ns; k++) dS += cvk[k] * om[k] + u[k] * dwdT[k];
        J[ns * n + ns] = -dS / (rho * cv) - fT * dcv / cv;
    }
    free(u);
    free(C);
}
