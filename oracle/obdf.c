/*
 * Oracle integrator (test infrastructure; see oracle.h): dense LU with
 * partial pivoting and a variable-order, variable-step BDF.
 *
 * BDF formulation: backward differences D_j = nabla^j y_n of the solution on
 * a grid of constant spacing h (Shampine & Reichelt, "The MATLAB ODE Suite",
 * SIAM J. Sci. Comput. 18 (1997), the quasi-constant step size BDF with
 * kappa = 0).  With gamma_k = sum_{i<=k} 1/i, the order-k formula
 *     sum_{j=1..k} (1/j) nabla^j y_{n+1} = h f(y_{n+1})
 * written around the predictor y0 = sum_{j<=k} D_j becomes, for the
 * correction d = y_{n+1} - y0 = nabla^{k+1} y_{n+1},
 *     d = (h/gamma_k) f(y0 + d) - psi,   psi = (1/gamma_k) sum_{j=1..k} gamma_j D_j,
 * solved by modified Newton with M = I - (h/gamma_k) J.  The local error is
 * estimated as d/(k+1).  A change of step size h -> rho h re-expresses the
 * differences of the interpolating polynomial on the new grid.
 *
 * Implementation source followed: SciPy's BDF solver
 * (scipy/integrate/_ivp/bdf.py, BSD-3-Clause licence), with kappa = 0.  The
 * modified-Newton loop (at most 4 iterations, the convergence-rate test
 * rate^(4-it)/(1-rate) |dy| against newton_tol = max(10 eps/rtol,
 * min(0.03, sqrt(rtol)))), the update of the difference array on acceptance
 * and the order and step selection (safety 0.9, factors clamped to
 * [0.2, 10]) follow it.  Written here: the re-expression of the differences
 * on a new grid (rescale), the Jacobian reuse policy, the last-step clamp
 * onto t1 and the starting step of Hairer, Norsett & Wanner.
 */
#include "oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define MAXORD 5

/* LU with partial pivoting, in place, row-major; returns 0 or -1 if singular */
static int lu_factor(int n, double *a, int *piv) {
    for (int k = 0; k < n; k++) {
        int p = k;
        double best = fabs(a[k * n + k]);
        for (int i = k + 1; i < n; i++)
            if (fabs(a[i * n + k]) > best) {
                best = fabs(a[i * n + k]);
                p = i;
            }
        piv[k] = p;
        if (best == 0.0) return -1;
        if (p != k)
            for (int j = 0; j < n; j++) {
                double t = a[k * n + j];
                a[k * n + j] = a[p * n + j];
                a[p * n + j] = t;
            }
        for (int i = k + 1; i < n; i++) {
            double l = a[i * n + k] / a[k * n + k];
            a[i * n + k] = l;
            for (int j = k + 1; j < n; j++) a[i * n + j] -= l * a[k * n + j];
        }
    }
    return 0;
}

static void lu_solve(int n, const double *a, const int *piv, double *b) {
    for (int k = 0; k < n; k++) {
        if (piv[k] != k) {
            double t = b[k];
            b[k] = b[piv[k]];
            b[piv[k]] = t;
        }
    }
    for (int i = 1; i < n; i++)
        for (int j = 0; j < i; j++) b[i] -= a[i * n + j] * b[j];
    for (int i = n - 1; i >= 0; i--) {
        for (int j = i + 1; j < n; j++) b[i] -= a[i * n + j] * b[j];
        b[i] /= a[i * n + i];
    }
}

static double wrms(int n, const double *v, const double *scale) {
    double s = 0.0;
    for (int i = 0; i < n; i++) {
        double r = v[i] / scale[i];
        s += r * r;
    }
    return sqrt(s / n);
}

/* binomial-type basis: b_i(x) = prod_{l=1..i} (l - 1 - x)/l, so that the
 * interpolant is P(t_n + s h) = sum_i D_i b_i(-s). */
static double basis(int i, double x) {
    double r = 1.0;
    for (int l = 1; l <= i; l++) r *= (l - 1 - x) / l;
    return r;
}

/* D_j <- nabla'^j P(t_n) on the grid of spacing rho*h:
 * nabla'^j P(t_n) = sum_m (-1)^m C(j,m) P(t_n - m rho h)
 *                 = sum_i D_i sum_m (-1)^m C(j,m) b_i(m rho). */
static void rescale(int n, int k, double *D, double rho, double *tmp) {
    double Tm[MAXORD + 1][MAXORD + 1];
    for (int j = 0; j <= k; j++) {
        for (int i = 0; i <= k; i++) {
            double s = 0.0, binom = 1.0;
            for (int mm = 0; mm <= j; mm++) {
                s += ((mm & 1) ? -binom : binom) * basis(i, mm * rho);
                binom = binom * (j - mm) / (mm + 1);
            }
            Tm[j][i] = s;
        }
    }
    for (int c = 0; c < n; c++) {
        for (int j = 0; j <= k; j++) {
            double s = 0.0;
            for (int i = 0; i <= k; i++) s += Tm[j][i] * D[i * n + c];
            tmp[j] = s;
        }
        for (int j = 0; j <= k; j++) D[j * n + c] = tmp[j];
    }
}

static const double GAMMA[MAXORD + 2] = {0.0, 1.0, 1.5, 11.0 / 6.0, 25.0 / 12.0, 137.0 / 60.0,
                                         147.0 / 60.0};

/* Initial step (Hairer, Norsett & Wanner, Solving ODEs I, Sec. II.4). */
static double initial_step(int n, double t0, double t1, const double *y0, const double *f0,
                           double rtol, double atol, o_rhs_fn rhs, void *ctx, double *w1,
                           double *w2, double *sc, long *nrhs) {
    for (int i = 0; i < n; i++) sc[i] = atol + rtol * fabs(y0[i]);
    double d0 = wrms(n, y0, sc), d1 = wrms(n, f0, sc);
    double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
    if (h0 > t1 - t0) h0 = t1 - t0;
    for (int i = 0; i < n; i++) w1[i] = y0[i] + h0 * f0[i];
    rhs(ctx, t0 + h0, w1, w2);
    (*nrhs)++;
    for (int i = 0; i < n; i++) w2[i] -= f0[i];
    double d2 = wrms(n, w2, sc) / h0;
    double mx = d1 > d2 ? d1 : d2;
    double h1 = (mx <= 1e-15) ? fmax(1e-6, h0 * 1e-3) : pow(0.01 / mx, 0.5);
    double h = fmin(100.0 * h0, h1);
    return fmin(h, t1 - t0);
}

int o_bdf(int n, double t0, double t1, double *y, double rtol, double atol, long max_steps,
          o_rhs_fn rhs, o_jac_fn jac, void *ctx, const double *tout, int nout, double *yout,
          o_bdf_stats *st) {
    o_bdf_stats dummy;
    if (!st) st = &dummy;
    memset(st, 0, sizeof *st);
    const double eps = DBL_EPSILON;
    double *D = calloc((size_t)(MAXORD + 3) * n, sizeof(double));
    double *J = malloc(sizeof(double) * n * n), *LU = malloc(sizeof(double) * n * n);
    double *work = malloc(sizeof(double) * (n * 9 + MAXORD + 3));
    double *f = work, *ypred = f + n, *psi = ypred + n, *d = psi + n, *ynew = d + n;
    double *dy = ynew + n, *sc = dy + n, *e1 = sc + n, *e2 = e1 + n;
    double *tmp = e2 + n; /* MAXORD + 3 entries, used by rescale() */
    int *piv = malloc(sizeof(int) * n);
    int iout = 0;
    while (iout < nout && tout[iout] <= t0) {
        memcpy(&yout[(size_t)iout * n], y, sizeof(double) * n);
        iout++;
    }
    int status = OR_ST_DONE;
    double t = t0;
    if (t1 <= t0) goto done;
    rhs(ctx, t, y, f);
    st->rhs++;
    double h = initial_step(n, t0, t1, y, f, rtol, atol, rhs, ctx, e1, e2, sc, &st->rhs);
    for (int i = 0; i < n; i++) {
        D[i] = y[i];
        D[n + i] = h * f[i];
    }
    int k = 1, neq = 0;
    jac(ctx, t, y, J);
    st->jac++;
    int jac_current = 1;
    double c_lu = -1.0;
    const double newton_tol = fmax(10.0 * eps / rtol, fmin(0.03, sqrt(rtol)));

    while (t < t1) {
        if (st->attempts >= max_steps) {
            status = OR_ST_KMAX;
            break;
        }
        st->attempts++;
        double hmin = 10.0 * eps * fabs(t); /* t + h must differ from t */
        if (!(h >= hmin)) {
            status = OR_ST_FAIL;
            break;
        }
        int last = 0;
        /* the step reaches t1 when t + h rounds to t1 or beyond, or when h
         * covers t1 - t: after the clamp below h = t1 - t exactly, and a
         * retry at that size must land on t1 although t + h may round below */
        if (t + h >= t1 || h >= t1 - t) {
            double hn = t1 - t;
            rescale(n, k, D, hn / h, tmp);
            h = hn;
            neq = 0;
            last = 1;
        }
        double tn = last ? t1 : t + h;
        /* predictor and psi */
        for (int i = 0; i < n; i++) {
            double yp = 0.0, ps = 0.0;
            for (int j = 0; j <= k; j++) yp += D[j * n + i];
            for (int j = 1; j <= k; j++) ps += GAMMA[j] * D[j * n + i];
            ypred[i] = yp;
            psi[i] = ps / GAMMA[k];
            sc[i] = atol + rtol * fabs(yp);
        }
        double c = h / GAMMA[k];
        if (c != c_lu) {
            for (int i = 0; i < n * n; i++) LU[i] = -c * J[i];
            for (int i = 0; i < n; i++) LU[i * n + i] += 1.0;
            st->lu++;
            if (lu_factor(n, LU, piv) != 0) {
                c_lu = -1.0;
                goto newton_failed;
            }
            c_lu = c;
        }
        /* modified Newton */
        int conv = 0;
        {
            double dn_old = -1.0;
            for (int i = 0; i < n; i++) {
                d[i] = 0.0;
                ynew[i] = ypred[i];
            }
            for (int it = 0; it < 4; it++) {
                rhs(ctx, tn, ynew, f);
                st->rhs++;
                int finite = 1;
                for (int i = 0; i < n; i++) {
                    dy[i] = c * f[i] - psi[i] - d[i];
                    if (!isfinite(dy[i])) finite = 0;
                }
                if (!finite) break;
                lu_solve(n, LU, piv, dy);
                double dn = wrms(n, dy, sc);
                double rate = dn_old > 0.0 ? dn / dn_old : -1.0;
                if (rate >= 0.0 && (rate >= 1.0 || pow(rate, 4 - it) / (1.0 - rate) * dn > newton_tol))
                    break;
                for (int i = 0; i < n; i++) {
                    ynew[i] += dy[i];
                    d[i] += dy[i];
                }
                if (dn == 0.0 || (rate >= 0.0 && rate / (1.0 - rate) * dn < newton_tol)) {
                    conv = 1;
                    break;
                }
                dn_old = dn;
            }
        }
        if (!conv) {
        newton_failed:
            if (!jac_current) {
                jac(ctx, tn, ypred, J);
                st->jac++;
                jac_current = 1;
                c_lu = -1.0;
                continue;
            }
            st->nfail++;
            rescale(n, k, D, 0.5, tmp);
            h *= 0.5;
            neq = 0;
            continue;
        }
        /* error test */
        for (int i = 0; i < n; i++) {
            sc[i] = atol + rtol * fabs(ynew[i]);
            e1[i] = d[i] / (k + 1);
        }
        double en = wrms(n, e1, sc);
        if (en > 1.0) {
            double fac = fmax(0.2, 0.9 * pow(en, -1.0 / (k + 1)));
            st->rej++;
            rescale(n, k, D, fac, tmp);
            h *= fac;
            neq = 0;
            continue;
        }
        /* accept: update the difference array */
        st->steps++;
        t = tn;
        jac_current = 0;
        for (int i = 0; i < n; i++) {
            D[(k + 2) * n + i] = d[i] - D[(k + 1) * n + i];
            D[(k + 1) * n + i] = d[i];
        }
        for (int j = k; j >= 0; j--)
            for (int i = 0; i < n; i++) D[j * n + i] += D[(j + 1) * n + i];
        neq++;
        /* dense output inside the accepted step */
        while (iout < nout && tout[iout] <= t) {
            double s = (tout[iout] - t) / h;
            for (int i = 0; i < n; i++) {
                double v = 0.0;
                for (int j = 0; j <= k; j++) v += D[j * n + i] * basis(j, -s);
                yout[(size_t)iout * n + i] = v;
            }
            iout++;
        }
        if (last) break;
        if (neq < k + 1) continue;
        /* order and step-size selection */
        double fm = 0.0, fp = 0.0;
        if (k > 1) {
            for (int i = 0; i < n; i++) e2[i] = D[k * n + i] / k;
            fm = pow(wrms(n, e2, sc), -1.0 / k);
        }
        if (k < MAXORD) {
            for (int i = 0; i < n; i++) e2[i] = D[(k + 2) * n + i] / (k + 2);
            fp = pow(wrms(n, e2, sc), -1.0 / (k + 2));
        }
        double f0 = pow(en, -1.0 / (k + 1));
        int dk = 0;
        double best = f0;
        if (fm > best) {
            best = fm;
            dk = -1;
        }
        if (fp > best) {
            best = fp;
            dk = 1;
        }
        k += dk;
        double fac = fmin(10.0, 0.9 * best);
        rescale(n, k, D, fac, tmp);
        h *= fac;
        neq = 0;
    }
    for (int i = 0; i < n; i++) y[i] = D[i];
done:
    while (iout < nout) { /* outputs beyond the reached time keep the last state */
        memcpy(&yout[(size_t)iout * n], y, sizeof(double) * n);
        iout++;
    }
    free(D);
    free(J);
    free(LU);
    free(work);
    free(piv);
    return status;
}
