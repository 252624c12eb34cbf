"""Ideal-gas chemical equilibrium at fixed (T, p, element moles) by direct
Gibbs-energy minimisation (test infrastructure only).

Primary method: the element-potential Newton iteration for a TP problem of
Gordon & McBride, NASA RP-1311 (1994), Part I, restated here.  With
mu_j/RT = g_j/RT + ln(n_j/n) + ln(p/p_ref) and element multipliers pi_i,

    dln n_j = -mu_j/RT + sum_i a_ij pi_i + dln n                     (species)
    sum_j a_ij n_j dln n_j = b_i0 - b_i                               (elements)
    sum_j n_j dln n_j - n dln n = n - sum_j n_j                       (total moles)

Eliminating dln n_j leaves an (ne+1) linear system for (pi, dln n).  The
step is damped by the report's control factors: major species may change
ln n by at most 2 (and dln n by 0.4), and a trace species whose mole fraction
is rising may not overshoot 1e-4.  Species made of absent elements are
dropped.  The result is checked by ``equilibrium_residuals`` (optimality of
the chemical potentials and element balance).

Cross-check: SLSQP on ln n_j with the element constraints (scipy).
g_j/RT comes from the oracle's NASA-7 thermo.
"""
from __future__ import annotations

import numpy as np

P_REF = 101325.0


def g_RT_all(orc, T):
    g = np.zeros(orc.ns)
    for k in range(orc.ns):
        cp, h, s, _ = orc.thermo(k, T)
        g[k] = h - s
    return g


def equilibrate_TP(orc, T, p, b, tol=1e-14, maxit=400):
    """Equilibrium mole fractions X (length ns) at (T, p) for element moles
    b (length ne)."""
    A = orc.comp.astype(np.float64)              # [ns, ne]
    b = np.asarray(b, dtype=np.float64)
    present_el = b > 0
    ok = np.all((A[:, ~present_el] == 0), axis=1)
    idx = np.where(ok)[0]
    Aa = A[np.ix_(idx, np.where(present_el)[0])]
    bb = b[present_el] / b[present_el].sum()   # the problem is scale-free in b
    g0 = g_RT_all(orc, T)[idx] + np.log(p / P_REF)
    m = len(idx)
    ne = Aa.shape[1]
    lnn = np.full(m, np.log(0.1 / m))
    lnN = np.log(0.1)
    for it in range(maxit):
        n = np.exp(lnn)
        N = np.exp(lnN)
        mu = g0 + lnn - lnN
        M = np.zeros((ne + 1, ne + 1))
        r = np.zeros(ne + 1)
        M[:ne, :ne] = (Aa * n[:, None]).T @ Aa
        M[:ne, ne] = Aa.T @ n
        r[:ne] = bb - Aa.T @ n + Aa.T @ (n * mu)
        M[ne, :ne] = Aa.T @ n
        M[ne, ne] = n.sum() - N
        r[ne] = N - n.sum() + np.sum(n * mu)
        sol = np.linalg.lstsq(M, r, rcond=None)[0]
        pi, dlnN = sol[:ne], sol[ne]
        dlnn = -mu + Aa @ pi + dlnN
        x = lnn - lnN
        major = x > np.log(1e-8)
        big = max(5.0 * abs(dlnN), np.max(np.abs(dlnn[major])) if major.any() else 0.0)
        lam1 = 2.0 / big if big > 2.0 else 1.0
        lam2 = 1.0
        sel = (~major) & (dlnn >= 0)
        if sel.any():
            den = dlnn[sel] - dlnN
            with np.errstate(divide="ignore", invalid="ignore"):
                c = np.abs((-x[sel] - 9.2103404) / den)
            c = c[np.isfinite(c) & (den > 0)]
            if c.size:
                lam2 = c.min()
        lam = min(1.0, lam1, lam2)
        lnn = lnn + lam * dlnn
        lnN = lnN + lam * dlnN
        conv = np.max(np.abs(n * dlnn)) / n.sum()
        if lam == 1.0 and conv < tol and abs(dlnN) < tol:
            break
    X = np.zeros(orc.ns)
    n = np.exp(lnn)
    X[idx] = n / n.sum()
    return X


def equilibrium_residuals(orc, T, p, X, b):
    """Optimality check: for species with X > 0, mu_j/RT must be a linear
    combination of element counts; returns (max mu residual over species with
    X > 1e-30 after a least-squares fit of the multipliers, element error)."""
    A = orc.comp.astype(np.float64)
    g = g_RT_all(orc, T) + np.log(p / P_REF)
    pres = X > 1e-30
    mu = g[pres] + np.log(X[pres])
    pi, *_ = np.linalg.lstsq(A[pres], mu, rcond=None)
    res = np.max(np.abs(A[pres] @ pi - mu))
    nel = A.T @ X
    b = np.asarray(b, dtype=float)
    el = np.max(np.abs(nel / nel.sum() - b / b.sum()))
    return res, el


def equilibrate_slsqp(orc, T, p, b, X0=None):
    """Cross-check by SLSQP on z = ln n (scipy.optimize), with element
    moles normalised to unit total so that n stays O(1)."""
    from scipy.optimize import minimize
    A = orc.comp.astype(np.float64)
    b = np.asarray(b, dtype=float)
    present_el = b > 0
    ok = np.all((A[:, ~present_el] == 0), axis=1)
    idx = np.where(ok)[0]
    Aa = A[np.ix_(idx, np.where(present_el)[0])]
    bb = b[present_el] / b[present_el].sum()
    g0 = g_RT_all(orc, T)[idx] + np.log(p / P_REF)

    def G(z):
        n = np.exp(z)
        return float(np.sum(n * (g0 + z - np.log(n.sum()))))

    def dG(z):
        n = np.exp(z)
        return n * (g0 + z - np.log(n.sum()))

    cons = {"type": "eq", "fun": lambda z: Aa.T @ np.exp(z) - bb,
            "jac": lambda z: Aa.T * np.exp(z)[None, :]}
    if X0 is None:
        z0 = np.full(len(idx), np.log(1.0 / len(idx)))
    else:
        x0 = np.maximum(np.asarray(X0, dtype=float)[idx], 1e-30)
        z0 = np.log(x0 / x0.sum() * 0.5)
    res = minimize(G, z0, jac=dG, constraints=[cons], method="SLSQP",
                   bounds=[(-200.0, 2.0)] * len(idx),
                   options={"ftol": 1e-16, "maxiter": 5000})
    X = np.zeros(orc.ns)
    n = np.exp(res.x)
    X[idx] = n / n.sum()
    return X


def element_moles_from_Y(orc, Y):
    """Element moles per kg of mixture for mass fractions Y."""
    return orc.comp.T.astype(float) @ (np.asarray(Y) / orc.W)


def Y_from_X(orc, X):
    w = np.asarray(X) * orc.W
    return w / w.sum()
