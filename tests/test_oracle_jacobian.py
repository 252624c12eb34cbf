"""Oracle analytic Jacobian pinned by finite differences (M9) and by sympy's
symbolic differentiation of the right-hand side of a 4-species mechanism with
an elementary, a third-body and a 4-parameter Troe falloff reaction."""
import numpy as np
import pytest
import sympy as sp

from tests import toymech

R = 8.314462618


def _fd_jac(o, rho, y):
    n = y.size
    J = np.zeros((n, n))
    for j in range(n):
        h = 1e-6 * max(abs(y[j]), 1e-8 if j < n - 1 else 1.0)
        yp, ym = y.copy(), y.copy()
        yp[j] += h
        ym[j] -= h
        J[:, j] = (o.rhs(rho, yp) - o.rhs(rho, ym)) / (2 * h)
    return J


def test_jacobian_vs_central_differences_m9(m9):
    rng = np.random.default_rng(2)
    for _ in range(40):
        T = rng.uniform(800, 3000)
        p = rng.uniform(1, 30) * 101325.0
        Y = rng.dirichlet(np.ones(m9.ns) * 0.8) + 1e-3
        Y /= Y.sum()
        rho = p / (R * T * np.sum(Y / m9.W))
        y = np.concatenate([Y, [T]])
        Ja = m9.jac(rho, y)
        Jf = _fd_jac(m9, rho, y)
        for i in range(m9.n):
            scale = np.max(np.abs(Ja[i] * np.maximum(np.abs(y), 1e-3)))
            err = np.abs(Ja[i] - Jf[i]) * np.maximum(np.abs(y), 1e-3)
            assert np.all(err <= 1e-6 * scale + 1e-300), (i, err.max(), scale)


def _symbolic_rhs(mech, rho):
    """Right-hand side of the constant-volume reactor from the textbook
    definitions, in sympy (for differentiation only)."""
    ns = len(mech.species)
    Ys = sp.symbols(f"Y0:{ns}")
    T = sp.Symbol("T")
    W = [toymech_mw(s) * sp.Rational(1, 1000) for s in mech.species]
    Rg = sp.Float(R, 30)
    names = [s.name for s in mech.species]
    C = [rho * Ys[k] / W[k] for k in range(ns)]

    def nasa(s):
        a = [sp.Float(v, 30) for v in s.nasa_low]
        cp = a[0] + a[1] * T + a[2] * T**2 + a[3] * T**3 + a[4] * T**4
        h = a[0] + a[1] * T / 2 + a[2] * T**2 / 3 + a[3] * T**3 / 4 + a[4] * T**4 / 5 + a[5] / T
        s_ = a[0] * sp.log(T) + a[1] * T + a[2] * T**2 / 2 + a[3] * T**3 / 3 + a[4] * T**4 / 4 + a[6]
        return cp, h, s_

    th = [nasa(s) for s in mech.species]
    omega = [0] * ns
    for r in mech.reactions:
        order = sum(r.reactants.values())
        oinf = order + (1 if r.kind == "THREEBODY" else 0)
        k = sp.Float(r.A, 30) * sp.Float(1e-6, 30) ** (oinf - 1) * T ** sp.Float(r.b, 30) * \
            sp.exp(-sp.Float(r.Ea * 4.184, 30) / (Rg * T))
        eff = [r.efficiencies.get(n, 1.0) for n in names]
        M = sum(sp.Float(eff[i], 30) * C[i] for i in range(ns))
        if r.kind == "FALLOFF":
            A0, b0, E0 = r.low
            k0 = sp.Float(A0, 30) * sp.Float(1e-6, 30) ** order * T ** sp.Float(b0, 30) * \
                sp.exp(-sp.Float(E0 * 4.184, 30) / (Rg * T))
            Pr = k0 * M / k
            a, T3, T1, T2 = [sp.Float(v, 30) for v in r.troe]
            Fc = (1 - a) * sp.exp(-T / T3) + a * sp.exp(-T / T1) + sp.exp(-T2 / T)
            lf = sp.log(Fc, 10)
            c = -sp.Float(0.4, 30) - sp.Float(0.67, 30) * lf
            nn = sp.Float(0.75, 30) - sp.Float(1.27, 30) * lf
            u = sp.log(Pr, 10) + c
            f1 = u / (nn - sp.Float(0.14, 30) * u)
            F = 10 ** (lf / (1 + f1**2))
            k = k * Pr / (1 + Pr) * F
        dnu = sum(r.products.values()) - order
        sg = sum(v * (th[names.index(s)][1] - th[names.index(s)][2]) for s, v in r.products.items()) - \
            sum(v * (th[names.index(s)][1] - th[names.index(s)][2]) for s, v in r.reactants.items())
        Kc = sp.exp(-sg) * (sp.Float(101325.0, 30) / (Rg * T)) ** dnu
        qf = k
        for s, v in r.reactants.items():
            qf = qf * C[names.index(s)] ** v
        qr = k / Kc
        for s, v in r.products.items():
            qr = qr * C[names.index(s)] ** v
        q = (qf - qr) * (M if r.kind == "THREEBODY" else 1)
        for s, v in r.reactants.items():
            omega[names.index(s)] -= v * q
        for s, v in r.products.items():
            omega[names.index(s)] += v * q
    cv = sum(Ys[k] * (th[k][0] - 1) * Rg / W[k] for k in range(ns))
    f = [W[k] * omega[k] / rho for k in range(ns)]
    f.append(-sum((th[k][1] - 1) * Rg * T * omega[k] for k in range(ns)) / (rho * cv))
    return sp.Matrix(f), list(Ys) + [T]


def toymech_mw(s):
    from synth.mechfile import molecular_weight
    return sp.Float(molecular_weight(s), 30)


def test_jacobian_vs_sympy_toy4(oracle_lib):
    mech = toymech.toy4()
    o = oracle_lib.Oracle(toymech.write(mech, "toy4"))
    rho = 0.35
    f, v = _symbolic_rhs(mech, sp.Float(rho, 30))
    Jsym = f.jacobian(v)
    import mpmath
    mpmath.mp.dps = 30
    Jfun = sp.lambdify(v, Jsym, modules="mpmath")
    ffun = sp.lambdify(v, f, modules="mpmath")
    rng = np.random.default_rng(4)
    for _ in range(3):
        Y = rng.dirichlet(np.ones(4))
        T = rng.uniform(900, 2500)
        y = np.concatenate([Y, [T]])
        args = [mpmath.mpf(float(x)) for x in y]
        Js = np.array(Jfun(*args).tolist(), dtype=float)
        fs = np.array(ffun(*args).tolist(), dtype=float).ravel()
        Jo = o.jac(rho, y)
        fo = o.rhs(rho, y)
        assert np.allclose(fo, fs, rtol=1e-11, atol=1e-11 * np.abs(fs).max())
        for i in range(5):
            sc = np.abs(Js[i]).max()
            assert np.allclose(Jo[i], Js[i], rtol=1e-10, atol=1e-11 * sc), (i, Jo[i], Js[i])
