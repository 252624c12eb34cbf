"""Oracle BDF pinned by closed-form ODE solutions, the matrix exponential,
an independent integrator family (scipy Radau), conservation laws, the
Gibbs equilibrium at long times and ignition-delay convergence."""
import numpy as np
import pytest
import scipy.linalg
from scipy.integrate import solve_ivp

import oracle
from oracle import gibbs
from synth import fields
from tests import toymech

R = 8.314462618


@pytest.mark.parametrize("lam", [-1.0, -1e3, -1e6, -1e9])
def test_dahlquist(oracle_lib, lam):
    t1 = 5.0 / abs(lam)      # y(t1) = e^-5, well above atol
    tout = np.linspace(0.0, t1, 41)[1:]
    errs = []
    for rtol in (1e-5, 1e-7, 1e-9, 1e-11):
        atol = rtol * 1e-6
        y, st, stats, yout = oracle.bdf_linear(np.array([[lam]]), [1.0], t1, rtol, atol, tout)
        assert st == 0
        exact = np.exp(lam * tout)
        err = np.max(np.abs(yout[:, 0] - exact) / (rtol * np.abs(exact) + atol))
        # BDF global error: a modest multiple of the local tolerance that grows
        # with the number of steps (scipy's BDF of the same family gives ~90x at 1e-11)
        assert err < 300.0, (rtol, err)
        errs.append(np.max(np.abs(yout[:, 0] - exact)))
    # error shrinks as the tolerance tightens
    assert all(errs[i + 1] < errs[i] for i in range(len(errs) - 1)), errs


def test_stiff_linear_system_vs_expm(oracle_lib):
    rng = np.random.default_rng(0)
    Q, _ = np.linalg.qr(rng.normal(size=(6, 6)))
    lam = -np.logspace(0, 7, 6)
    A = Q @ np.diag(lam) @ Q.T
    y0 = rng.normal(size=6)
    tout = np.array([1e-6, 1e-4, 1e-2, 0.3, 1.0])
    y, st, stats, yout = oracle.bdf_linear(A, y0, 1.0, 1e-10, 1e-14, tout)
    assert st == 0
    for i, t in enumerate(tout):
        ex = scipy.linalg.expm(A * t) @ y0
        assert np.allclose(yout[i], ex, rtol=1e-7, atol=1e-9 * np.abs(y0).max())


def _one_cell(o, T, p, Y):
    rho, e = o.state_from_TPY(np.array([T]), p, np.asarray(Y, dtype=float).reshape(-1, 1))
    return rho[0], e[0]


def test_isomerisation_closed_form(oracle_lib):
    kf = 2.0e6          # 1/s (unimolecular: no unit conversion)
    o = oracle_lib.Oracle(toymech.write(toymech.isomer_AB(A=kf, da7=0.7), "iso"))
    Kc = np.exp(0.7)
    kr = kf / Kc
    Y = np.array([0.3, 0.05, 0.65])
    T0, p = 1200.0, 2e5
    rho, e = _one_cell(o, T0, p, Y)
    for dt in (1e-7, 5e-7, 3e-6):
        Yo, To, st = o.integrate([rho], [e], Y.reshape(3, 1), dt, 1e-11, 1e-16)
        assert st[0] == 0
        assert To[0] == pytest.approx(T0, rel=1e-12)          # no heat release
        tot = Y[0] + Y[1]
        Aeq = tot / (1 + Kc)
        A_t = Aeq + (Y[0] - Aeq) * np.exp(-(kf + kr) * dt)
        assert Yo[0, 0] == pytest.approx(A_t, rel=1e-8)
        assert Yo[1, 0] == pytest.approx(tot - A_t, rel=1e-8)


def test_dimerisation_closed_form(oracle_lib):
    A_cgs = 3e12        # cm^3/mol/s
    k = A_cgs * 1e-6    # m^3/mol/s
    o = oracle_lib.Oracle(toymech.write(toymech.dimer(A=A_cgs), "dimer"))
    Y = np.array([0.2, 0.0, 0.8])
    rho, e = _one_cell(o, 1500.0, 5e5, Y)
    C0 = rho * Y[0] / o.W[0]
    for dt in (1e-7, 1e-6, 1e-5):
        Yo, To, st = o.integrate([rho], [e], Y.reshape(3, 1), dt, 1e-11, 1e-16)
        assert st[0] == 0 and To[0] == pytest.approx(1500.0, rel=1e-12)
        CA = rho * Yo[0, 0] / o.W[0]
        assert 1.0 / CA == pytest.approx(1.0 / C0 + 2 * k * dt, rel=1e-8)


def test_third_body_closed_form(oracle_lib):
    # A + M => B + M is second order overall (order = reactants + 1): cm^3/mol/s
    A_cgs = 5e9
    k = A_cgs * 1e-6
    o = oracle_lib.Oracle(toymech.write(toymech.thirdbody_iso(A=A_cgs), "tb"))
    Y = np.array([0.25, 0.0, 0.75])
    rho, e = _one_cell(o, 1000.0, 3e5, Y)
    CN2 = rho * Y[2] / o.W[2]
    for dt in (1e-6, 1e-5):
        Yo, To, st = o.integrate([rho], [e], Y.reshape(3, 1), dt, 1e-11, 1e-16)
        assert Yo[0, 0] == pytest.approx(Y[0] * np.exp(-k * CN2 * dt), rel=1e-8)


def test_lindemann_closed_form(oracle_lib):
    Ainf, A0 = 3e5, 1e12    # 1/s and cm^3/mol/s
    o = oracle_lib.Oracle(toymech.write(toymech.falloff_iso(Ainf=Ainf, A0=A0), "lind2"))
    Y = np.array([0.25, 0.0, 0.75])
    rho, e = _one_cell(o, 1000.0, 2e5, Y)
    M = rho * Y[2] / o.W[2]
    Pr = A0 * 1e-6 * M / Ainf
    keff = Ainf * Pr / (1 + Pr)
    Yo, To, st = o.integrate([rho], [e], Y.reshape(3, 1), 2e-6, 1e-11, 1e-16)
    assert Yo[0, 0] == pytest.approx(Y[0] * np.exp(-keff * 2e-6), rel=1e-8)


def _c1(o, n, seed=1001):
    c = fields.c1_cells(n, seed=seed)
    rho, e = o.state_from_TPY(c.T, c.p, c.Y)
    return c, rho, e


def test_radau_cross_check(m9):
    # independent integrator family (implicit Runge-Kutta, scipy) on the oracle RHS
    c, rho, e = _c1(m9, 32)
    Yo, To, st = m9.integrate(rho, e, c.Y, 1e-7, 1e-12, 1e-20, T=c.T)
    assert np.all(st == 0)
    for i in range(32):
        y0 = np.concatenate([c.Y[:, i], [m9.T_from_e(e[i], c.Y[:, i])]])
        sol = solve_ivp(lambda t, y: m9.rhs(rho[i], y), (0.0, 1e-7), y0, method="Radau",
                        rtol=1e-12, atol=np.r_[np.full(m9.ns, 1e-20), 1e-9],
                        jac=lambda t, y: m9.jac(rho[i], y))
        yr = sol.y[:, -1]
        big = yr[:-1] > 1e-10
        assert np.all(np.abs(Yo[big, i] - yr[:-1][big]) <= 1e-8 * yr[:-1][big] + 1e-16)
        assert abs(To[i] - yr[-1]) < 1e-7


def test_conservation_at_tight_tolerance(m9):
    c, rho, e = _c1(m9, 64, seed=77)
    Yo, To, st = m9.integrate(rho, e, c.Y, 1e-6, 1e-12, 1e-20, T=c.T)
    assert np.all(st == 0)
    assert np.max(np.abs(Yo.sum(0) - 1.0)) < 1e-13
    el0 = m9.comp.T @ (c.Y / m9.W[:, None])
    el1 = m9.comp.T @ (Yo / m9.W[:, None])
    assert np.max(np.abs(el1 - el0) / el0.max(0)) < 1e-13
    for i in range(64):
        assert m9.e_mass(To[i], Yo[:, i]) == pytest.approx(e[i], rel=1e-10, abs=1e-10 * 3e6)


def test_long_time_equilibrium_matches_gibbs(m9):
    c, rho, e = _c1(m9, 6, seed=5)
    Yo, To, st = m9.integrate(rho, e, c.Y, 1.0, 1e-11, 1e-22, T=c.T)
    assert np.all(st == 0)
    for i in range(6):
        p = rho[i] * R * To[i] * np.sum(Yo[:, i] / m9.W)
        b = gibbs.element_moles_from_Y(m9, c.Y[:, i])
        Ye = gibbs.Y_from_X(m9, gibbs.equilibrate_TP(m9, To[i], p, b))
        big = Ye > 1e-10
        assert np.all(np.abs(Yo[big, i] - Ye[big]) <= 1e-6 * Ye[big]), (i, Yo[:, i], Ye)


def _ignition_delay(o, T0, rtol):
    X = np.zeros(o.ns)
    X[0], X[1], X[-1] = 2.0, 1.0, 3.76
    Y = gibbs.Y_from_X(o, X / X.sum())
    rho, e = _one_cell(o, T0, 101325.0, Y)
    tout = np.linspace(0.0, 3e-4 if T0 < 1200 else 4e-5, 4001)
    yo, st = o.trajectory(rho, e, Y, tout[-1], tout, rtol, rtol * 1e-6)
    assert st == 0
    dT = np.array([o.rhs(rho, yo[i])[-1] for i in range(len(tout))])
    i = int(np.argmax(dT))
    # parabolic refinement of the maximum of dT/dt
    a, b, cc = dT[i - 1], dT[i], dT[i + 1]
    h = tout[1] - tout[0]
    return tout[i] + 0.5 * h * (a - cc) / (a - 2 * b + cc)


def test_ignition_delay_converges_under_refinement(m9):
    for T0 in (1100.0, 1800.0):
        taus = [_ignition_delay(m9, T0, r) for r in (1e-6, 1e-8, 1e-10, 1e-12)]
        d = np.abs(np.diff(taus))
        assert d[-1] < d[0] and d[-1] < 1e-5 * taus[-1], (T0, taus)
        assert 1e-6 < taus[-1] < 1e-3


def test_kmax_status(m9):
    c, rho, e = _c1(m9, 4)
    Yo, To, st = m9.integrate(rho, e, c.Y, 1e-7, 1e-8, 1e-14, T=c.T, max_steps=3)
    assert np.all(st == oracle.ST_KMAX)
