"""The oracle's minimal flow step (HLLC + MUSCL + SSP-RK2, Sec. 2.1) pinned
by the exact solution of the Riemann problem for a calorically perfect gas,
the exact preservation of uniform flow and of a stationary contact,
conservation, mirror symmetry, and the Strang coupling's reduction to the
chemistry alone on a uniform state."""
import numpy as np
import pytest

from oracle import oflow
from synth import fields
from synth.mechfile import Mechanism, Species
from tests.toymech import write

R = 8.314462618


@pytest.fixture(scope="module")
def ideal(oracle_lib):
    # one species with cp/R = 3.5 and no formation energy: gamma = 1.4, e = cv T
    a = [3.5, 0, 0, 0, 0, 0.0, 4.0]
    m = Mechanism("ideal", ["N"], [Species("Q", {"N": 2}, a, a, W=28.0)], [])
    return oracle_lib.Oracle(write(m, "ideal"))


def exact_riemann(rL, uL, pL, rR, uR, pR, g, x_over_t):
    """Exact solution of the Riemann problem for an ideal gas with constant
    gamma (Toro, Ch. 4): Newton on the pressure function, then sampling."""
    cL, cR = np.sqrt(g * pL / rL), np.sqrt(g * pR / rR)

    def fk(p, rk, pk, ck):
        if p > pk:   # shock
            A, B = 2.0 / ((g + 1) * rk), (g - 1) / (g + 1) * pk
            q = np.sqrt(A / (p + B))
            return (p - pk) * q, q * (1 - 0.5 * (p - pk) / (B + p))
        pr = p / pk  # rarefaction
        return 2 * ck / (g - 1) * (pr ** ((g - 1) / (2 * g)) - 1), 1.0 / (rk * ck) * pr ** (-(g + 1) / (2 * g))

    p = 0.5 * (pL + pR)
    for _ in range(100):
        f1, d1 = fk(p, rL, pL, cL)
        f2, d2 = fk(p, rR, pR, cR)
        dp = (f1 + f2 + uR - uL) / (d1 + d2)
        p = max(p - dp, 1e-12 * p)
        if abs(dp) < 1e-14 * p:
            break
    us = 0.5 * (uL + uR) + 0.5 * (fk(p, rR, pR, cR)[0] - fk(p, rL, pL, cL)[0])
    out = []
    for s in x_over_t:
        if s <= us:   # left of the contact
            if p > pL:
                SL = uL - cL * np.sqrt((g + 1) / (2 * g) * p / pL + (g - 1) / (2 * g))
                out.append((rL, uL, pL) if s <= SL else
                           (rL * (p / pL + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * p / pL + 1), us, p))
            else:
                csL = cL * (p / pL) ** ((g - 1) / (2 * g))
                if s <= uL - cL:
                    out.append((rL, uL, pL))
                elif s >= us - csL:
                    out.append((rL * (p / pL) ** (1 / g), us, p))
                else:
                    u = 2 / (g + 1) * (cL + (g - 1) / 2 * uL + s)
                    c = 2 / (g + 1) * (cL + (g - 1) / 2 * (uL - s))
                    r = rL * (c / cL) ** (2 / (g - 1))
                    out.append((r, u, pL * (c / cL) ** (2 * g / (g - 1))))
        else:
            if p > pR:
                SR = uR + cR * np.sqrt((g + 1) / (2 * g) * p / pR + (g - 1) / (2 * g))
                out.append((rR, uR, pR) if s >= SR else
                           (rR * (p / pR + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * p / pR + 1), us, p))
            else:
                csR = cR * (p / pR) ** ((g - 1) / (2 * g))
                if s >= uR + cR:
                    out.append((rR, uR, pR))
                elif s <= us + csR:
                    out.append((rR * (p / pR) ** (1 / g), us, p))
                else:
                    u = 2 / (g + 1) * (-cR + (g - 1) / 2 * uR + s)
                    c = 2 / (g + 1) * (cR - (g - 1) / 2 * (uR - s))
                    r = rR * (c / cR) ** (2 / (g - 1))
                    out.append((r, u, pR * (c / cR) ** (2 * g / (g - 1))))
    return np.array(out).T


def _sod(orc, n):
    x = (np.arange(n) + 0.5) / n
    left = x < 0.5
    rho = np.where(left, 1.0, 0.125)
    p = np.where(left, 1e5, 1e4)
    u = np.zeros(n)
    Y = np.ones((1, n))
    return x, oflow.cons_from_prim(orc, rho, u, p, Y)


def test_sod_against_exact_riemann_solution(ideal):
    errs = []
    t_end = 5e-4
    for n in (100, 200, 400):
        x, U = _sod(ideal, n)
        dx = 1.0 / n
        dt = 0.4 * dx / 450.0                   # CFL 0.4 with max |u| + c below 450 m/s
        nsteps = int(np.ceil(t_end / dt))
        dt = t_end / nsteps
        for _ in range(nsteps):
            U = oflow.flow_step(ideal, U, dx, dt)
        rho_ex, u_ex, p_ex = exact_riemann(1.0, 0.0, 1e5, 0.125, 0.0, 1e4, 1.4, (x - 0.5) / t_end)
        errs.append(np.mean(np.abs(U[0] - rho_ex)))
        rho, u, p, T, Y = oflow.prim_from_cons(ideal, U)
        assert np.mean(np.abs(p - p_ex)) < 0.03 * 1e5
        assert np.mean(np.abs(u - u_ex)) < 0.03 * 300.0
    print("L1 density errors", errs)
    assert errs[0] < 0.02
    assert errs[2] < 0.7 * errs[1] < 0.7 * 0.7 * errs[0]


def test_uniform_flow_and_stationary_contact_are_exact(oracle_lib, m9):
    n = 64
    c = fields.c1_cells(1, seed=5)
    Y = np.repeat(c.Y, n, axis=1)
    rho = np.full(n, 2.0)
    U = oflow.cons_from_prim(m9, rho, np.full(n, 150.0), np.full(n, 3e5), Y)
    U1 = oflow.flow_step(m9, U, 1e-4, 1e-8)
    assert np.allclose(U1, U, rtol=1e-14, atol=0)
    # u = 0 and uniform p with a jump in density and composition: HLLC keeps it still
    Y2 = Y.copy()
    c2 = fields.c1_cells(2, seed=6)
    Y2[:, n // 2:] = c2.Y[:, 1:2]
    rho2 = np.where(np.arange(n) < n // 2, 2.0, 0.7)
    U = oflow.cons_from_prim(m9, rho2, np.zeros(n), np.full(n, 3e5), Y2)
    U1 = oflow.flow_step(m9, U, 1e-4, 1e-8)
    scale = np.abs(U).max(axis=1, keepdims=True)
    scale[1] = 2.0 * 1000.0                    # momentum: rho c (the state has none)
    assert np.allclose(U1, U, rtol=1e-12, atol=1e-12 * scale)


def test_conservation_and_mirror_symmetry(m9):
    n = 120
    x = (np.arange(n) + 0.5) / n
    c = fields.c1_cells(n, seed=8)
    bump = np.exp(-((x - 0.5) / 0.08) ** 2)
    rho = 1.0 + 0.5 * bump
    p = 1e5 * (1.0 + 2.0 * bump)
    u = 40.0 * np.sin(2 * np.pi * x) * bump
    Y = c.Y
    Y = 0.5 * (Y + Y[:, ::-1])                 # symmetric composition
    U = oflow.cons_from_prim(m9, rho, u, p, Y)
    Um = oflow.cons_from_prim(m9, rho[::-1], -u[::-1], p[::-1], Y[:, ::-1])
    dx, dt = 1e-3, 2e-7
    for _ in range(5):
        U = oflow.flow_step(m9, U, dx, dt)
        Um = oflow.flow_step(m9, Um, dx, dt)
    tot0 = oflow.cons_from_prim(m9, rho, u, p, Y).sum(axis=1)
    assert np.allclose(U.sum(axis=1), tot0, rtol=1e-13, atol=1e-13 * np.abs(tot0).max())
    mir = Um[:, ::-1].copy()
    mir[1] = -mir[1]
    assert np.allclose(U, mir, rtol=1e-11, atol=1e-11 * np.abs(U).max(axis=1, keepdims=True))


def test_strang_step_on_a_uniform_state_is_the_chemistry_alone(m9):
    # no gradients: both flow half steps leave U unchanged, so one Strang step
    # equals the chemistry of one cell over dt
    n = 8
    c = fields.c1_cells(1, seed=12)
    Y = np.repeat(c.Y, n, axis=1)
    T = np.full(n, c.T[0])
    rho, e = m9.state_from_TPY(T, c.p[0], Y)
    U = oflow.cons_from_prim(m9, rho, np.full(n, 30.0), np.full(n, c.p[0]), Y)
    U1, st = oflow.strang_step(m9, U, 1e-4, 1e-7, 1e-10, 1e-20)
    assert np.all(st == 0)
    Yo, To, so = m9.integrate(rho[:1], e[:1], Y[:, :1], 1e-7, 1e-10, 1e-20, T=T[:1])
    assert np.allclose(U1[3:] / U1[0], np.repeat(Yo, n, axis=1), rtol=1e-12, atol=1e-18)
    assert np.allclose(U1[:3], U[:3], rtol=1e-13)
