"""Pins of the CPU explicit scheme (the paper's first-order kinetics steps,
Sec. 2.1 / Alg. 2): the closed form of the discrete scheme on an
irreversible isomerisation, first-order convergence to the exact solution,
and conservation plus convergence to the BDF oracle on the 9-species
mechanism."""
import numpy as np
import pytest

from oracle import oexplicit
from synth import fields
from tests import toymech


def _one_cell(o, T, p, Y):
    rho, e = o.state_from_TPY(np.array([T]), p, np.asarray(Y, dtype=float).reshape(-1, 1))
    return rho, e


@pytest.fixture(scope="module")
def iso(oracle_lib):
    kf = 2.0e6
    return kf, oracle_lib.Oracle(toymech.write(toymech.isomer_AB(A=kf, reversible=False), "iso_irr"))


def test_discrete_closed_form(iso):
    # A -> B at rate kf with Y_B >= Y_A throughout: A's limit binds, every full
    # step is frac/kf and multiplies Y_A by (1 - frac); dt = 10.5 full steps
    kf, o = iso
    frac = 0.02
    Y = np.array([0.2, 0.3, 0.5])
    T0 = 1300.0
    rho, e = _one_cell(o, T0, 2e5, Y)
    dt = 10.5 * frac / kf
    Yo, To, st, steps = oexplicit.integrate_explicit(o, rho, e, Y.reshape(3, 1), [T0], dt, frac)
    assert st[0] == 0 and steps[0] == 11
    A = 0.2 * (1 - frac) ** 10 * (1 - 0.5 * frac)
    assert Yo[0, 0] == pytest.approx(A, rel=1e-12)
    assert Yo[1, 0] == pytest.approx(0.5 - A, rel=1e-12)
    assert Yo[2, 0] == 0.5
    assert To[0] == pytest.approx(T0, abs=1e-8)


def test_first_order_convergence(iso):
    kf, o = iso
    Y = np.array([0.2, 0.3, 0.5])
    rho, e = _one_cell(o, 1300.0, 2e5, Y)
    dt = 3.0 / kf
    exact = 0.2 * np.exp(-kf * dt)
    err = []
    for frac in (0.02, 0.01, 0.005):
        Yo, _, st, _ = oexplicit.integrate_explicit(o, rho, e, Y.reshape(3, 1), [1300.0], dt, frac)
        assert st[0] == 0
        err.append(abs(Yo[0, 0] - exact) / exact)
    assert 1.8 < err[0] / err[1] < 2.2 and 1.8 < err[1] / err[2] < 2.2
    assert err[2] < 1e-2


def test_zero_species_does_not_stall(iso):
    # B starts at zero: the floor under the relative limit keeps steps finite
    kf, o = iso
    Y = np.array([0.5, 0.0, 0.5])
    rho, e = _one_cell(o, 1300.0, 2e5, Y)
    Yo, _, st, steps = oexplicit.integrate_explicit(o, rho, e, Y.reshape(3, 1), [1300.0], 1.0 / kf, 0.05)
    assert st[0] == 0 and steps[0] < 2000
    assert Yo[0, 0] + Yo[1, 0] == pytest.approx(0.5, rel=1e-13)
    assert Yo[0, 0] == pytest.approx(0.5 * np.exp(-1.0), rel=0.05)


def test_m9_conservation_and_convergence_to_bdf(m9):
    c = fields.c1_cells(5, seed=2024)
    rho, e = m9.state_from_TPY(c.T, c.p, c.Y)
    Yr, Tr, st = m9.integrate(rho, e, c.Y, c.dt, 1e-12, 1e-20, T=c.T)
    assert np.all(st == 0)
    big = Yr > 1e-6
    errs = []
    for frac in (0.02, 0.01):
        Yx, Tx, sx, steps = oexplicit.integrate_explicit(m9, rho, e, c.Y, c.T, c.dt, frac)
        assert np.all(sx == 0)
        assert np.allclose(Yx.sum(axis=0), c.Y.sum(axis=0), rtol=0, atol=1e-12)
        for i in range(rho.size):
            assert m9.e_mass(Tx[i], Yx[:, i]) == pytest.approx(e[i], rel=1e-10)
        errs.append(np.where(big, np.abs(Yx - Yr) / np.where(big, Yr, 1.0), 0.0).max(axis=0))
    # first order, cell by cell, where the scheme's error is above rounding
    sel = errs[1] > 1e-9
    assert sel.any()
    ratio = errs[0][sel] / errs[1][sel]
    assert np.all((ratio > 1.5) & (ratio < 2.5)), ratio
