"""The paper's explicit first-order scheme (method = 1) on the GPU against
the oracle's implementation of the same scheme, option checks, and its error
and time on the detonation patch beside the BDF path.

Tolerance: both sides take the same steps of the same discrete scheme (the
step counts agree); they differ by the rounding of the rates (log form
against integer powers, ~1e-14 relative) and by where each temperature
Newton iteration stops (1e-12 T), which the hundreds of steps of a cell
carry forward, largest relative to species just above 1e-10.  The bound is
the path's parity criterion: 1e-6 relative on species above 1e-10, 1e-3 K
(measured on C1: 2.2e-7, 6e-8 K)."""
import numpy as np
import pytest

from oracle import oexplicit
from synth import fields
from tests.gpu_util import JUDGE_ATOL, JUDGE_RTOL, host, oracle_inputs, run_gpu, to_dev

pytestmark = pytest.mark.gpu

REL, TABS = 1e-6, 1e-3


@pytest.fixture(scope="module")
def chem():
    import paper_2510_23993_amd as chem
    return chem


@pytest.fixture(scope="module")
def mech(chem, m9_path):
    return chem.Mechanism(m9_path)


def _rel(Yg, Yr):
    big = Yr > 1e-10
    return float(np.where(big, np.abs(Yg - Yr) / np.where(big, Yr, 1.0), 0.0).max())


@pytest.mark.parametrize("frac", [0.05, 0.01])
def test_explicit_vs_oracle_c1(chem, mech, m9, frac):
    c = fields.c1_cells(64 + 5, seed=2025)
    rho, e = oracle_inputs(m9, c)
    Yr, Tr, sr, kr = oexplicit.integrate_explicit(m9, rho, e, c.Y, c.T, c.dt, frac)
    assert np.all(sr == 0)
    ctx = chem.Context(mech, method=1, explicit_frac=frac)
    Yg, Tg, st, stats = run_gpu(ctx, rho, e, c.Y, c.T, c.dt, 1e-8, 1e-14)
    assert stats["rc"] == 0 and np.all(st == 0), np.bincount(st)
    assert stats["steps_total"] == pytest.approx(kr.sum(), rel=1e-3)
    rel, dT = _rel(Yg, Yr), float(np.abs(Tg - Tr).max())
    print(f"explicit frac {frac}: {kr.sum()} steps (oracle) / {stats['steps_total']} (GPU), "
          f"max rel {rel:.2e}, max |dT| {dT:.2e} K")
    assert rel <= REL and dT <= TABS


def test_explicit_skips_cold_and_masked_cells(chem, mech, m9):
    c = fields.c1_cells(40, seed=2026)
    c.T[:10] = 320.0
    rho, e = oracle_inputs(m9, c)
    mask = np.zeros(40, dtype=np.uint8)
    mask[10:15] = 1
    ctx = chem.Context(mech, method=1)
    Yg, Tg, st, stats = run_gpu(ctx, rho, e, c.Y, c.T, c.dt, 1e-8, 1e-14, mask=mask)
    assert np.all(st[:15] == chem.ST_SKIPPED) and np.all(st[15:] == chem.ST_DONE)
    assert np.array_equal(Yg[:, :15], c.Y[:, :15])
    Yr, Tr, sr, _ = oexplicit.integrate_explicit(m9, rho[15:], e[15:], c.Y[:, 15:], c.T[15:], c.dt, 0.01)
    assert _rel(Yg[:, 15:], Yr) <= REL


def test_explicit_options(chem, mech, m9_path):
    ctx = chem.Context(mech)
    assert ctx.get_option("method") == 0 and ctx.get_option("explicit_frac") == 0.01
    for k, v in (("method", 2), ("explicit_frac", 0.2), ("explicit_frac", 0.0)):
        with pytest.raises(chem.ChemError) as ei:
            ctx.set_option(k, v)
        assert ei.value.rc == -1
    m53 = chem.Mechanism(fields.M53_PATH)
    with pytest.raises(chem.ChemError) as ei:
        chem.Context(m53).set_option("method", 1)
    assert ei.value.rc == -1


def test_explicit_on_detonation_patch(chem, mech, m9):
    """The full 256x256x32 field: 48 sampled integrated cells against the
    oracle's explicit scheme (parity), and the error of the scheme itself
    against the tight BDF oracle beside the BDF path's, with both times."""
    import torch
    cells = fields.c2_field(256, 256, 32)
    n = cells.T.size
    rho, e = oracle_inputs(m9, cells)
    d_rho, d_e = to_dev(rho), to_dev(e)
    idx = np.sort(np.random.default_rng(9).choice(np.where(cells.cls > 0)[0], 48, replace=False))
    Yj, Tj, sj = m9.integrate(rho[idx], e[idx], cells.Y[:, idx], cells.dt, JUDGE_RTOL, JUDGE_ATOL, T=cells.T[idx])
    assert np.all(sj == 0)
    rows = []
    for frac in (0.05, 0.01):
        ctx = chem.Context(mech, method=1, explicit_frac=frac)
        Y, T = to_dev(cells.Y), to_dev(cells.T)
        status = torch.zeros(n, dtype=torch.uint8, device="cuda")
        st = ctx.integrate(d_rho, d_e, Y, T, cells.dt, 1e-8, 1e-14, status=status)
        assert st["rc"] == 0
        Yg, Tg = host(Y)[:, idx], host(T)[idx]
        Yr, Tr, sr, _ = oexplicit.integrate_explicit(m9, rho[idx], e[idx], cells.Y[:, idx], cells.T[idx],
                                                     cells.dt, frac)
        assert _rel(Yg, Yr) <= REL and np.abs(Tg - Tr).max() <= TABS
        rows.append((f"explicit {frac}", st["t_total_ms"], st["steps_total"], _rel(Yg, Yj),
                     float(np.abs(Tg - Tj).max())))
    ctx = chem.Context(mech)
    Y, T = to_dev(cells.Y), to_dev(cells.T)
    st = ctx.integrate(d_rho, d_e, Y, T, cells.dt, 1e-8, 1e-14)
    rows.append(("BDF 1e-8", st["t_total_ms"], st["steps_total"], _rel(host(Y)[:, idx], Yj),
                 float(np.abs(host(T)[idx] - Tj).max())))
    print()
    for name, ms, steps, rel, dT in rows:
        print(f"{name:14s} {ms:9.2f} ms {steps:10d} steps  error vs oracle: {rel:.2e} rel, {dT:.2e} K")
    assert rows[1][3] < rows[0][3]      # first order: the smaller step limit is closer
