"""Throughput at fixed error on the detonation patch: the FP64 and the
FP32-exponential modes across tolerances, each timed on the whole
256x256x32 field and checked on a sample of its integrated cells against the
FP64 oracle at tight tolerance.  The budget is 1e-4 relative on species
above 1e-10 and 1 K; the test reports which settings meet it and asserts
that the FP64 path at the default tolerances does."""
import numpy as np
import pytest

from synth import fields
from tests.gpu_util import JUDGE_ATOL, JUDGE_RTOL, host

pytestmark = pytest.mark.gpu

BUDGET_REL, BUDGET_T = 1e-4, 1.0


@pytest.fixture(scope="module")
def setup(m9):
    import torch
    import paper_2510_23993_amd as chem
    cells = fields.c2_field(256, 256, 32)
    n = cells.T.size
    mech = chem.Mechanism(fields.M9_PATH)
    ctx = chem.Context(mech)
    T0 = torch.as_tensor(cells.T, device="cuda")
    Y0 = torch.as_tensor(cells.Y, device="cuda").contiguous()
    rho = torch.empty(n, dtype=torch.float64, device="cuda")
    e = torch.empty_like(rho)
    ctx.prepare_state(T0, torch.as_tensor(cells.p, device="cuda"), Y0, rho, e)
    rng = np.random.default_rng(7)
    hot = np.where(cells.cls > 0)[0]
    idx = np.sort(rng.choice(hot, 400, replace=False))
    rho_h, e_h = host(rho)[idx], host(e)[idx]
    Yr, Tr, st = m9.integrate(rho_h, e_h, cells.Y[:, idx], cells.dt, JUDGE_RTOL, JUDGE_ATOL, T=cells.T[idx])
    assert np.all(st == 0)
    return chem, mech, cells, T0, Y0, rho, e, idx, Yr, Tr


def _run(setup, precision, rtol, atol=1e-14, algorithm=1):
    import torch
    chem, mech, cells, T0, Y0, rho, e, idx, Yr, Tr = setup
    ctx = chem.Context(mech, precision=precision, algorithm=algorithm)
    Y, T = torch.empty_like(Y0), torch.empty_like(T0)
    best = None
    for _ in range(2):
        Y.copy_(Y0)
        T.copy_(T0)
        st = ctx.integrate(rho, e, Y, T, cells.dt, rtol, atol)
        best = st if best is None or st["t_total_ms"] < best["t_total_ms"] else best
    Yg, Tg = host(Y)[:, idx], host(T)[idx]
    big = Yr > 1e-10
    rel = float(np.where(big, np.abs(Yg - Yr) / np.where(big, Yr, 1.0), 0.0).max())
    return best, rel, float(np.abs(Tg - Tr).max())


def test_throughput_at_fixed_error(setup):
    rows = []
    for precision in (0, 1):
        for rtol in (1e-4, 1e-5, 1e-6, 1e-7, 1e-8, 1e-9, 1e-10):
            st, rel, dT = _run(setup, precision, rtol)
            ok = rel <= BUDGET_REL and dT <= BUDGET_T and st["n_incomplete"] == 0
            rows.append((precision, rtol, st["t_total_ms"], rel, dT, ok, st["attempts_total"]))
    plain = []
    for rtol in (1e-4, 1e-5, 1e-8):   # every cell, no skip, no compaction
        st, rel, dT = _run(setup, 0, rtol, algorithm=0)
        plain.append((rtol, st["t_total_ms"], rel, dT, rel <= BUDGET_REL and dT <= BUDGET_T))
    print("\nmode  rtol    ms      max rel   max |dT| K  budget  attempts")
    for p, r, ms, rel, dT, ok, att in rows:
        print(f"{'fp32x' if p else 'fp64 '} {r:.0e} {ms:8.2f} {rel:9.2e} {dT:9.2e}  {'yes' if ok else 'no ':3s}  {att}")
    for r, ms, rel, dT, ok in plain:
        print(f"plain {r:.0e} {ms:8.2f} {rel:9.2e} {dT:9.2e}  {'yes' if ok else 'no ':3s}")
    ok_rows = [r for r in rows if r[5]]
    best = min(ok_rows, key=lambda r: r[2])
    fp64_default = [r for r in rows if r[0] == 0 and r[1] == 1e-8][0]
    print(f"fastest within budget: {'fp32x' if best[0] else 'fp64'} at rtol {best[1]:.0e}, {best[2]:.2f} ms "
          f"({fp64_default[2] / best[2]:.2f}x the FP64 path at rtol 1e-8)")
    assert fp64_default[5]


def test_bench_configuration_sample(setup):
    """The whole 2,097,152-cell field in the benchmark's launch configuration
    (the options its autotuner picks: one lane per cell, 24 bulk-round
    launches of 20 steps, N* = 1e5) at its tolerances (rtol 1e-8, atol
    1e-14): the 400 sampled hot cells against the oracle at tight tolerance,
    relative bound where the relative tolerance dominates (Y > 1e-6),
    temperature everywhere."""
    import torch
    chem, mech, cells, T0, Y0, rho, e, idx, Yr, Tr = setup
    ctx = chem.Context(mech, group=0, max_rounds=24, nactive_star=100000, kmax_bulk=20)
    Y, T = Y0.clone(), T0.clone()
    status = torch.zeros(T.numel(), dtype=torch.uint8, device="cuda")
    st = ctx.integrate(rho, e, Y, T, cells.dt, 1e-8, 1e-14, status=status)
    assert st["rc"] == 0 and int(status.max()) <= chem.ST_SKIPPED
    Yg, Tg = host(Y)[:, idx], host(T)[idx]
    dom = Yr > 1e-14 / 1e-8
    rel = float(np.where(dom, np.abs(Yg - Yr) / np.where(dom, Yr, 1.0), 0.0).max())
    dT = float(np.abs(Tg - Tr).max())
    print(f"bench configuration ({st['t_total_ms']:.1f} ms): max rel (Y > 1e-6) {rel:.2e}, max |dT| {dT:.2e} K")
    assert rel <= 1e-6 and dT <= 1e-3
