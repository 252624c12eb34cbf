"""GPU parity on the two-range variant of the 9-species mechanism (distinct
NASA-7 sets below and above Tmid = 1000 K, same reaction structure, so the
compiled one-lane kernels run it): RHS, Jacobian, state preparation and the
full integration with temperatures on both sides of Tmid, for the compiled
one-lane and the cooperative schedules."""
import numpy as np
import pytest

from synth import fields
from tests.gpu_util import JUDGE_ATOL, JUDGE_RTOL, host, parity_report, run_gpu, to_dev

pytestmark = pytest.mark.gpu

R = 8.314462618


@pytest.fixture(scope="module")
def o2r(oracle_lib):
    return oracle_lib.Oracle(fields.M9_TWO_RANGE_PATH)


@pytest.fixture(scope="module")
def mech2r():
    import paper_2510_23993_amd as chem
    return chem.Mechanism(fields.M9_TWO_RANGE_PATH)


def _cells_near_tmid(n, seed):
    c = fields.c1_cells(n, seed=seed)
    c.T = np.random.default_rng(seed).uniform(850.0, 1150.0, n)
    return c


def test_two_range_uses_the_compiled_kernels(mech2r, m9_path):
    import paper_2510_23993_amd as chem
    assert mech2r.hash == chem.Mechanism(m9_path).hash
    chem.Context(mech2r, group=0)       # refused for mechanisms without compiled kernels


@pytest.mark.parametrize("group", [0, 16])
def test_two_range_rhs_jacobian_and_state(mech2r, o2r, group):
    import torch
    import paper_2510_23993_amd as chem
    ctx = chem.Context(mech2r, group=group)
    n = 4000
    rng = np.random.default_rng(31)
    T = rng.uniform(700.0, 1300.0, n)
    p = rng.uniform(0.5, 30.0, n) * 101325.0
    Y = rng.dirichlet(np.ones(o2r.ns) * 0.6, n).T.copy()
    rho = p / (R * T * np.sum(Y / o2r.W[:, None], axis=0))
    y = np.vstack([Y, T[None, :]])
    f = torch.zeros((o2r.n, n), dtype=torch.float64, device="cuda")
    J = torch.zeros((o2r.n * o2r.n, n), dtype=torch.float64, device="cuda")
    ctx.eval_rhs(to_dev(rho), to_dev(y), f, J)
    rho_d, e_d = torch.zeros(n, dtype=torch.float64, device="cuda"), torch.zeros(n, dtype=torch.float64, device="cuda")
    ctx.prepare_state(to_dev(T), to_dev(p), to_dev(Y), rho_d, e_d)
    torch.cuda.synchronize()
    rho_o, e_o = o2r.state_from_TPY(T, p, Y)
    assert np.allclose(host(rho_d), rho_o, rtol=1e-14, atol=0)
    assert np.allclose(host(e_d), e_o, rtol=1e-12, atol=1e-9)
    fg, Jg = host(f), host(J).reshape(o2r.n, o2r.n, n)
    worst_f = worst_J = 0.0
    for c in range(0, n, 11):
        fo, Jo = o2r.rhs(rho[c], y[:, c]), o2r.jac(rho[c], y[:, c])
        kf, kr, qf, qr = o2r.rates(T[c], rho[c] * Y[:, c] / o2r.W)
        gross = np.sum(np.abs(qf) + np.abs(qr)) * max(o2r.W) * 3 / rho[c]
        worst_f = max(worst_f, np.max(np.abs(fg[:-1, c] - fo[:-1])) / gross,
                      abs(fg[-1, c] - fo[-1]) / (abs(fo[-1]) + gross * 1e4))
        ysc = np.maximum(np.abs(y[:, c]), 1e-8)
        for i in range(o2r.n):
            sc = np.max(np.abs(Jo[i] * ysc))
            worst_J = max(worst_J, np.max(np.abs(Jg[i, :, c] - Jo[i]) * ysc) / (sc + 1e-300))
    print(f"two-range group={group}: rhs {worst_f:.2e}, jac {worst_J:.2e}")
    assert worst_f < 1e-12 and worst_J < 1e-11


@pytest.mark.parametrize("group", [0, 16])
def test_two_range_integration_parity(mech2r, o2r, group):
    import paper_2510_23993_amd as chem
    c = _cells_near_tmid(1024 + 29, seed=77)
    rho, e = o2r.state_from_TPY(c.T, c.p, c.Y)
    Yr, Tr, st = o2r.integrate(rho, e, c.Y, c.dt, JUDGE_RTOL, JUDGE_ATOL, T=c.T)
    assert np.all(st == 0)
    below = (c.T < 1000.0).sum()
    assert 100 < below < c.T.size - 100      # both ranges are exercised
    ctx = chem.Context(mech2r, group=group, t_react_min=0.0)
    Yg, Tg, sg, stats = run_gpu(ctx, rho, e, c.Y, c.T, c.dt, 1e-8, 1e-20)
    assert stats["rc"] == 0 and np.all(sg == 0)
    rel, dT, _ = parity_report(Yg, Tg, Yr, Tr)
    print(f"two-range integration group={group}: max rel {rel:.2e}, |dT| {dT:.2e} K ({below} cells below Tmid)")
    assert rel <= 1e-6 and dT <= 1e-3
