"""HIP path vs the CPU oracle through the C ABI: building blocks (state
preparation, RHS, Jacobian) and the full integration (plain and
bulk-sparse) at the C1 tolerances, element by element."""
import numpy as np
import pytest

from synth import fields
from tests.gpu_util import (ATOL_C1, JUDGE_ATOL, JUDGE_RTOL, RTOL_C1, SPECIES_REL, T_ABS, host,
                            oracle_inputs, parity_report, run_gpu, to_dev)

pytestmark = pytest.mark.gpu

R = 8.314462618


@pytest.fixture(scope="module")
def chem():
    import paper_2510_23993_amd as chem
    return chem


@pytest.fixture(scope="module")
def mech(chem, m9_path):
    return chem.Mechanism(m9_path)


@pytest.fixture()
def ctx(chem, mech):
    return chem.Context(mech)


# 0 = compiled kernel with one cell per lane; G > 0 = G lanes cooperate on a cell
SCHEDULES = [0, 8, 16, 64]


def test_mechanism_info(mech, m9):
    assert mech.ns == 9 and mech.nr == 21
    assert mech.species == m9.species
    assert np.allclose(mech.W, m9.W, rtol=0, atol=0)


def test_prepare_state_vs_oracle(ctx, m9):
    import torch
    c = fields.c1_cells(1000 + 37, seed=11)
    rho_o, e_o = oracle_inputs(m9, c)
    n = c.T.size
    rho, e = torch.zeros(n, dtype=torch.float64, device="cuda"), torch.zeros(n, dtype=torch.float64, device="cuda")
    ctx.prepare_state(to_dev(c.T), to_dev(c.p), to_dev(c.Y), rho, e)
    torch.cuda.synchronize()
    assert np.allclose(host(rho), rho_o, rtol=1e-14, atol=0)
    assert np.allclose(host(e), e_o, rtol=1e-12, atol=1e-9)


def _random_states(m, n, seed):
    """Random states; one entry in ten is a small negative mass fraction (an
    implicit integrator's iterates and error-controlled solutions can hold
    them), where mass action is the signed integer power."""
    rng = np.random.default_rng(seed)
    T = rng.uniform(300.0, 3200.0, n)
    p = rng.uniform(0.5, 40.0, n) * 101325.0
    Y = rng.dirichlet(np.ones(m.ns) * 0.6, n).T.copy()
    neg = rng.uniform(size=Y.shape) < 0.1
    Y[neg] = -1e-3 * Y[neg]
    rho = p / (R * T * np.sum(Y / m.W[:, None], axis=0))
    return rho, np.vstack([Y, T[None, :]])


@pytest.mark.parametrize("group", SCHEDULES)
def test_rhs_and_jacobian_vs_oracle(chem, mech, m9, group):
    import torch
    ctx = chem.Context(mech, group=group)
    n = 10000
    rho, y = _random_states(m9, n, 21)
    f = torch.zeros((m9.n, n), dtype=torch.float64, device="cuda")
    J = torch.zeros((m9.n * m9.n, n), dtype=torch.float64, device="cuda")
    ctx.eval_rhs(to_dev(rho), to_dev(y), f, J)
    torch.cuda.synchronize()
    fg, Jg = host(f), host(J).reshape(m9.n, m9.n, n)
    worst_f = worst_J = 0.0
    for c in range(0, n, 7):
        fo = m9.rhs(rho[c], y[:, c])
        Jo = m9.jac(rho[c], y[:, c])
        # scale: the gross (unsigned) production of each row
        kf, kr, qf, qr = m9.rates(y[-1, c], rho[c] * y[:-1, c] / m9.W)
        gross = np.sum(np.abs(qf) + np.abs(qr)) * max(m9.W) * 3 / rho[c]
        worst_f = max(worst_f, np.max(np.abs(fg[:-1, c] - fo[:-1])) / gross)
        worst_f = max(worst_f, abs(fg[-1, c] - fo[-1]) / (abs(fo[-1]) + gross * 1e4))
        for i in range(m9.n):
            sc = np.max(np.abs(Jo[i] * np.maximum(np.abs(y[:, c]), 1e-8)))
            err = np.abs(Jg[i, :, c] - Jo[i]) * np.maximum(np.abs(y[:, c]), 1e-8)
            worst_J = max(worst_J, np.max(err) / (sc + 1e-300))
    assert worst_f < 1e-12, worst_f
    assert worst_J < 1e-11, worst_J


@pytest.fixture(scope="module")
def c1_reference(m9):
    """C1 cells (4096 + a ragged 37) and the tight-tolerance oracle solution."""
    c = fields.c1_cells(4096 + 37, seed=1001)
    rho, e = oracle_inputs(m9, c)
    Yr, Tr, st = m9.integrate(rho, e, c.Y, c.dt, JUDGE_RTOL, JUDGE_ATOL, T=c.T)
    assert np.all(st == 0)
    return c, rho, e, Yr, Tr


@pytest.mark.parametrize("group", SCHEDULES)
@pytest.mark.parametrize("algorithm", [0, 1])
def test_c1_parity_strict(chem, mech, c1_reference, algorithm, group):
    # 1e-6 relative on every species above 1e-10 and 1e-3 K, with atol small
    # enough (1e-20) that the error control is relative on all those species
    c, rho, e, Yr, Tr = c1_reference
    ctx = chem.Context(mech, algorithm=algorithm, group=group)
    Yg, Tg, st, stats = run_gpu(ctx, rho, e, c.Y, c.T, c.dt, RTOL_C1, 1e-20)
    assert stats["rc"] == 0 and np.all(st == 0), np.bincount(st)
    rel, dT, _ = parity_report(Yg, Tg, Yr, Tr)
    print(f"C1 strict algorithm={algorithm} group={group}: max rel species err {rel:.3e}, "
          f"max |dT| {dT:.3e} K, {stats['t_total_ms']:.2f} ms")
    assert dT <= T_ABS
    assert rel <= SPECIES_REL


@pytest.mark.parametrize("algorithm", [0, 1])
def test_c1_parity_at_c1_tolerances(chem, mech, c1_reference, algorithm):
    # at rtol 1e-8 / atol 1e-14 the error of species below atol/rtol = 1e-6 is
    # only controlled in absolute terms; the relative bound is checked where
    # the relative tolerance dominates, temperature everywhere
    c, rho, e, Yr, Tr = c1_reference
    ctx = chem.Context(mech, algorithm=algorithm)
    Yg, Tg, st, stats = run_gpu(ctx, rho, e, c.Y, c.T, c.dt, RTOL_C1, ATOL_C1)
    assert stats["rc"] == 0 and np.all(st == 0), np.bincount(st)
    rel, dT, relmat = parity_report(Yg, Tg, Yr, Tr)
    dom = Yr > ATOL_C1 / RTOL_C1
    rel_dom = float(np.where(dom, relmat, 0.0).max())
    print(f"C1 algorithm={algorithm}: max rel err (Y>1e-6) {rel_dom:.3e}, (Y>1e-10) {rel:.3e}, "
          f"max |dT| {dT:.3e} K, stats {stats}")
    assert dT <= T_ABS
    assert rel_dom <= SPECIES_REL


@pytest.mark.parametrize("group", SCHEDULES)
def test_bulk_sparse_bitwise_equals_plain(chem, mech, m9, group):
    # detonation-patch sample: plain all-cells vs bulk-sparse with several
    # switch points; integrated cells must agree bit for bit
    c = fields.c2_field(64, 64, 4, x_scale=1.0)
    rho, e = oracle_inputs(m9, c)
    ref = None
    for opts in ({"algorithm": 0}, {"algorithm": 1, "nactive_star": 0, "kmax_bulk": 3},
                 {"algorithm": 1, "nactive_star": 500, "kmax_bulk": 5},
                 {"algorithm": 1, "nactive_star": 0, "kmax_bulk": 2, "round_decay": 0.5},
                 {"algorithm": 1, "max_rounds": 0},
                 # lanes take the cells in predicted-cost order (longest first)
                 {"algorithm": 1, "max_rounds": 0, "order": 1},
                 {"algorithm": 1, "nactive_star": 0, "kmax_bulk": 3, "order": 1},
                 # later rounds and the sparse phase in predicted-remaining order, and
                 # step limits set from the completion predictions
                 {"algorithm": 1, "nactive_star": 500, "kmax_bulk": 3, "order": 1},
                 {"algorithm": 1, "nactive_star": 0, "kmax_bulk": 2, "kmax_adapt": 0.5},
                 {"algorithm": 1, "nactive_star": 300, "kmax_bulk": 4, "order": 1, "kmax_adapt": 0.75},
                 # no round runs (N* above the active count): every cell comes from the ordered sparse list
                 {"algorithm": 1, "nactive_star": 1e9, "order": 1},
                 # more rounds than the ordered ones: later rounds run over the active list
                 {"algorithm": 1, "nactive_star": 0, "kmax_bulk": 1, "order": 1}):
        ctx = chem.Context(mech, t_react_min=0.0, group=group, **opts)
        Yg, Tg, st, stats = run_gpu(ctx, rho, e, c.Y, c.T, c.dt, RTOL_C1, ATOL_C1)
        assert np.all(st == 0)
        if ref is None:
            ref = (Yg, Tg)
        else:
            assert np.array_equal(Yg, ref[0]) and np.array_equal(Tg, ref[1]), opts


def test_skipped_cold_cells_change_little(chem, mech, m9):
    c = fields.c2_field(64, 32, 2)
    rho, e = oracle_inputs(m9, c)
    ctx = chem.Context(mech, algorithm=1, t_react_min=500.0)
    Yg, Tg, st, stats = run_gpu(ctx, rho, e, c.Y, c.T, c.dt, RTOL_C1, ATOL_C1)
    cold = c.cls == 0
    assert np.all(st[cold] == 1) and np.all(st[~cold] == 0)
    assert np.array_equal(Yg[:, cold], c.Y[:, cold])
    # what the oracle does to the skipped cells over dt is below the parity tolerance
    idx = np.where(cold)[0][:64]
    Yr, Tr, sto = m9.integrate(rho[idx], e[idx], c.Y[:, idx], c.dt, JUDGE_RTOL, JUDGE_ATOL, T=c.T[idx])
    rel, dT, _ = parity_report(c.Y[:, idx], Tg[idx], Yr, Tr)
    assert rel <= SPECIES_REL and dT <= T_ABS


def test_edge_cases(chem, mech, m9):
    import torch
    ctx = chem.Context(mech)
    # empty call
    z = torch.zeros(0, dtype=torch.float64, device="cuda")
    st = ctx.integrate(z, z, torch.zeros((9, 0), dtype=torch.float64, device="cuda"), z, 1e-7, 1e-8, 1e-14)
    assert st["rc"] == 0 and st["ncell"] == 0
    # invalid states and masked cells
    c = fields.c1_cells(70, seed=3)
    rho, e = oracle_inputs(m9, c)
    rho[5] = -1.0
    e[6] = np.nan
    mask = np.zeros(70, dtype=np.uint8)
    mask[10:20] = 1
    Yg, Tg, st, stats = run_gpu(ctx, rho, e, c.Y, c.T, c.dt, RTOL_C1, ATOL_C1, mask=mask)
    assert st[5] == chem.ST_TINV and st[6] == chem.ST_TINV
    assert np.all(st[10:20] == chem.ST_SKIPPED)
    assert np.array_equal(Yg[:, 10:20], c.Y[:, 10:20])
    # step limit reached -> incomplete, last accepted state kept
    ctx2 = chem.Context(mech, kmax_sparse=2, max_rounds=0)
    Yg, Tg, st, stats = run_gpu(ctx2, rho, e, c.Y, c.T, c.dt, RTOL_C1, ATOL_C1)
    assert stats["rc"] == chem.CHEM_W_INCOMPLETE
    assert np.all(st[20:] == chem.ST_KMAX)


@pytest.mark.parametrize("group", SCHEDULES)
def test_repeat_runs_bitwise_identical(chem, mech, m9, group):
    c = fields.c1_cells(2000, seed=9)
    rho, e = oracle_inputs(m9, c)
    ctx = chem.Context(mech, group=group)
    a = run_gpu(ctx, rho, e, c.Y, c.T, c.dt, RTOL_C1, ATOL_C1)
    b = run_gpu(ctx, rho, e, c.Y, c.T, c.dt, RTOL_C1, ATOL_C1)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_round_decay_gate_stops_rounds_early(chem, mech, m9):
    # with N* = 0 and 2 steps per round the rounds run until the limit; the
    # decay gate stops them once a round retires under half of its cells
    c = fields.c2_field(64, 64, 4, x_scale=1.0)
    rho, e = oracle_inputs(m9, c)
    out = []
    for decay in (0.0, 0.5):
        ctx = chem.Context(mech, t_react_min=0.0, group=0, nactive_star=0, kmax_bulk=2, max_rounds=24,
                           round_decay=decay)
        Yg, Tg, st, stats = run_gpu(ctx, rho, e, c.Y, c.T, c.dt, RTOL_C1, ATOL_C1)
        assert np.all(st == 0)
        out.append((stats["n_bulk_rounds"], Yg, Tg))
    print(f"bulk rounds: {out[0][0]} without the decay gate, {out[1][0]} with it")
    assert out[1][0] < out[0][0]
    assert np.array_equal(out[0][1], out[1][1]) and np.array_equal(out[0][2], out[1][2])


def test_cells_per_wave_selects_the_schedule(chem, mech, m9):
    # cells_per_wave is group counted per 64-lane wave: setting one reads back
    # as the other, and the integration equals the same group's bit for bit
    ctx = chem.Context(mech)
    for cpw, grp in ((64, 0), (16, 4), (8, 8), (4, 16), (2, 32), (1, 64), (0, -1)):
        ctx.set_option("cells_per_wave", cpw)
        assert ctx.get_option("group") == grp and ctx.get_option("cells_per_wave") == cpw
    for bad in (3, 32, 65, -1):
        with pytest.raises(chem.ChemError):
            ctx.set_option("cells_per_wave", bad)
    c = fields.c1_cells(200, seed=1007)
    rho, e = oracle_inputs(m9, c)
    outs = []
    for key, val in (("cells_per_wave", 8), ("group", 8), ("cells_per_wave", 64), ("group", 0)):
        cx = chem.Context(mech)
        cx.set_option(key, val)
        outs.append(run_gpu(cx, rho, e, c.Y, c.T, c.dt, RTOL_C1, ATOL_C1))
    for a, b in ((0, 1), (2, 3)):
        assert np.array_equal(outs[a][0], outs[b][0]) and np.array_equal(outs[a][1], outs[b][1])
