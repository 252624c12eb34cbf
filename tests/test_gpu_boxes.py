"""AMR box batching through chem_integrate_boxes and chem_autotune: one
pipeline over many separately allocated boxes with their own dt must give
each cell exactly what a call on its box alone gives (the fusion is an
exact reorganisation), graph replays must match the eager run on every
replay, and a sample must match the oracle."""
import numpy as np
import pytest

from synth import fields
from tests.gpu_util import (JUDGE_ATOL, JUDGE_RTOL, RTOL_C1, SPECIES_REL, T_ABS, host,
                            parity_report, to_dev)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def chem():
    import paper_2510_23993_amd as chem
    return chem


@pytest.fixture(scope="module")
def mech(chem, m9_path):
    return chem.Mechanism(m9_path)


@pytest.fixture(scope="module")
def small_boxes(m9):
    """Nine boxes of the three-level jet-in-crossflow hierarchy (8^3 to
    16x16x32 cells, all three dt) plus one empty box; host arrays."""
    boxes = fields.c3_boxes()
    pick = []
    for lev in range(3):
        cand = [i for i, b in enumerate(boxes) if b.level == lev and np.prod(b.shape) <= 8192]
        pick += cand[:3]
    out = []
    for i in pick:
        c = fields.c3_box_state(boxes[i], box_id=i)
        rho, e = m9.state_from_TPY(c.T, c.p, c.Y)
        out.append(dict(rho=rho, e=e, Y=c.Y, T=c.T, dt=c.dt, level=boxes[i].level))
    out.insert(4, dict(rho=np.zeros(0), e=np.zeros(0), Y=np.zeros((9, 0)), T=np.zeros(0),
                       dt=2e-8, level=1))
    return out


def _dev_boxes(hb):
    import torch
    d = []
    for b in hb:
        n = b["rho"].size
        d.append(dict(rho=to_dev(b["rho"]), e=to_dev(b["e"]), Y=to_dev(b["Y"]), T=to_dev(b["T"]),
                      status=torch.full((n,), 255, dtype=torch.uint8, device="cuda"),
                      dt=b["dt"], level=b["level"]))
    return d


def _reset(d, hb):
    for x, b in zip(d, hb):
        x["Y"].copy_(to_dev(b["Y"]))
        x["T"].copy_(to_dev(b["T"]))
        x["status"].fill_(255)


@pytest.mark.parametrize("group", [0, 16])
def test_boxes_bitwise_equal_per_box_calls(chem, mech, small_boxes, group):
    ctx = chem.Context(mech, group=group, use_graph=0)
    d = _dev_boxes(small_boxes)
    st = ctx.integrate_boxes(d, RTOL_C1, 1e-20)
    assert st["rc"] == 0
    assert st["ncell"] == sum(b["rho"].size for b in small_boxes)
    for b, x in zip(small_boxes, d):
        if b["rho"].size == 0:
            continue
        s = host(x["status"])
        assert np.all((s == chem.ST_DONE) | (s == chem.ST_SKIPPED))
        ref = _dev_boxes([b])[0]
        ctx.integrate(ref["rho"], ref["e"], ref["Y"], ref["T"], b["dt"], RTOL_C1, 1e-20,
                      status=ref["status"])
        assert np.array_equal(host(ref["Y"]), host(x["Y"]))
        assert np.array_equal(host(ref["T"]), host(x["T"]))
        assert np.array_equal(host(ref["status"]), s)


def test_boxes_graph_replays_match_eager(chem, mech, small_boxes):
    import torch
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        eager = chem.Context(mech, use_graph=0, stream=stream)
        d = _dev_boxes(small_boxes)
        eager.integrate_boxes(d, RTOL_C1, 1e-20)
        ref = [(host(x["Y"]), host(x["T"]), host(x["status"])) for x in d]
        g = chem.Context(mech, use_graph=1, stream=stream)
        for rep in range(4):
            _reset(d, small_boxes)
            torch.cuda.synchronize()
            g.integrate_boxes(d, RTOL_C1, 1e-20, stats=False)
            torch.cuda.synchronize()
            for (Yr, Tr, sr), x in zip(ref, d):
                assert np.array_equal(host(x["Y"]), Yr), rep
                assert np.array_equal(host(x["T"]), Tr), rep
                assert np.array_equal(host(x["status"]), sr), rep
            if rep == 1:
                # a single-box call in between re-stages the box table
                one = _dev_boxes([small_boxes[0]])[0]
                g.integrate(one["rho"], one["e"], one["Y"], one["T"], small_boxes[0]["dt"],
                            RTOL_C1, 1e-20)
            # eager work between replays
            torch.cuda.synchronize()
            _ = (d[0]["Y"] * 2.0).sum().item()


def test_boxes_sample_vs_oracle(chem, mech, m9, small_boxes):
    ctx = chem.Context(mech, use_graph=0)
    d = _dev_boxes(small_boxes)
    ctx.integrate_boxes(d, RTOL_C1, 1e-20)
    rng = np.random.default_rng(5)
    worst_rel = worst_dT = 0.0
    compared = 0
    for b, x in zip(small_boxes, d):
        n = b["rho"].size
        if n == 0:
            continue
        idx = np.sort(rng.choice(n, size=min(n, 24), replace=False))
        Yr, Tr, st = m9.integrate(b["rho"][idx], b["e"][idx], b["Y"][:, idx], b["dt"], JUDGE_RTOL,
                                  JUDGE_ATOL, T=b["T"][idx])
        s = host(x["status"])[idx]
        assert np.all((s == chem.ST_DONE) | (s == chem.ST_SKIPPED))
        done = s == chem.ST_DONE
        if not done.any():
            continue
        compared += int(done.sum())
        rel, dT, _ = parity_report(host(x["Y"])[:, idx][:, done], host(x["T"])[idx][done],
                                   Yr[:, done], Tr[done])
        worst_rel, worst_dT = max(worst_rel, rel), max(worst_dT, dT)
    print(f"boxes vs oracle ({compared} cells): max rel {worst_rel:.3e}, max |dT| {worst_dT:.3e} K")
    assert compared >= 50
    assert worst_rel <= SPECIES_REL and worst_dT <= T_ABS


def test_autotune_restores_state_and_caches(chem, mech, small_boxes, tmp_path):
    ctx = chem.Context(mech, use_graph=0)
    d = _dev_boxes(small_boxes)
    cache = str(tmp_path / "tune.json")
    opts, ms = ctx.autotune(d, RTOL_C1, 1e-20, cache_path=cache)
    assert ms > 0
    for b, x in zip(small_boxes, d):
        assert np.array_equal(host(x["Y"]), b["Y"]) and np.array_equal(host(x["T"]), b["T"])
    assert opts["group"] in (0, 4, 8, 16, 32, 64)
    lines = open(cache).read().strip().splitlines()
    assert len(lines) == 1 and '"group"' in lines[0]
    # a second context on the same boxes takes the cached choice
    ctx2 = chem.Context(mech, use_graph=0)
    opts2, ms2 = ctx2.autotune(d, RTOL_C1, 1e-20, cache_path=cache)
    assert opts2 == opts and ms2 == pytest.approx(ms, rel=1e-5)
    assert len(open(cache).read().strip().splitlines()) == 1
    st = ctx2.integrate_boxes(d, RTOL_C1, 1e-20)
    assert st["rc"] == 0


def test_full_hierarchy_sample_vs_oracle(chem, mech, m9):
    """All 400 boxes of the three-level hierarchy (5,750,784 cells) in one
    graph-replayed pipeline with the options the autotuner picks for it (one
    lane per cell, no bulk rounds), at the benchmark's tolerances (rtol 1e-8,
    atol 1e-14).  300 sampled integrated cells against the oracle at tight
    tolerance: relative bound where the relative tolerance dominates
    (Y > atol/rtol), temperature everywhere."""
    import torch
    atol = 1e-14
    boxes = fields.c3_boxes()
    hb, d = [], []
    for i, b in enumerate(boxes):
        c = fields.c3_box_state(b, box_id=i)
        rho, e = m9.state_from_TPY(c.T, c.p, c.Y)
        hb.append(dict(rho=rho, e=e, Y=c.Y, T=c.T, dt=c.dt))
        n = c.T.size
        d.append(dict(rho=to_dev(rho), e=to_dev(e), Y=to_dev(c.Y), T=to_dev(c.T),
                      status=torch.full((n,), 255, dtype=torch.uint8, device="cuda"), dt=c.dt, level=b.level))
    assert sum(b["rho"].size for b in hb) == 5750784
    ctx = chem.Context(mech, use_graph=1, group=0, max_rounds=0, nactive_star=1e4, kmax_bulk=5)
    st = ctx.integrate_boxes(d, RTOL_C1, atol)
    assert st["rc"] == 0
    rng = np.random.default_rng(11)
    picks = {}
    for _ in range(300):
        while True:
            bi = int(rng.integers(len(hb)))
            s = host(d[bi]["status"])
            ok = np.where(s == chem.ST_DONE)[0]
            if ok.size:
                picks.setdefault(bi, set()).add(int(rng.choice(ok)))
                break
    worst_rel = worst_dT = 0.0
    compared = 0
    for bi, cells in picks.items():
        idx = np.array(sorted(cells))
        b = hb[bi]
        Yr, Tr, so = m9.integrate(b["rho"][idx], b["e"][idx], b["Y"][:, idx], b["dt"], JUDGE_RTOL, JUDGE_ATOL,
                                  T=b["T"][idx])
        assert np.all(so == 0)
        Yg, Tg = host(d[bi]["Y"])[:, idx], host(d[bi]["T"])[idx]
        _, dT, relmat = parity_report(Yg, Tg, Yr, Tr)
        dom = Yr > atol / RTOL_C1
        worst_rel = max(worst_rel, float(np.where(dom, relmat, 0.0).max()))
        worst_dT = max(worst_dT, dT)
        compared += idx.size
    print(f"full hierarchy vs oracle ({compared} cells in {len(picks)} boxes, {st['t_total_ms']:.1f} ms): "
          f"max rel (Y > 1e-6) {worst_rel:.3e}, max |dT| {worst_dT:.3e} K")
    assert compared >= 250
    assert worst_rel <= SPECIES_REL and worst_dT <= T_ABS
