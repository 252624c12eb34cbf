"""The allocation-free entry point (chem_integrate_noalloc) against
chem_integrate with the same schedule: the cooperative kernels without bulk
rounds.  Two calls in a row, the second smaller, so stale scratch contents of
the first call would show in the second; a regular call in between, and a
call past the scratch's size limit."""
import numpy as np
import pytest

from tests.gpu_util import RTOL_C1, ATOL_C1, to_dev, host

pytestmark = pytest.mark.gpu


def _state(orc, n, seed):
    from synth import fields
    c = fields.c1_cells(n, seed=seed)
    rho, e = orc.state_from_TPY(c.T, c.p, c.Y)
    return c, rho, e


def _run(ctx, rho, e, Y, T, dt, noalloc):
    import torch
    n = rho.size
    d_rho, d_e, d_Y, d_T = to_dev(rho), to_dev(e), to_dev(Y), to_dev(T)
    d_st = torch.full((n,), 255, dtype=torch.uint8, device="cuda")
    if noalloc:
        rc = ctx.integrate_noalloc(d_rho, d_e, d_Y, d_T, dt, RTOL_C1, ATOL_C1, status=d_st)
        torch.cuda.synchronize()
    else:
        rc = ctx.integrate(d_rho, d_e, d_Y, d_T, dt, RTOL_C1, ATOL_C1, status=d_st)["rc"]
    return rc, host(d_Y), host(d_T), host(d_st)


def test_noalloc_matches_integrate(m9, m9_path):
    import paper_2510_23993_amd as chem
    mech = chem.Mechanism(m9_path)
    ref = chem.Context(mech, group=16, max_rounds=0)
    na = chem.Context(mech, group=16, max_rounds=0)
    for n, seed in ((6000, 11), (1237, 12)):
        c, rho, e = _state(m9, n, seed)
        print(f"noalloc case: {n} cells, seed {seed}", flush=True)
        rc0, Y0, T0, s0 = _run(ref, rho, e, c.Y, c.T, c.dt, noalloc=False)
        rc1, Y1, T1, s1 = _run(na, rho, e, c.Y, c.T, c.dt, noalloc=True)
        assert rc0 == 0 and rc1 == 0
        assert (s0 == 0).all(), np.bincount(s0)
        np.testing.assert_array_equal(s1, s0)
        np.testing.assert_array_equal(Y1, Y0)
        np.testing.assert_array_equal(T1, T0)


def test_noalloc_default_group_and_limits(m9, m9_path):
    import torch
    import paper_2510_23993_amd as chem
    mech = chem.Mechanism(m9_path)
    # default options: the entry point takes 16 lanes per cell for 10 components
    ref = chem.Context(mech, group=16, max_rounds=0)
    na = chem.Context(mech)
    c, rho, e = _state(m9, 777, 13)
    _, Y0, T0, s0 = _run(ref, rho, e, c.Y, c.T, c.dt, noalloc=False)
    _, Y1, T1, s1 = _run(na, rho, e, c.Y, c.T, c.dt, noalloc=True)
    np.testing.assert_array_equal(s1, s0)
    np.testing.assert_array_equal(Y1, Y0)
    np.testing.assert_array_equal(T1, T0)
    # past the scratch's limit: a clear error, nothing enqueued
    n = (1 << 20) + 1
    z = torch.zeros(n, dtype=torch.float64, device="cuda")
    Yz = torch.zeros((mech.ns, n), dtype=torch.float64, device="cuda")
    with pytest.raises(chem.ChemError, match="1048576") as ei:
        na.integrate_noalloc(z, z, Yz, z.clone(), 1e-7, 1e-8, 1e-14)
    assert ei.value.rc == -1
