"""Regression tests for launch-configuration faults of the HIP library."""
import numpy as np
import pytest

from synth import fields
from tests.gpu_util import oracle_inputs, parity_report, run_gpu

pytestmark = pytest.mark.gpu


def test_cooperative_lds_limit_follows_the_largest_call(m9_path):
    # The 9-species mechanism at 32 lanes per cell needs little LDS per
    # workgroup, the 53-species one 79,920 B (above the default 64 KB limit).
    # Both run in one process, small first, with bulk rounds (so the BULK and
    # SPARSE kernels of the same schedule are both launched), and both must
    # match the oracle.
    import oracle
    import paper_2510_23993_amd as chem
    for path, n, rtol in ((m9_path, 96, 1e-8), (fields.M53_PATH, 48, 1e-11)):
        orc = oracle.Oracle(path)
        if path == m9_path:
            c = fields.c1_cells(n, seed=321)
        else:
            c = fields.c4_cells(n, seed=322)
        rho, e = oracle_inputs(orc, c)
        Yr, Tr, st = orc.integrate(rho, e, c.Y, c.dt, 1e-12, 1e-20, T=c.T)
        assert np.all(st == 0)
        mech = chem.Mechanism(path)
        ctx = chem.Context(mech, group=32, algorithm=1, max_rounds=4, kmax_bulk=5, nactive_star=0)
        Yg, Tg, sg, stats = run_gpu(ctx, rho, e, c.Y, c.T, c.dt, rtol, 1e-20)
        assert stats["rc"] == 0 and np.all(sg == 0), np.bincount(sg)
        assert stats["n_bulk_rounds"] >= 1
        rel, dT, _ = parity_report(Yg, Tg, Yr, Tr)
        print(f"{mech.ns} species, 32 lanes per cell: max rel {rel:.2e}, max |dT| {dT:.2e} K")
        assert rel <= 1e-6 and dT <= 1e-3
