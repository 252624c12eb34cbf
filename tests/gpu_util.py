"""Helpers shared by the GPU tests: seeded inputs prepared by the oracle and
copied to the device, and the parity criterion."""
import numpy as np

RTOL_C1, ATOL_C1 = 1e-8, 1e-14          # the plain FP64 path's tolerances (C1)
JUDGE_RTOL, JUDGE_ATOL = 1e-12, 1e-20     # tight oracle run used as reference
SPECIES_REL, SPECIES_FLOOR, T_ABS = 1e-6, 1e-10, 1e-3


def to_dev(a, dtype=None):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype or torch.float64, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def oracle_inputs(orc, cells):
    """(rho, e) for a Cells object, computed by the oracle's thermo."""
    rho, e = orc.state_from_TPY(cells.T, cells.p, cells.Y)
    return rho, e


def run_gpu(ctx, rho, e, Y, T0, dt, rtol, atol, mask=None, status=True):
    import torch
    n = rho.size
    d_rho, d_e = to_dev(rho), to_dev(e)
    d_Y, d_T = to_dev(Y), to_dev(T0)
    d_st = torch.zeros(n, dtype=torch.uint8, device="cuda") if status else None
    d_mask = to_dev(mask, torch.uint8) if mask is not None else None
    stats = ctx.integrate(d_rho, d_e, d_Y, d_T, dt, rtol, atol, mask=d_mask, status=d_st)
    return host(d_Y), host(d_T), (host(d_st) if status else None), stats


def parity_report(Yg, Tg, Yr, Tr):
    """Max relative species error over species with Y_ref > 1e-10 and max |dT|."""
    big = Yr > SPECIES_FLOOR
    rel = np.abs(Yg - Yr) / np.where(big, Yr, 1.0)
    rel = np.where(big, rel, 0.0)
    return float(rel.max()), float(np.abs(Tg - Tr).max()), rel
