"""Writes the stored inputs under synth/data: the synthetic mechanism files
(from the seeded generators) and the equilibrium tables that the field
generators interpolate.  Equilibria come from the oracle's Gibbs
minimiser only.  Run:  python synth/data/make_eq_tables.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from synth.mechfile import write_mechanism  # noqa: E402
from synth.mechgen import make_m9, make_m53  # noqa: E402
from synth.fields import unburnt_Y, m53_base_Y, ATM  # noqa: E402
import oracle  # noqa: E402
from oracle import gibbs  # noqa: E402

Z_GRID = np.array([0.0, 0.002, 0.005, 0.008, 0.011, 0.014, 0.017, 0.020, 0.024, 0.028, 0.032,
                   0.036, 0.040, 0.045, 0.050, 0.055, 0.060, 0.07, 0.08, 0.10, 0.13, 0.17,
                   0.25, 0.40, 0.60, 1.0])
T_GRID = np.arange(300.0, 3201.0, 100.0)
P_GRID = np.array([0.8, 1.5, 3.0, 6.0, 12.0, 20.0, 30.0, 46.0]) * ATM


def m9_table(path_mech):
    o = oracle.Oracle(path_mech)
    Y = np.zeros((len(Z_GRID), len(T_GRID), len(P_GRID), o.ns))
    for a, Z in enumerate(Z_GRID):
        Yu = unburnt_Y(np.array([Z]))[:, 0]
        b = gibbs.element_moles_from_Y(o, Yu)
        for i, T in enumerate(T_GRID):
            for j, p in enumerate(P_GRID):
                X = gibbs.equilibrate_TP(o, T, p, b)
                Y[a, i, j] = gibbs.Y_from_X(o, X)
    return Y


def m53_table(path_mech, T_grid, P_grid):
    o = oracle.Oracle(path_mech)
    base = m53_base_Y(o.species, o.W)
    b = gibbs.element_moles_from_Y(o, base)
    Y = np.zeros((len(T_grid), len(P_grid), o.ns))
    for i, T in enumerate(T_grid):
        for j, p in enumerate(P_grid):
            X = gibbs.equilibrate_TP(o, T, p, b)
            Y[i, j] = gibbs.Y_from_X(o, X)
    return Y, base


def main(which=("m9", "m53")):
    oracle.build(force=False)
    m9p = os.path.join(HERE, "m9.mech")
    m53p = os.path.join(HERE, "m53.mech")
    write_mechanism(make_m9(), m9p)
    write_mechanism(make_m53(), m53p)
    if "m9" in which:
        Y = m9_table(m9p)
        np.savez(os.path.join(HERE, "m9_eq_ZTp.npz"), Z=Z_GRID, T=T_GRID, lnp=np.log(P_GRID), Y=Y)
    if "m53" in which:
        Tg = np.arange(700.0, 2701.0, 100.0)
        Pg = np.array([0.8, 2.0, 4.0, 8.0, 16.0, 32.0]) * ATM
        Y, base = m53_table(m53p, Tg, Pg)
        np.savez(os.path.join(HERE, "m53_eq_Tp.npz"), T=Tg, lnp=np.log(Pg), Y=Y, base=base)


if __name__ == "__main__":
    main(tuple(sys.argv[1:]) or ("m9", "m53"))
