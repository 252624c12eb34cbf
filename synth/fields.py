"""Seeded synthetic reactor fields with the shapes of the paper's workloads.

Each generator returns primitive states (T [K], p [Pa], Y [ns][ncell]
column-major mass fractions).  Conversion to the reactor inputs (rho, e)
is done by the caller with its own thermo (the oracle in tests, the
product's state-preparation kernel in the benchmark), so this module holds
no thermochemistry: the "equilibrium" end of each composition blend is
read from a stored table of equilibrium mass fractions (written by
``synth/data/make_eq_tables.py`` with the oracle's Gibbs minimiser) and
interpolated linearly.
"""
from __future__ import annotations

import os
from dataclasses import dataclass
from typing import Dict, List, Optional

import numpy as np

from .mechgen import M9_SPECIES

ATM = 101325.0
DATA = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data")
M9_PATH = os.path.join(DATA, "m9.mech")
M53_PATH = os.path.join(DATA, "m53.mech")
M9_TWO_RANGE_PATH = os.path.join(DATA, "m9_two_range.mech")   # distinct NASA-7 sets below / above 1000 K

# molecular weights of the M9 species [g/mol] from the standard atomic masses
_W9 = np.array([2.016, 31.998, 18.015, 1.008, 15.999, 17.007, 33.006, 34.014, 28.014])
_I = {s: i for i, s in enumerate(M9_SPECIES)}
Z_ST = 2 * 2.016 / (2 * 2.016 + 31.998 + 3.76 * 28.014)  # stoichiometric mixture fraction


def unburnt_Y(Z: np.ndarray) -> np.ndarray:
    """Unburnt H2 / air mass fractions for mixture fraction Z (fuel stream =
    pure H2, oxidiser = O2 + 3.76 N2 by moles).  Returns [9][n]."""
    Z = np.atleast_1d(np.asarray(Z, dtype=np.float64))
    air_O2 = 31.998 / (31.998 + 3.76 * 28.014)
    Y = np.zeros((9, Z.size))
    Y[_I["H2"]] = Z
    Y[_I["O2"]] = (1 - Z) * air_O2
    Y[_I["N2"]] = (1 - Z) * (1 - air_O2)
    return Y


def Z_from_phi(phi):
    phi = np.asarray(phi, dtype=np.float64)
    r = phi * Z_ST / (1 - Z_ST)
    return r / (1 + r)


class EqTable:
    """Trilinear interpolation of stored equilibrium mass fractions on a
    (Z, T, ln p) grid (or (T, ln p) for a fixed base composition)."""

    def __init__(self, path: str):
        with np.load(path, allow_pickle=False) as d:
            self.axes = [np.asarray(d[k]) for k in ("Z", "T", "lnp") if k in d.files]
            self.names = [k for k in ("Z", "T", "lnp") if k in d.files]
            self.Y = np.asarray(d["Y"])      # [..grid.., ns]

    def __call__(self, **q) -> np.ndarray:
        coords = [np.asarray(q[n], dtype=np.float64) for n in self.names]
        n = np.broadcast(*coords).size
        coords = [np.broadcast_to(c, (n,)) for c in coords]
        idx, wts = [], []
        for ax, c in zip(self.axes, coords):
            c = np.clip(c, ax[0], ax[-1])
            i = np.clip(np.searchsorted(ax, c, side="right") - 1, 0, len(ax) - 2)
            w = (c - ax[i]) / (ax[i + 1] - ax[i])
            idx.append(i)
            wts.append(w)
        out = np.zeros((n, self.Y.shape[-1]))
        d = len(self.axes)
        for corner in range(1 << d):
            sel = []
            w = np.ones(n)
            for a in range(d):
                bit = (corner >> a) & 1
                sel.append(idx[a] + bit)
                w = w * (wts[a] if bit else 1 - wts[a])
            out += w[:, None] * self.Y[tuple(sel)]
        return out.T  # [ns][n]


_tables: Dict[str, EqTable] = {}


def eq_table(name: str) -> EqTable:
    if name not in _tables:
        _tables[name] = EqTable(os.path.join(DATA, name))
    return _tables[name]


@dataclass
class Cells:
    T: np.ndarray          # [n] K
    p: np.ndarray          # [n] Pa
    Y: np.ndarray          # [ns][n]
    dt: np.ndarray | float
    cls: Optional[np.ndarray] = None   # per-cell class label (0 cold, 1 induction, 2 burnt ...)
    extra: Optional[dict] = None


def _renorm(Y):
    Y = np.maximum(Y, 0.0)
    return Y / Y.sum(axis=0, keepdims=True)


def c1_cells(n: int = 4096, seed: int = 1001) -> Cells:
    """Independent reactors: T0 ~ U(1000, 2500) K, p0 ~ U(1, 20) atm,
    phi ~ U(0.5, 2), progress lambda ~ U(0, 1) blending the unburnt mix with
    its TP equilibrium at (T0, p0).  dt = 1e-7 s."""
    rng = np.random.default_rng(seed)
    T = rng.uniform(1000.0, 2500.0, n)
    p = rng.uniform(1.0, 20.0, n) * ATM
    phi = rng.uniform(0.5, 2.0, n)
    lam = rng.uniform(0.0, 1.0, n)
    Z = Z_from_phi(phi)
    Yu = unburnt_Y(Z)
    Ye = eq_table("m9_eq_ZTp.npz")(Z=Z, T=T, lnp=np.log(p))
    Y = _renorm((1 - lam) * Yu + lam * Ye)
    return Cells(T=T, p=p, Y=np.ascontiguousarray(Y), dt=1e-7, extra={"phi": phi, "lam": lam})


def c2_field(nx: int = 256, ny: int = 256, nz: int = 32, seed: int = 1002,
             x_scale: float = 1.0) -> Cells:
    """Planar detonation patch, x fastest (id = x + nx (y + ny z)).  Cold
    premixed stoichiometric H2-air at 300 K, 1 atm ahead of a wrinkled front;
    a shocked induction band (T 1500-3000 K, p 20-40 atm, +/-5% noise, small
    progress); burnt gas near equilibrium behind.  dt = 5e-9 s.
    ``x_scale`` < 1 keeps the class fractions on a narrower patch."""
    rng = np.random.default_rng(seed)
    ph1, ph2 = rng.uniform(0, 2 * np.pi, 2)
    x = np.arange(nx, dtype=np.float64)[None, None, :]
    y = np.arange(ny, dtype=np.float64)[None, :, None]
    z = np.arange(nz, dtype=np.float64)[:, None, None]
    L = nx * x_scale
    xs = (0.15 * L + 3 * x_scale * np.sin(2 * np.pi * y / 64 + ph1)
          + 2 * x_scale * np.sin(2 * np.pi * z / 32 + ph2)
          + rng.uniform(-1, 1, (nz, ny, 1)) * x_scale)
    band = 0.05 * L
    shape = (nz, ny, nx)
    xx = np.broadcast_to(x, shape)
    xsb = np.broadcast_to(xs, shape)
    cold = xx >= xsb
    ind = (~cold) & (xx >= xsb - band)
    burnt = ~(cold | ind)
    N = nx * ny * nz
    T = np.empty(shape)
    p = np.empty(shape)
    lam = np.zeros(shape)
    T[cold] = 300.0
    p[cold] = ATM
    s = np.where(ind, (xsb - xx) / band, 0.0)
    ni = int(ind.sum())
    T[ind] = (1500.0 + 1500.0 * s[ind]) * (1 + rng.uniform(-0.05, 0.05, ni))
    p[ind] = (40.0 - 20.0 * s[ind]) * ATM * (1 + rng.uniform(-0.05, 0.05, ni))
    lam[ind] = 0.5 * s[ind] ** 3
    nb = int(burnt.sum())
    T[burnt] = 2900.0 * (1 + rng.uniform(-0.02, 0.02, nb))
    p[burnt] = 18.0 * ATM * (1 + rng.uniform(-0.02, 0.02, nb))
    lam[burnt] = rng.uniform(0.98, 1.0, nb)
    T = T.reshape(N)
    p = p.reshape(N)
    lam = lam.reshape(N)
    cls = np.zeros(N, dtype=np.int8)
    cls[ind.reshape(N)] = 1
    cls[burnt.reshape(N)] = 2
    Yu = unburnt_Y(np.full(N, Z_ST))
    Y = Yu.copy()
    hot = cls > 0
    Ye = eq_table("m9_eq_ZTp.npz")(Z=np.full(int(hot.sum()), Z_ST), T=T[hot], lnp=np.log(p[hot]))
    Y[:, hot] = _renorm((1 - lam[hot]) * Yu[:, hot] + lam[hot] * Ye)
    return Cells(T=T, p=p, Y=np.ascontiguousarray(Y), dt=5e-9, cls=cls)


@dataclass
class Box:
    level: int
    shape: tuple          # (nz, ny, nx)
    origin: tuple         # (z0, y0, x0) in level index space
    dt: float


def c3_boxes(seed: int = 1003, nbox=(100, 140, 160), total=(5.7e6, 6.3e6)) -> List[Box]:
    """400 AMR boxes over three levels (refinement ratio 2): per-axis box
    sizes from {8, 16, 32, 64} with p = {0.25, 0.35, 0.28, 0.12} (mean total
    about 5.7M cells), redrawn until the total lands in [5.7M, 6.3M].
    dt by level 4e-8/2e-8/1e-8 s."""
    rng = np.random.default_rng(seed)
    sizes = np.array([8, 16, 32, 64])
    probs = np.array([0.25, 0.35, 0.28, 0.12])
    dts = [4e-8, 2e-8, 1e-8]
    for _ in range(100000):
        boxes = []
        for lev, nb in enumerate(nbox):
            dom = np.array([64, 128, 256]) * (2 ** lev)   # (z, y, x) domain at this level
            for _ in range(nb):
                shp = tuple(int(s) for s in rng.choice(sizes, 3, p=probs))
                org = tuple(int(rng.integers(0, max(1, d - s + 1))) for d, s in zip(dom, shp))
                boxes.append(Box(level=lev, shape=shp, origin=org, dt=dts[lev]))
        tot = sum(int(np.prod(b.shape)) for b in boxes)
        if total[0] <= tot <= total[1]:
            return boxes
    raise RuntimeError("c3_boxes: no draw landed in the requested total")


def c3_box_state(box: Box, seed: int = 1003, box_id: int = 0) -> Cells:
    """Jet-in-crossflow-like state inside one box: Gaussian H2 plume (mixture
    fraction Z in [0, 1]) bending into air at 1200 K; mixing-line temperature
    from the two stream temperatures; flame progress peaked around Z_st;
    p = 1 + 2 U atm, smooth in space.  Coordinates are in coarse-level units."""
    rng = np.random.default_rng(seed * 1000 + box_id)
    r = 2.0 ** box.level
    nz, ny, nx = box.shape
    z0, y0, x0 = box.origin
    zz = (z0 + np.arange(nz) + 0.5)[:, None, None] / r
    yy = (y0 + np.arange(ny) + 0.5)[None, :, None] / r
    xx = (x0 + np.arange(nx) + 0.5)[None, None, :] / r
    yc = 20.0 + 12.0 * np.cbrt(np.maximum(xx, 0.0))
    sig = 6.0 + 0.05 * xx
    Z = np.exp(-((yy - yc) ** 2 + (zz - 32.0) ** 2) / (2 * sig ** 2))
    Z = np.broadcast_to(Z, box.shape).reshape(-1)
    N = Z.size
    # mixing line between H2 at 300 K and air at 1200 K (cp-weighted, H2 ~ 14.3 kJ/kg/K, air ~ 1.1)
    cf, co = 14.3, 1.1
    Tmix = (Z * cf * 300.0 + (1 - Z) * co * 1200.0) / (Z * cf + (1 - Z) * co)
    prog = rng.uniform(0.5, 1.0, N) * np.exp(-((Z - Z_ST) / 0.02) ** 2)
    T = Tmix + prog * (2800.0 - Tmix)
    pb = 1.0 + 2.0 * rng.uniform()
    p = (pb + 0.1 * np.sin(np.broadcast_to(xx, box.shape).reshape(-1) / 16.0)) * ATM
    Yu = unburnt_Y(Z)
    Ye = eq_table("m9_eq_ZTp.npz")(Z=Z, T=T, lnp=np.log(p))
    Y = _renorm((1 - prog) * Yu + prog * Ye)
    return Cells(T=T, p=p, Y=np.ascontiguousarray(Y), dt=box.dt)


def c4_cells(n: int = 4_194_304, seed: int = 1004, ns: int = 53) -> Cells:
    """Cells for the 53-species mechanism: T ~ U(800, 2600) K, p ~ U(1, 30)
    atm; composition = seeded fuel/O2/N2 base blended toward its TP
    equilibrium by lambda ~ U(0, 1), plus log-uniform traces 1e-12..1e-4 on
    every species, renormalised.  dt = 1e-7 s (C4 states none; C1's is used)."""
    rng = np.random.default_rng(seed)
    T = rng.uniform(800.0, 2600.0, n)
    p = rng.uniform(1.0, 30.0, n) * ATM
    lam = rng.uniform(0.0, 1.0, n)
    tab = eq_table("m53_eq_Tp.npz")
    base = tab.extra_base if hasattr(tab, "extra_base") else None
    with np.load(os.path.join(DATA, "m53_eq_Tp.npz"), allow_pickle=False) as d:
        base = np.asarray(d["base"])
    Ye = tab(T=T, lnp=np.log(p))
    Y = (1 - lam) * base[:, None] + lam * Ye
    Y = Y + 10.0 ** rng.uniform(-12.0, -4.0, (ns, n))
    Y = Y / Y.sum(axis=0, keepdims=True)
    return Cells(T=T, p=p, Y=np.ascontiguousarray(Y), dt=1e-7)


def m53_base_Y(species: List[str], W: np.ndarray) -> np.ndarray:
    """Fuel/O2/N2 base of the 53-species cells: CH4 + H2 fuel at phi = 1 in air
    (moles CH4:H2:O2:N2 = 0.5:1:1.5:5.64)."""
    X = np.zeros(len(species))
    for s, v in (("CH4", 0.5), ("H2", 1.0), ("O2", 1.5), ("N2", 5.64)):
        X[species.index(s)] = v
    w = X * W
    return w / w.sum()


def c5_training_states(n: int, seed: int = 1005) -> Cells:
    """Initial states for the surrogate's training pairs, drawn from the
    distributions of the other workloads and somewhat wider: 40% burnt gas
    near equilibrium (T 2900 K +-4%, p 18 atm +-4%, progress 0.95-1), 35%
    shocked induction gas (T 1500-3000 K and p 40-20 atm along the band,
    +-6% noise, progress 0.5 s^3), 25% independent reactors as in c1_cells.
    Per-cell dt: 5e-9 s x 10^U(-0.3, 0.3) for the first two groups,
    10^U(-9, -7) s for the reactors.  cls: 0 burnt, 1 induction, 2 reactor."""
    rng = np.random.default_rng(seed)
    nb, ni = int(0.40 * n), int(0.35 * n)
    nc = n - nb - ni
    T = np.empty(n)
    p = np.empty(n)
    lam = np.empty(n)
    Z = np.full(n, Z_ST)
    dt = np.empty(n)
    cls = np.zeros(n, dtype=np.int8)
    b = slice(0, nb)
    T[b] = 2900.0 * (1 + rng.uniform(-0.04, 0.04, nb))
    p[b] = 18.0 * ATM * (1 + rng.uniform(-0.04, 0.04, nb))
    lam[b] = rng.uniform(0.95, 1.0, nb)
    i = slice(nb, nb + ni)
    s = rng.uniform(0.0, 1.0, ni)
    T[i] = (1500.0 + 1500.0 * s) * (1 + rng.uniform(-0.06, 0.06, ni))
    p[i] = (40.0 - 20.0 * s) * ATM * (1 + rng.uniform(-0.06, 0.06, ni))
    lam[i] = 0.5 * s ** 3
    cls[i] = 1
    dt[:nb + ni] = 5e-9 * 10.0 ** rng.uniform(-0.3, 0.3, nb + ni)
    c = slice(nb + ni, n)
    T[c] = rng.uniform(1000.0, 2500.0, nc)
    p[c] = rng.uniform(1.0, 20.0, nc) * ATM
    Z[c] = Z_from_phi(rng.uniform(0.5, 2.0, nc))
    lam[c] = rng.uniform(0.0, 1.0, nc)
    dt[c] = 10.0 ** rng.uniform(-9.0, -7.0, nc)
    cls[c] = 2
    Yu = unburnt_Y(Z)
    Ye = eq_table("m9_eq_ZTp.npz")(Z=Z, T=T, lnp=np.log(p))
    Y = _renorm((1 - lam) * Yu + lam * Ye)
    return Cells(T=T, p=p, Y=np.ascontiguousarray(Y), dt=dt, cls=cls)
