"""Seeded generators of synthetic kinetic mechanisms.

No published mechanism data are used: thermochemistry comes from a smooth
rigid-rotor / harmonic-oscillator style heat-capacity model with seeded
vibrational temperatures, anchored to seeded round-number formation
enthalpies and entropies; Arrhenius parameters are drawn inside broad
class-wise ranges. Element balance holds by construction.

The functions here produce mechanism *data*; they never evaluate rates,
equilibrium constants or the reactor right-hand side.
"""
from __future__ import annotations

import itertools
import math
from typing import Dict, List, Tuple

import numpy as np
from numpy.polynomial import polynomial as P

from .mechfile import Mechanism, Reaction, Species

R_GAS = 8.314462618  # J/mol/K
T_REF = 298.15

M9_SEED = 1004  # chosen so stoichiometric 1 atm ignition delays fall in 1e-6..1e-3 s over 1000-2500 K
M53_SEED = 1075  # seeded so that C4-style cells integrate without step-size failures in the oracle


def _einstein_cp(T: np.ndarray, thetas) -> np.ndarray:
    out = np.zeros_like(T)
    for th in thetas:
        x = th / T
        em = np.exp(-x)
        out += x * x * em / (1.0 - em) ** 2
    return out


def nasa7_from_cp_model(base: float, thetas, dHf: float, S298: float):
    """Fit one quartic to cp/R over 300-5000 K (used for both NASA ranges,
    so every derivative is continuous at Tmid) and anchor the integration
    constants so that h(298.15 K) = dHf [J/mol] and s(298.15 K) = S298."""
    T = np.linspace(300.0, 5000.0, 240)
    cp = base + _einstein_cp(T, thetas)
    x = T / 1000.0
    c = P.polyfit(x, cp, 4)                    # cp/R in powers of T/1000
    a = [c[i] / 1000.0 ** i for i in range(5)]  # powers of T
    # antiderivatives of the fitted polynomial, evaluated with numpy
    h_poly = P.polyint(a)                       # int cp/R dT (constant 0)
    s_poly = P.polyint(a[1:])                   # int (cp/R - a1)/T dT
    a6 = dHf / R_GAS - P.polyval(T_REF, h_poly)
    a7 = S298 / R_GAS - (a[0] * math.log(T_REF) + P.polyval(T_REF, s_poly))
    return [float(v) for v in a] + [float(a6), float(a7)]


def _species(name, comp, rng, dHf_kJ, S298, theta_lo=600.0, theta_hi=5500.0):
    natom = sum(comp.values())
    if natom == 1:
        base, nmodes = 2.5, 0
    elif natom == 2:
        base, nmodes = 3.5, 1
    else:
        base, nmodes = 4.0, 3 * natom - 6
    lo = theta_lo if natom > 2 else 2000.0
    thetas = sorted(rng.uniform(lo, theta_hi, size=nmodes))
    coeffs = nasa7_from_cp_model(base, thetas, dHf_kJ * 1000.0, S298)
    return Species(name=name, comp=dict(comp), nasa_low=coeffs, nasa_high=coeffs)


def _round(x, step):
    return float(round(x / step) * step)


M9_SPECIES = ["H2", "O2", "H2O", "H", "O", "OH", "HO2", "H2O2", "N2"]
_M9_COMP = {"H2": {"H": 2}, "O2": {"O": 2}, "H2O": {"H": 2, "O": 1}, "H": {"H": 1},
            "O": {"O": 1}, "OH": {"O": 1, "H": 1}, "HO2": {"H": 1, "O": 2},
            "H2O2": {"H": 2, "O": 2}, "N2": {"N": 2}}
# seeded round-number ranges: formation enthalpy [kJ/mol], entropy [J/mol/K]
_M9_THERMO_RANGES = {
    "H2": ((0, 0), (125, 135)), "O2": ((0, 0), (200, 210)),
    "H2O": ((-250, -230), (185, 195)), "H": ((210, 225), (110, 118)),
    "O": ((240, 255), (157, 165)), "OH": ((30, 45), (180, 188)),
    "HO2": ((0, 20), (225, 233)), "H2O2": ((-145, -125), (228, 238)),
    "N2": ((0, 0), (187, 197)),
}


def _u(rng, lo, hi):
    return float(rng.uniform(lo, hi))


def _arr(rng, log10A, b, Ea_kcal):
    return (10.0 ** _u(rng, *log10A), _u(rng, *b) if isinstance(b, tuple) else float(b),
            1000.0 * (_u(rng, *Ea_kcal) if isinstance(Ea_kcal, tuple) else float(Ea_kcal)))


def make_m9(seed: int = M9_SEED) -> Mechanism:
    """9-species / 21-reaction H2-air-shaped mechanism: 4 chain-branching and
    shuffle reactions, 4 third-body recombinations, 2 Troe falloff reactions,
    11 HO2/H2O2 reactions (two duplicate pairs). N2 is inert but collides."""
    rng = np.random.default_rng(seed)
    species = []
    for name in M9_SPECIES:
        (h0, h1), (s0, s1) = _M9_THERMO_RANGES[name]
        dH = _round(_u(rng, h0, h1), 5.0) if h1 > h0 else 0.0
        S = _round(_u(rng, s0, s1), 0.5)
        species.append(_species(name, _M9_COMP[name], rng, dH, S))

    def eff(extra=None):
        e = {"H2": _round(_u(rng, 2.0, 3.0), 0.1), "H2O": _round(_u(rng, 10.0, 14.0), 0.1)}
        if extra:
            e.update(extra)
        return e

    Rx = []

    def add(reac, prod, log10A, b, Ea, kind="ELEMENTARY", **kw):
        A, bb, E = _arr(rng, log10A, b, Ea)
        Rx.append(Reaction(reactants=reac, products=prod, A=A, b=bb, Ea=E, kind=kind, **kw))

    # chain branching / shuffle
    add({"H": 1, "O2": 1}, {"O": 1, "OH": 1}, (13.8, 14.4), (-0.4, 0.0), (14.5, 17.0))
    add({"O": 1, "H2": 1}, {"H": 1, "OH": 1}, (13.3, 13.8), 0.0, (8.0, 10.0))
    add({"H2": 1, "OH": 1}, {"H2O": 1, "H": 1}, (12.8, 13.5), 0.0, (4.0, 6.0))
    add({"O": 1, "H2O": 1}, {"OH": 2}, (13.3, 14.0), 0.0, (16.0, 19.0))
    # third-body recombinations
    add({"H": 2}, {"H2": 1}, (17.5, 18.7), (-1.2, -0.6), 0.0, kind="THREEBODY", efficiencies=eff())
    add({"O": 2}, {"O2": 1}, (17.0, 18.0), (-1.0, -0.5), 0.0, kind="THREEBODY", efficiencies=eff())
    add({"O": 1, "H": 1}, {"OH": 1}, (17.8, 18.8), (-1.2, -0.6), 0.0, kind="THREEBODY", efficiencies=eff())
    add({"H": 1, "OH": 1}, {"H2O": 1}, (21.5, 22.5), (-2.2, -1.8), 0.0, kind="THREEBODY", efficiencies=eff())
    # falloff
    Ainf, binf, Einf = _arr(rng, (12.3, 12.9), (0.3, 0.6), 0.0)
    A0, b0, E0 = _arr(rng, (19.0, 20.0), (-1.8, -1.3), 0.0)
    Rx.append(Reaction({"H": 1, "O2": 1}, {"HO2": 1}, Ainf, binf, Einf, kind="FALLOFF",
                       efficiencies=eff(), low=(A0, b0, E0),
                       troe=[_u(rng, 0.5, 0.8), _u(rng, 1.0, 50.0), _u(rng, 1e3, 1e5)]))
    Ainf, binf, Einf = _arr(rng, (12.0, 12.8), 0.0, (47.0, 50.0))
    A0, b0, E0 = _arr(rng, (16.5, 17.5), 0.0, (42.0, 46.0))
    Rx.append(Reaction({"H2O2": 1}, {"OH": 2}, Ainf, binf, Einf, kind="FALLOFF",
                       efficiencies=eff(), low=(A0, b0, E0),
                       troe=[_u(rng, 0.4, 0.8), _u(rng, 1.0, 100.0), _u(rng, 1e3, 1e5),
                             _u(rng, 1e3, 1e4)]))
    # HO2 / H2O2
    rr = ((12.8, 13.8), (-0.5, 0.5), (0.0, 2.0))
    add({"HO2": 1, "H": 1}, {"H2": 1, "O2": 1}, *rr)
    add({"HO2": 1, "H": 1}, {"OH": 2}, *rr)
    add({"HO2": 1, "O": 1}, {"O2": 1, "OH": 1}, *rr)
    add({"HO2": 1, "OH": 1}, {"H2O": 1, "O2": 1}, *rr)
    add({"HO2": 2}, {"H2O2": 1, "O2": 1}, (11.0, 11.5), 0.0, (0.0, 1.0))
    add({"HO2": 2}, {"H2O2": 1, "O2": 1}, (13.8, 14.5), 0.0, (10.0, 12.0))
    add({"H2O2": 1, "H": 1}, {"H2O": 1, "OH": 1}, (12.8, 13.5), 0.0, (3.0, 5.0))
    add({"H2O2": 1, "H": 1}, {"HO2": 1, "H2": 1}, (13.0, 13.5), 0.0, (7.0, 9.0))
    add({"H2O2": 1, "O": 1}, {"OH": 1, "HO2": 1}, (12.0, 13.0), 0.0, (3.0, 6.0))
    add({"H2O2": 1, "OH": 1}, {"HO2": 1, "H2O": 1}, (12.0, 12.5), 0.0, (0.0, 1.0))
    add({"H2O2": 1, "OH": 1}, {"HO2": 1, "H2O": 1}, (14.0, 15.0), 0.0, (8.0, 10.0))
    assert len(Rx) == 21
    return Mechanism(name=f"M9-synthetic-H2-air-seed{seed}", elements=["H", "O", "N"],
                     species=species, reactions=Rx)


# ---------------------------------------------------------------------------
# 53-species C/H/O/N mechanism


M9_TWO_RANGE_SEED = 1009


def two_range_thermo(coeffs, kappa: float, Tmid: float = 1000.0):
    """A NASA-7 high-temperature set that differs from the low set by
    cp/R += kappa (T - Tmid)^2 for T >= Tmid, with the enthalpy and entropy
    constants chosen so that h and s are continuous at Tmid (cp is C1 there).
    The added cp term integrates to kappa (T - Tmid)^3 / 3 in h/R and to
    kappa (T^2/2 - 2 Tmid T + Tmid^2 ln T) + const in s/R."""
    a = list(coeffs)
    hi = list(a)
    hi[0] += kappa * Tmid * Tmid
    hi[1] += -2.0 * kappa * Tmid
    hi[2] += kappa
    hi[5] += -kappa * Tmid ** 3 / 3.0
    hi[6] += -kappa * Tmid * Tmid * (math.log(Tmid) - 1.5)
    return a, hi


def make_m9_two_range(seed: int = M9_TWO_RANGE_SEED) -> Mechanism:
    """The 9-species mechanism with distinct NASA-7 sets below and above
    Tmid = 1000 K (same reactions, so the same compiled structure): each
    species' high set adds a seeded kappa (T - Tmid)^2 to cp/R, |kappa| in
    [3e-8, 1.2e-7] (a 0.1-0.5 change of cp/R at 3000 K), with h, s and cp
    continuous at Tmid."""
    m = make_m9()
    rng = np.random.default_rng(seed)
    for sp in m.species:
        kappa = float(rng.uniform(3e-8, 1.2e-7) * rng.choice([-1.0, 1.0]))
        lo, hi = two_range_thermo(sp.nasa_low, kappa, sp.T_range[1])
        sp.nasa_low, sp.nasa_high = lo, hi
    m.name = "m9_two_range"
    return m


def _formula_name(comp: Dict[str, int]) -> str:
    s = ""
    for e in ("C", "H", "O", "N"):
        n = comp.get(e, 0)
        if n:
            s += e + (str(n) if n > 1 else "")
    return s


def make_m53(seed: int = M53_SEED, nspec: int = 53, nreac: int = 325) -> Mechanism:
    """Seeded element-balanced C/H/O/N mechanism. The nine H2-air species and
    a few carbon carriers are always present; the remaining species are seeded
    formulas C_aH_bO_cN_d (unique names, isomers get a suffix). Reactions are
    sampled from the balanced A+B<=>C+D, A+B<=>C and A<=>B+C sets; about 10%
    are THREEBODY and 5% FALLOFF (Troe)."""
    rng = np.random.default_rng(seed)
    comps: List[Dict[str, int]] = [dict(_M9_COMP[n]) for n in M9_SPECIES]
    names = list(M9_SPECIES)
    for c in ({"C": 1, "O": 1}, {"C": 1, "O": 2}, {"C": 1, "H": 4}, {"C": 1, "H": 3},
              {"C": 1, "H": 2, "O": 1}, {"C": 1, "H": 1, "O": 1}, {"C": 2, "H": 2},
              {"C": 2, "H": 4}, {"N": 1, "O": 1}, {"N": 1}):
        comps.append(c)
        names.append(_formula_name(c))
    while len(comps) < nspec:
        c = {"C": int(rng.integers(0, 4)), "H": int(rng.integers(0, 7)),
             "O": int(rng.integers(0, 3)), "N": int(rng.integers(0, 2))}
        c = {k: v for k, v in c.items() if v}
        na = sum(c.values())
        if na < 2 or na > 9:
            continue
        nm = _formula_name(c)
        k = 1
        base = nm
        while nm in names:
            k += 1
            nm = f"{base}-{k}"
        if k > 2:
            continue
        comps.append(c)
        names.append(nm)
    species = []
    for nm, c in zip(names, comps):
        na = sum(c.values())
        if nm in _M9_THERMO_RANGES:
            (h0, h1), (s0, s1) = _M9_THERMO_RANGES[nm]
            dH = _round(_u(rng, h0, h1), 5.0) if h1 > h0 else 0.0
            S = _round(_u(rng, s0, s1), 0.5)
        else:
            # group-additivity style enthalpy: O-rich species stable, odd-H
            # (radical) species penalised, seeded scatter
            rad = 120.0 if (c.get("H", 0) + c.get("N", 0)) % 2 else 0.0
            dH = _round(-100.0 * c.get("O", 0) + 20.0 * c.get("C", 0) - 10.0 * c.get("H", 0)
                        + 30.0 * c.get("N", 0) + rad + _u(rng, -30.0, 30.0), 5.0)
            S = _round(110.0 + 28.0 * na + _u(rng, -15.0, 15.0), 0.5)
        species.append(_species(nm, c, rng, dH, S, theta_lo=400.0))

    elems = ["C", "H", "O", "N"]
    vec = [np.array([c.get(e, 0) for e in elems]) for c in comps]
    ns = len(comps)
    inert = names.index("N2")
    # enumerate balanced candidate reactions
    cand: List[Tuple[Tuple[int, ...], Tuple[int, ...]]] = []
    pairs = [(i, j) for i in range(ns) for j in range(i, ns) if inert not in (i, j)]
    sums: Dict[Tuple[int, ...], List[Tuple[int, int]]] = {}
    for (i, j) in pairs:
        sums.setdefault(tuple(vec[i] + vec[j]), []).append((i, j))
    for key, lst in sums.items():
        for a, b in itertools.combinations(lst, 2):
            if set(a) & set(b):
                continue
            cand.append((a, b))           # A+B <=> C+D
    single = {tuple(v): k for k, v in enumerate(vec) if k != inert}
    for key, lst in sums.items():
        if key in single:
            for a in lst:
                cand.append((a, (single[key],)))   # A+B <=> C
    cand = sorted(set(cand))
    order = rng.permutation(len(cand))
    chosen = [cand[k] for k in order[:nreac]]
    if len(chosen) < nreac:
        raise RuntimeError("not enough balanced candidate reactions")

    def stoich(idx):
        d: Dict[str, int] = {}
        for k in idx:
            d[names[k]] = d.get(names[k], 0) + 1
        return d

    Rx = []
    for (lhs, rhs) in chosen:
        u = rng.uniform()
        if len(rhs) == 1:
            # association written as A+B(+M) <=> C: third-body or falloff
            kind = "FALLOFF" if u < 0.3 else "THREEBODY"
        else:
            kind = "THREEBODY" if u < 0.04 else "ELEMENTARY"
        # A log-uniform 1e8..1e14 read as the rate coefficient at 1000 K, so the
        # file's pre-exponential is A_1000 / 1000^b (keeps k(T) bounded for b = +2)
        b = _u(rng, -2.0, 2.0)
        A = 10.0 ** _u(rng, 8.0, 14.0) / 1000.0 ** b
        Ea = 1000.0 * _u(rng, 0.0, 50.0)
        r = Reaction(reactants=stoich(lhs), products=stoich(rhs), A=A, b=b, Ea=Ea, kind=kind)
        if kind in ("THREEBODY", "FALLOFF"):
            r.efficiencies = {"H2O": _round(_u(rng, 5.0, 12.0), 0.1),
                              "CO2": _round(_u(rng, 1.5, 3.5), 0.1)}
        if kind == "FALLOFF":
            r.low = (r.A * 10.0 ** _u(rng, 3.0, 6.0), r.b - _u(rng, 0.0, 1.0), 0.0)
            r.troe = [_u(rng, 0.3, 0.9), _u(rng, 10.0, 300.0), _u(rng, 800.0, 5000.0)]
        Rx.append(r)
    return Mechanism(name=f"M53-synthetic-CHON-seed{seed}", elements=elems,
                     species=species, reactions=Rx)
