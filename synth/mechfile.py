"""Writer for the plain-text kinetic mechanism format read by both the CPU
oracle and the HIP library (each has its own parser).

Format (whitespace-separated tokens, '#' starts a comment to end of line)::

    MECHANISM <name>
    UNITS CM-MOL-S CAL/MOL
    ELEMENTS <ne> <E1> ... <Ene>
    SPECIES <ns>
      <name> <W g/mol> <count E1> ... <count Ene>          (ns lines)
    THERMO
      <name> <Tlow> <Tmid> <Thigh> <a1..a7 for T < Tmid> <a1..a7 for T >= Tmid>
    REACTIONS <nr>
      REACTION <ELEMENTARY|THREEBODY|FALLOFF> <REV|IRREV>
        REACTANTS <m> <sp> <nu> ...   PRODUCTS <m> <sp> <nu> ...
        ARRHENIUS <A> <b> <Ea>
        [EFFICIENCIES <m> <sp> <alpha> ...]   (THREEBODY / FALLOFF; default 1)
        [LOW <A0> <b0> <Ea0>]                 (FALLOFF, required)
        [TROE <3|4> <a> <T***> <T*> [<T**>]]  (FALLOFF; absent = Lindemann)
      END
    END

Units follow the CHEMKIN convention: A in (cm^3/mol)^(order-1)/s with order
= sum of reactant coefficients (+1 for a THREEBODY reaction and for the
low-pressure limit of a FALLOFF reaction), Ea in cal/mol, W in g/mol.
NASA-7 polynomials are the usual ones (cp/R = a1 + a2 T + ... + a5 T^4,
a6 the enthalpy constant, a7 the entropy constant).

This module only serialises data; it evaluates none of the kinetics.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

ATOMIC_MASS = {"H": 1.008, "C": 12.011, "N": 14.007, "O": 15.999, "X": 10.0}


@dataclass
class Species:
    name: str
    comp: Dict[str, int]                 # element -> atom count
    nasa_low: Sequence[float]            # a1..a7 for T < Tmid
    nasa_high: Sequence[float]           # a1..a7 for T >= Tmid
    T_range: Tuple[float, float, float] = (200.0, 1000.0, 6000.0)
    W: Optional[float] = None            # g/mol; default from composition


@dataclass
class Reaction:
    reactants: Dict[str, int]
    products: Dict[str, int]
    A: float
    b: float
    Ea: float                            # cal/mol
    kind: str = "ELEMENTARY"             # ELEMENTARY | THREEBODY | FALLOFF
    reversible: bool = True
    efficiencies: Dict[str, float] = field(default_factory=dict)
    low: Optional[Tuple[float, float, float]] = None
    troe: Optional[Sequence[float]] = None

    def equation(self) -> str:
        def side(d):
            return " + ".join((f"{n} " if n > 1 else "") + s for s, n in d.items())
        m = {"ELEMENTARY": "", "THREEBODY": " + M", "FALLOFF": " (+M)"}[self.kind]
        arrow = " <=> " if self.reversible else " => "
        return side(self.reactants) + m + arrow + side(self.products) + m


@dataclass
class Mechanism:
    name: str
    elements: List[str]
    species: List[Species]
    reactions: List[Reaction]


def molecular_weight(sp: Species) -> float:
    if sp.W is not None:
        return sp.W
    return sum(ATOMIC_MASS[e] * n for e, n in sp.comp.items())


def _f(x: float) -> str:
    return repr(float(x))


def format_mechanism(m: Mechanism) -> str:
    names = [s.name for s in m.species]
    if len(set(names)) != len(names):
        raise ValueError("duplicate species names")
    out = [f"# {m.name}: {len(m.species)} species, {len(m.reactions)} reactions",
           f"MECHANISM {m.name}", "UNITS CM-MOL-S CAL/MOL",
           "ELEMENTS " + str(len(m.elements)) + " " + " ".join(m.elements),
           f"SPECIES {len(m.species)}"]
    for s in m.species:
        cnt = " ".join(str(int(s.comp.get(e, 0))) for e in m.elements)
        out.append(f"  {s.name} {_f(molecular_weight(s))} {cnt}")
    out.append("THERMO")
    for s in m.species:
        lo = " ".join(_f(a) for a in s.nasa_low)
        hi = " ".join(_f(a) for a in s.nasa_high)
        tl, tm, th = s.T_range
        out.append(f"  {s.name} {_f(tl)} {_f(tm)} {_f(th)}")
        out.append(f"    {lo}")
        out.append(f"    {hi}")
    out.append(f"REACTIONS {len(m.reactions)}")
    for j, r in enumerate(m.reactions):
        for d in (r.reactants, r.products):
            for s, n in d.items():
                if s not in names or int(n) != n or n <= 0:
                    raise ValueError(f"reaction {j}: bad participant {s}:{n}")
        out.append(f"  # R{j + 1}: {r.equation()}")
        out.append(f"  REACTION {r.kind} {'REV' if r.reversible else 'IRREV'}")
        out.append("    REACTANTS " + str(len(r.reactants)) + " " +
                   " ".join(f"{s} {n}" for s, n in r.reactants.items()))
        out.append("    PRODUCTS " + str(len(r.products)) + " " +
                   " ".join(f"{s} {n}" for s, n in r.products.items()))
        out.append(f"    ARRHENIUS {_f(r.A)} {_f(r.b)} {_f(r.Ea)}")
        if r.kind in ("THREEBODY", "FALLOFF") and r.efficiencies:
            out.append("    EFFICIENCIES " + str(len(r.efficiencies)) + " " +
                       " ".join(f"{s} {_f(a)}" for s, a in r.efficiencies.items()))
        if r.kind == "FALLOFF":
            if r.low is None:
                raise ValueError("FALLOFF reaction without LOW")
            out.append("    LOW " + " ".join(_f(x) for x in r.low))
            if r.troe is not None:
                out.append(f"    TROE {len(r.troe)} " + " ".join(_f(x) for x in r.troe))
        out.append("  END")
    out.append("END")
    return "\n".join(out) + "\n"


def write_mechanism(m: Mechanism, path: str) -> str:
    txt = format_mechanism(m)
    with open(path, "w") as fh:
        fh.write(txt)
    return path
