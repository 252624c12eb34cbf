"""Small hand-built mechanisms used to pin the oracle against closed forms."""
import os
import tempfile

from synth.mechfile import Mechanism, Reaction, Species, write_mechanism


def const_cp_species(name, comp, cp_R=3.5, a6=0.0, a7=0.0, W=None, scale=1.0):
    a = [cp_R * scale, 0.0, 0.0, 0.0, 0.0, a6 * scale, a7]
    return Species(name=name, comp=comp, nasa_low=a, nasa_high=a, W=W)


def write(m: Mechanism, tag: str) -> str:
    d = tempfile.mkdtemp(prefix="toymech_")
    return write_mechanism(m, os.path.join(d, tag + ".mech"))


def isomer_AB(A=1e6, Ea=0.0, b=0.0, da7=0.7, reversible=True):
    """A <=> B with identical a1..a6 (same h, cp) and different a7, equal W:
    T stays exactly constant and Kc = exp(a7_B - a7_A)."""
    sp = [const_cp_species("A", {"X": 1}, a6=-1000.0, a7=2.0, W=20.0),
          const_cp_species("B", {"X": 1}, a6=-1000.0, a7=2.0 + da7, W=20.0),
          const_cp_species("N2", {"N": 2})]
    rx = [Reaction({"A": 1}, {"B": 1}, A=A, b=b, Ea=Ea, reversible=reversible)]
    return Mechanism("isomer", ["X", "N"], sp, rx)


def dimer(A=3e12, reversible=False, b=0.0, Ea=0.0):
    """2A => B with molar internal energies u_B = 2 u_A at every T (so
    h_B/RT = 2 h_A/RT - 1): the reaction releases no heat and T is constant."""
    sp = [const_cp_species("A", {"X": 1}, a6=500.0, a7=3.0, W=20.0),
          const_cp_species("B", {"X": 2}, a6=500.0, a7=3.0, W=40.0, scale=2.0),
          const_cp_species("N2", {"N": 2})]
    sp[1].nasa_low = [6.0, 0, 0, 0, 0, 1000.0, 5.0]
    sp[1].nasa_high = list(sp[1].nasa_low)
    rx = [Reaction({"A": 2}, {"B": 1}, A=A, b=b, Ea=Ea, reversible=reversible)]
    return Mechanism("dimer", ["X", "N"], sp, rx)


def thirdbody_iso(A=5e9, effA=0.0, effB=0.0):
    """A + M => B + M with zero efficiency for A and B, so [M] = C_N2."""
    m = isomer_AB()
    m.reactions = [Reaction({"A": 1}, {"B": 1}, A=A, b=0.0, Ea=0.0, kind="THREEBODY",
                            reversible=False, efficiencies={"A": effA, "B": effB})]
    m.name = "thirdbody"
    return m


def falloff_iso(Ainf=1e7, A0=1e13, troe=None):
    """A (+M) => B (+M), Lindemann or Troe, temperature-independent k_inf and
    k0, zero efficiency for A and B (so [M] = C_N2)."""
    m = isomer_AB()
    m.reactions = [Reaction({"A": 1}, {"B": 1}, A=Ainf, b=0.0, Ea=0.0, kind="FALLOFF",
                            reversible=False, efficiencies={"A": 0.0, "B": 0.0},
                            low=(A0, 0.0, 0.0), troe=troe)]
    m.name = "falloff"
    return m


def toy4():
    """4 species, 3 reversible reactions: elementary, third-body, Troe falloff,
    with temperature-dependent cp.  Used for the symbolic Jacobian check."""
    def sp(name, comp, a, W=None):
        return Species(name=name, comp=comp, nasa_low=a, nasa_high=a, W=W)
    s = [sp("A2", {"X": 2}, [3.3, 1.2e-3, -3.0e-7, 4.0e-11, -2.0e-15, -900.0, 4.0]),
         sp("A", {"X": 1}, [2.5, 1.0e-5, 0.0, 0.0, 0.0, 25000.0, 3.0]),
         sp("A3", {"X": 3}, [4.1, 2.0e-3, -6.0e-7, 8.0e-11, -4.0e-15, 5000.0, 6.0]),
         sp("N2", {"N": 2}, [3.5, 2.0e-4, 0.0, 0.0, 0.0, -1000.0, 4.5])]
    rx = [Reaction({"A2": 1, "A": 1}, {"A3": 1}, A=2e12, b=0.3, Ea=3000.0),
          Reaction({"A": 2}, {"A2": 1}, A=1e17, b=-0.8, Ea=0.0, kind="THREEBODY",
                   efficiencies={"A2": 2.5, "N2": 0.7}),
          Reaction({"A2": 1, "A": 1}, {"A3": 1}, A=5e12, b=0.5, Ea=1000.0, kind="FALLOFF",
                   efficiencies={"A3": 3.0}, low=(1e19, -1.4, 0.0),
                   troe=[0.6, 200.0, 1500.0, 3000.0])]
    return Mechanism("toy4", ["X", "N"], s, rx)
