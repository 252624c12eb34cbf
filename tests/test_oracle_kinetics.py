"""Oracle rates pinned by conservation laws, detailed balance at an
independently computed equilibrium, falloff limits and the parser's checks."""
import numpy as np
import pytest

from oracle import gibbs
from synth.mechfile import Reaction
from tests import toymech

R = 8.314462618


def _random_state(m, rng):
    T = rng.uniform(600.0, 3200.0)
    p = rng.uniform(0.5, 40.0) * 101325.0
    Y = rng.dirichlet(np.ones(m.ns) * 0.7)
    rho = p / (R * T * np.sum(Y / m.W))
    return rho, np.concatenate([Y, [T]])


def test_mass_and_element_conservation(m9):
    rng = np.random.default_rng(11)
    for _ in range(300):
        rho, y = _random_state(m9, rng)
        f = m9.rhs(rho, y)
        om = f[:-1] * rho / m9.W                      # molar production rates
        kf, kr, qf, qr = m9.rates(y[-1], rho * y[:-1] / m9.W)
        gross = np.sum(qf + qr) * np.max(m9.W) * 4
        assert abs(np.sum(f[:-1])) * rho <= 1e-14 * gross + 1e-300
        for e in range(m9.ne):
            el = m9.comp[:, e] @ om
            assert abs(el) <= 1e-13 * np.sum(qf + qr) * 6 + 1e-300


def test_detailed_balance_at_gibbs_equilibrium(m9):
    # q_f = q_r for every reaction at the TP equilibrium from the Gibbs minimiser
    rng = np.random.default_rng(5)
    for _ in range(12):
        T = rng.uniform(900.0, 3200.0)
        p = rng.uniform(0.5, 40.0) * 101325.0
        Y0 = rng.dirichlet(np.ones(m9.ns))
        b = gibbs.element_moles_from_Y(m9, Y0)
        X = gibbs.equilibrate_TP(m9, T, p, b)
        res, el = gibbs.equilibrium_residuals(m9, T, p, X, b)
        assert res < 1e-9 and el < 1e-12
        Ye = gibbs.Y_from_X(m9, X)
        rho = p / (R * T * np.sum(Ye / m9.W))
        kf, kr, qf, qr = m9.rates(T, rho * Ye / m9.W)
        assert np.all(np.abs(qf - qr) <= 1e-9 * np.maximum(qf, qr))


def test_gibbs_minimiser_cross_checked_by_slsqp(m9):
    X0 = np.zeros(m9.ns)
    X0[0], X0[1], X0[-1] = 2.0, 1.0, 3.76
    Y0 = gibbs.Y_from_X(m9, X0 / X0.sum())
    b = gibbs.element_moles_from_Y(m9, Y0)
    for T, p in ((2500.0, 20 * 101325.0), (3000.0, 101325.0)):
        Xe = gibbs.equilibrate_TP(m9, T, p, b)
        Xs = gibbs.equilibrate_slsqp(m9, T, p, b, np.full(m9.ns, 1.0 / m9.ns))
        big = Xe > 1e-4
        assert np.allclose(Xs[big], Xe[big], rtol=1e-5)


def test_equilibrium_constant_of_isomerisation(oracle_lib):
    # A <=> B with equal enthalpies: Kc = exp(a7_B - a7_A), independent of T
    o = oracle_lib.Oracle(toymech.write(toymech.isomer_AB(da7=0.7), "iso"))
    for T in (500.0, 1500.0):
        kf, kr, _, _ = o.rates(T, np.array([1.0, 1.0, 1.0]))
        assert kf[0] / kr[0] == pytest.approx(np.exp(0.7), rel=1e-13)


def test_lindemann_limits(oracle_lib):
    # k = kinf Pr/(1+Pr): Pr -> 0 gives k0 [M], Pr -> inf gives kinf (SI units)
    Ainf, A0 = 1e7, 1e13
    o = oracle_lib.Oracle(toymech.write(toymech.falloff_iso(Ainf=Ainf, A0=A0), "lind"))
    k0_SI = A0 * 1e-6
    for M in (1e-10, 1e-6):
        kf = o.rates(1000.0, np.array([1.0, 1.0, M]))[0][0]
        assert kf == pytest.approx(k0_SI * M, rel=1e-5)
    kf = o.rates(1000.0, np.array([1.0, 1.0, 1e14]))[0][0]
    assert kf == pytest.approx(Ainf, rel=1e-6)


def test_troe_center_point(oracle_lib):
    # at log10 Pr = -c (c = -0.4 - 0.67 log10 Fcent) the broadening factor is Fcent
    a, T3, T1 = 1.0, 1e30, 700.0
    T = 1400.0
    Fc = np.exp(-T / T1)
    c = -0.4 - 0.67 * np.log10(Fc)
    Ainf, A0 = 1e7, 1e13
    Pr = 10 ** (-c)
    M = Pr * Ainf / (A0 * 1e-6)
    o = oracle_lib.Oracle(toymech.write(toymech.falloff_iso(Ainf, A0, troe=[a, T3, T1]), "troe"))
    kf = o.rates(T, np.array([1.0, 1.0, M]))[0][0]
    assert kf == pytest.approx(Ainf * Pr / (1 + Pr) * Fc, rel=1e-12)


def test_parser_rejects_unbalanced_and_bad_input(oracle_lib, tmp_path):
    m = toymech.isomer_AB()
    m.reactions.append(Reaction({"A": 1}, {"N2": 1}, A=1.0, b=0.0, Ea=0.0))
    p = tmp_path / "bad.mech"
    from synth.mechfile import format_mechanism
    p.write_text(format_mechanism(m))
    with pytest.raises(ValueError, match="balanced"):
        oracle_lib.Oracle(str(p))
    good = format_mechanism(toymech.isomer_AB())
    for bad in (good.replace("CM-MOL-S", "MKS"), good.replace("ARRHENIUS", "ARRH"),
                good.replace("REACTIONS 1", "REACTIONS 2")):
        p.write_text(bad)
        with pytest.raises(ValueError):
            oracle_lib.Oracle(str(p))


def test_m9_is_balanced_and_every_species_reachable(m9):
    # the parser enforces element balance; every species takes part in a reaction
    # (N2 only as a collider)
    import re
    txt = open(m9_path_str()).read()
    used = set(re.findall(r"(?:REACTANTS|PRODUCTS) \d+ ((?:\S+ \d+ ?)+)", txt))
    names = set()
    for grp in used:
        toks = grp.split()
        names.update(toks[0::2])
    assert names == set(m9.species) - {"N2"}
    assert m9.nr == 21


def m9_path_str():
    from synth.fields import M9_PATH
    return M9_PATH


def test_m9_file_matches_generator():
    from synth.mechfile import format_mechanism
    from synth.mechgen import make_m9
    assert open(m9_path_str()).read() == format_mechanism(make_m9())
