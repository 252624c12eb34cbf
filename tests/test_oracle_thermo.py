"""Oracle thermo pinned by calculus identities, closed forms and a round trip."""
import numpy as np
import pytest

from synth.mechfile import Mechanism, Species
from tests.toymech import write

R = 8.314462618


def _richardson(fun, T, d):
    """Central difference with one Richardson step (error O(d^4))."""
    D1 = (fun(T + d) - fun(T - d)) / (2 * d)
    D2 = (fun(T + d / 2) - fun(T - d / 2)) / d
    return (4 * D2 - D1) / 3


def test_cp_is_dh_dT_and_ds_dT(m9):
    # cp = d h / dT,  ds/dT = cp/T,  d cp/dT reported consistently
    for k in range(m9.ns):
        for T in (350.0, 800.0, 1500.0, 2600.0, 3400.0):
            d = 1e-3 * T
            cp, h, s, dcp = m9.thermo(k, T)
            dhdT = _richardson(lambda t: t * m9.thermo(k, t)[1], T, d)
            dsdT = _richardson(lambda t: m9.thermo(k, t)[2], T, d)
            dcpdT = _richardson(lambda t: m9.thermo(k, t)[0], T, d)
            assert dhdT == pytest.approx(cp, rel=1e-9)
            assert dsdT == pytest.approx(cp / T, rel=1e-9)
            assert dcpdT == pytest.approx(dcp, rel=1e-7, abs=1e-12)


def test_constant_cp_closed_form(oracle_lib):
    a = [3.5, 0, 0, 0, 0, -1200.0, 4.25]
    m = Mechanism("cp", ["N"], [Species("Q", {"N": 2}, a, a)], [])
    o = oracle_lib.Oracle(write(m, "cp"))
    for T in (300.0, 1000.0, 2500.0):
        cp, h, s, dcp = o.thermo(0, T)
        assert cp == 3.5 and dcp == 0.0
        assert h == pytest.approx(3.5 - 1200.0 / T, rel=1e-15)
        assert s == pytest.approx(3.5 * np.log(T) + 4.25, rel=1e-15)
        # e = (h - RT)/W, c_v = (cp - R)/W  (mass based)
        W = o.W[0]
        assert o.e_mass(T, [1.0]) == pytest.approx((2.5 * T - 1200.0) * R / W, rel=1e-14)
        assert o.cv_mass(T, [1.0]) == pytest.approx(2.5 * R / W, rel=1e-15)


def test_tmid_tie_uses_high_range(oracle_lib):
    lo = [3.0, 0, 0, 0, 0, 0.0, 0.0]
    hi = [4.0, 0, 0, 0, 0, 0.0, 0.0]
    m = Mechanism("tie", ["N"], [Species("Q", {"N": 2}, lo, hi, T_range=(200.0, 1000.0, 6000.0))], [])
    o = oracle_lib.Oracle(write(m, "tie"))
    assert o.thermo(0, 999.999)[0] == 3.0
    assert o.thermo(0, 1000.0)[0] == 4.0
    # outside the fitted range the polynomial is evaluated as is (no clamping)
    assert o.thermo(0, 100.0)[0] == 3.0 and o.thermo(0, 7000.0)[0] == 4.0


def test_T_e_round_trip(m9):
    rng = np.random.default_rng(7)
    for _ in range(200):
        T = rng.uniform(250.0, 4500.0)
        Y = rng.dirichlet(np.ones(m9.ns) * 0.5)
        e = m9.e_mass(T, Y)
        Tb = m9.T_from_e(e, Y, Tguess=rng.uniform(300, 3000))
        assert abs(Tb - T) < 1e-9


def test_T_inversion_rejects_out_of_bracket(m9):
    Y = np.zeros(m9.ns)
    Y[-1] = 1.0
    with pytest.raises(ValueError):
        m9.T_from_e(m9.e_mass(7000.0, Y), Y)


def test_state_from_TPY_ideal_gas(m9):
    rng = np.random.default_rng(3)
    n = 50
    T = rng.uniform(300, 3000, n)
    p = rng.uniform(1e5, 4e6, n)
    Y = rng.dirichlet(np.ones(m9.ns), n).T.copy()
    rho, e = m9.state_from_TPY(T, p, Y)
    Wmix = 1.0 / (Y / m9.W[:, None]).sum(0)
    assert np.allclose(p, rho * R * T / Wmix, rtol=1e-14)
    for i in range(n):
        assert e[i] == pytest.approx(m9.e_mass(T[i], Y[:, i]), rel=1e-15)


def test_two_range_thermo_continuous_at_tmid(oracle_lib):
    # the two-range variant of the 9-species mechanism: distinct sets below and
    # above 1000 K, cp, dcp/dT, h and s continuous at Tmid, the high set in use
    # above it (cp differs from the low polynomial by kappa (T - Tmid)^2)
    from synth import fields
    from synth.mechgen import make_m9_two_range
    o = oracle_lib.Oracle(fields.M9_TWO_RANGE_PATH)
    m = make_m9_two_range()
    for k in range(o.ns):
        below = o.thermo(k, 1000.0 * (1 - 1e-12))
        at = o.thermo(k, 1000.0)
        assert np.allclose(below[:3], at[:3], rtol=1e-9), (k, below, at)
        assert below[3] == pytest.approx(at[3], rel=1e-6, abs=1e-12)
        lo = m.species[k].nasa_low
        T = 2500.0
        cp_lo = sum(lo[i] * T ** i for i in range(5))
        kappa = m.species[k].nasa_high[2] - lo[2]
        assert abs(kappa) > 1e-8
        assert o.thermo(k, T)[0] == pytest.approx(cp_lo + kappa * (T - 1000.0) ** 2, rel=1e-12)
        for T in (700.0, 1300.0, 2800.0):     # calculus identities on both sides
            d = 1e-3 * T
            dhdT = _richardson(lambda t: t * o.thermo(k, t)[1], T, d)
            assert dhdT == pytest.approx(o.thermo(k, T)[0], rel=1e-9)


def test_two_range_file_matches_generator():
    from synth import fields
    from synth.mechfile import format_mechanism
    from synth.mechgen import make_m9_two_range
    assert open(fields.M9_TWO_RANGE_PATH).read() == format_mechanism(make_m9_two_range())
