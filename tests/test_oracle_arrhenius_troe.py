"""Oracle rate constants pinned away from the special cases b = Ea = 0 and
the Troe centre point (Sec. 2.1: Arrhenius rates with third-body and
falloff reactions; Troe's broadening of the falloff curve).

- Arrhenius temperature dependence: closed-form solutions of isothermal
  model reactions with b != 0 and Ea != 0 (so a slip in the cal -> J
  conversion, in R, or in the sign or placement of b or Ea changes the
  integrated composition), and the log-linear structure of k(T).
- Troe: points where the broadening exponent f1 takes the values 0, +-1
  and +-2 (log10 F = log10 Fcent / (1 + f1^2) is then Fcent, Fcent^(1/2)
  and Fcent^(1/5)), the limit |log10 Pr| -> infinity where f1 -> -1/0.14,
  and each of the three Fcent terms isolated, including the optional T**
  term exp(-T**/T).
"""
import numpy as np
import pytest

from synth.mechfile import Reaction
from tests import toymech

R = 8.314462618
CAL = 4.184


def arrhenius_SI(A_SI, b, Ea_cal, T):
    """k = A T^b exp(-Ea/(R T)) with Ea given in cal/mol."""
    return A_SI * T ** b * np.exp(-Ea_cal * CAL / (R * T))


def _cell(o, T, p, Y):
    rho, e = o.state_from_TPY(np.array([T]), p, np.asarray(Y, dtype=float).reshape(-1, 1))
    return rho[0], e[0]


@pytest.mark.parametrize("b,Ea", [(1.7, 12000.0), (-1.3, 3000.0), (0.0, 25000.0), (2.5, 0.0)])
def test_isomerisation_with_temperature_dependent_rate(oracle_lib, b, Ea):
    # A <=> B, equal h and cp: T stays exactly at T0, Kc = exp(0.7), and the
    # composition relaxes as A_eq + (A0 - A_eq) exp(-(kf + kr) t)
    A = 50.0                                   # 1/s (first order: no unit conversion)
    o = oracle_lib.Oracle(toymech.write(toymech.isomer_AB(A=A, b=b, Ea=Ea, da7=0.7), "isoT"))
    Kc = np.exp(0.7)
    Y = np.array([0.3, 0.05, 0.65])
    for T0 in (800.0, 1500.0, 2400.0):
        kf = arrhenius_SI(A, b, Ea, T0)
        kr = kf / Kc
        dt = 0.7 / (kf + kr)                   # about half the relaxation done
        rho, e = _cell(o, T0, 3e5, Y)
        Yo, To, st = o.integrate([rho], [e], Y.reshape(3, 1), dt, 1e-11, 1e-16)
        assert st[0] == 0
        assert To[0] == pytest.approx(T0, rel=1e-12)
        tot = Y[0] + Y[1]
        Aeq = tot / (1 + Kc)
        A_t = Aeq + (Y[0] - Aeq) * np.exp(-(kf + kr) * dt)
        assert Yo[0, 0] == pytest.approx(A_t, rel=1e-8), (T0, b, Ea)
        # a units slip in Ea (J read as cal, or the reverse) moves the answer far
        wrong = arrhenius_SI(A, b, Ea / CAL, T0) if Ea else 2 * kf
        A_w = Aeq + (Y[0] - Aeq) * np.exp(-(wrong + wrong / Kc) * dt)
        assert abs(Yo[0, 0] - A_w) > 1e-4 * Y[0]


def test_dimerisation_with_temperature_dependent_rate(oracle_lib):
    # 2A => B releases no heat: 1/C_A = 1/C_A0 + 2 k t with the second-order
    # A converted from cm^3/mol/s and T^b exp(-Ea/RT) at the constant T
    A_cgs, b, Ea = 4e9, 0.8, 6000.0
    o = oracle_lib.Oracle(toymech.write(toymech.dimer(A=A_cgs, b=b, Ea=Ea), "dimerT"))
    Y = np.array([0.2, 0.0, 0.8])
    for T0 in (900.0, 2000.0):
        k = arrhenius_SI(A_cgs * 1e-6, b, Ea, T0)
        rho, e = _cell(o, T0, 5e5, Y)
        C0 = rho * Y[0] / o.W[0]
        dt = 1.0 / (2 * k * C0)                # C_A halves
        Yo, To, st = o.integrate([rho], [e], Y.reshape(3, 1), dt, 1e-11, 1e-16)
        assert st[0] == 0 and To[0] == pytest.approx(T0, rel=1e-12)
        CA = rho * Yo[0, 0] / o.W[0]
        assert 1.0 / CA == pytest.approx(1.0 / C0 + 2 * k * dt, rel=1e-8)


def test_rate_constant_is_log_linear_in_inverse_T_and_log_T(oracle_lib):
    # ln k = ln A + b ln T - Ea/(R T): a least-squares plane through
    # (1, ln T, 1/T) reproduces ln A, b and -Ea/R exactly (to rounding)
    A, b, Ea = 3.0e4, -0.9, 17000.0
    o = oracle_lib.Oracle(toymech.write(toymech.isomer_AB(A=A, b=b, Ea=Ea), "loglin"))
    Ts = np.array([400.0, 700.0, 1000.0, 1600.0, 2300.0, 3100.0])
    lnk = np.array([np.log(o.rates(T, np.array([1.0, 1.0, 1.0]))[0][0]) for T in Ts])
    X = np.stack([np.ones_like(Ts), np.log(Ts), 1.0 / Ts], axis=1)
    coef, res, *_ = np.linalg.lstsq(X, lnk, rcond=None)
    assert coef[0] == pytest.approx(np.log(A), rel=1e-10)
    assert coef[1] == pytest.approx(b, rel=1e-9)
    assert -coef[2] * R == pytest.approx(Ea * CAL, rel=1e-10)      # slope in J/mol
    assert np.max(np.abs(X @ coef - lnk)) < 1e-11


def test_low_pressure_limit_carries_its_own_arrhenius(oracle_lib):
    # Pr -> 0: kf -> k0 [M] with k0 = A0 T^b0 exp(-Ea0/RT) (second order: cm^3 -> m^3)
    A0, b0, Ea0 = 2e14, -1.1, 4000.0
    m = toymech.isomer_AB()
    m.reactions = [Reaction({"A": 1}, {"B": 1}, A=1e9, b=0.4, Ea=9000.0, kind="FALLOFF",
                            reversible=False, efficiencies={"A": 0.0, "B": 0.0},
                            low=(A0, b0, Ea0))]
    o = oracle_lib.Oracle(toymech.write(m, "lowT"))
    for T in (700.0, 1800.0):
        M = 1e-12
        kf = o.rates(T, np.array([1.0, 1.0, M]))[0][0]
        assert kf == pytest.approx(arrhenius_SI(A0 * 1e-6, b0, Ea0, T) * M, rel=1e-8)


# ------------------------------------------------------------------ Troe
AINF, A0 = 1e7, 1e13          # 1/s and cm^3/mol/s: k0 = 1e7 m^3/mol/s


def _troe_oracle(oracle_lib, troe, tag):
    return oracle_lib.Oracle(toymech.write(toymech.falloff_iso(AINF, A0, troe=list(troe)), tag))


def _F(o, T, log10Pr):
    """Broadening factor F = kf / (kinf Pr/(1+Pr)) at the given Pr."""
    Pr = 10.0 ** log10Pr
    M = Pr * AINF / (A0 * 1e-6)
    kf = o.rates(T, np.array([1.0, 1.0, M]))[0][0]
    return kf / (AINF * Pr / (1.0 + Pr))


def _x_for_f1(Fc, f1):
    """log10 Pr at which the Troe parameter f1 = u/(n - 0.14 u), u = log10 Pr + c,
    takes the value f1 (c = -0.4 - 0.67 log10 Fcent, n = 0.75 - 1.27 log10 Fcent)."""
    lf = np.log10(Fc)
    c, n = -0.4 - 0.67 * lf, 0.75 - 1.27 * lf
    u = f1 * n / (1.0 + 0.14 * f1)
    return u - c


@pytest.mark.parametrize("f1,power", [(0.0, 1.0), (1.0, 0.5), (-1.0, 0.5), (2.0, 0.2), (-2.0, 0.2)])
def test_troe_broadening_off_centre(oracle_lib, f1, power):
    # log10 F = log10 Fcent / (1 + f1^2): F = Fcent^(1/(1+f1^2)) at chosen f1
    a, T3, T1, T = 0.6, 200.0, 1500.0, 1300.0
    o = _troe_oracle(oracle_lib, (a, T3, T1), "troe3")
    Fc = (1 - a) * np.exp(-T / T3) + a * np.exp(-T / T1)
    F = _F(o, T, _x_for_f1(Fc, f1))
    assert F == pytest.approx(Fc ** power, rel=1e-11)


def test_troe_limit_of_large_log_Pr(oracle_lib):
    # |log10 Pr| -> infinity: f1 -> -1/0.14 on both sides, so
    # log10 F -> log10 Fcent / (1 + (1/0.14)^2); the approach is O(1/|log10 Pr|)
    a, T3, T1, T = 1.0, 1e30, 700.0, 1400.0
    o = _troe_oracle(oracle_lib, (a, T3, T1), "troelim")
    Fc = np.exp(-T / T1)
    lim = np.log10(Fc) / (1.0 + (1.0 / 0.14) ** 2)
    for sgn in (1.0, -1.0):
        L = {x: np.log10(_F(o, T, sgn * x)) for x in (37.5, 75.0, 150.0, 300.0)}
        errs = [abs(L[x] - lim) for x in (37.5, 75.0, 150.0, 300.0)]
        assert all(errs[i + 1] < 0.6 * errs[i] for i in range(3)), errs
        # two Richardson steps on the expansion in 1/x land on the limit
        ext = (8 * L[300.0] - 6 * L[150.0] + L[75.0]) / 3
        assert ext == pytest.approx(lim, rel=2e-4)
    # with u = log10 Pr + c, |f1| = |u| / |n - 0.14 u| exceeds 1/0.14 for u -> +inf
    # and stays below it for u -> -inf, so log10 F (< 0) approaches the limit
    # from above on the high-pressure side and from below on the low-pressure
    # side; a sign slip in the 0.14 term reverses the order
    assert np.log10(_F(o, T, -300.0)) < lim < np.log10(_F(o, T, 300.0))


@pytest.mark.parametrize("params,Fc_of_T", [
    # T*** term alone (a = 0, T* -> 0): Fcent = exp(-T/T***)
    ((0.0, 300.0, 1e-30), lambda T: np.exp(-T / 300.0)),
    # T* term alone (a = 1): Fcent = exp(-T/T*)
    ((1.0, 1e-30, 900.0), lambda T: np.exp(-T / 900.0)),
    # the fourth parameter alone (a = 0, T*** -> 0, T* -> 0): Fcent = exp(-T**/T)
    ((0.0, 1e-30, 1e-30, 1800.0), lambda T: np.exp(-1800.0 / T)),
])
def test_troe_fcent_terms_one_at_a_time(oracle_lib, params, Fc_of_T):
    o = _troe_oracle(oracle_lib, params, "troeterm")
    for T in (900.0, 1600.0, 2500.0):
        Fc = Fc_of_T(T)
        assert _F(o, T, _x_for_f1(Fc, 0.0)) == pytest.approx(Fc, rel=1e-11)   # centre: F = Fcent
        assert _F(o, T, _x_for_f1(Fc, 1.0)) == pytest.approx(np.sqrt(Fc), rel=1e-11)
