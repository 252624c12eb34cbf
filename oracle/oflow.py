"""CPU FP64 reference of the minimal compressible flow step used for the
Strang-split coupling (test infrastructure only: the test suite, the smoke
check and the benchmark's CPU-baseline leg may import it; the product library
shares no code with it).

The paper advances the reacting Euler equations with HLLC convective fluxes
and second-order SSP Runge-Kutta time stepping, and treats the chemical
source term by operator splitting (Sec. 2.1).  Here, in one dimension, the
conserved state per cell is U = (rho, rho u, rho E, rho Y_1 .. rho Y_ns) with
E = e + u^2/2 and e the mass-specific internal energy including formation
energy (NASA-7 absolute-enthalpy basis, the same e as the chemistry step).

Readings fixed here (the paper gives the scheme's names, not its details):
  * primitive reconstruction: piecewise linear in (rho, u, p, Y_k) with the
    minmod slope limiter (MUSCL), face states q_i +- slope_i / 2;
  * wave speeds of the HLLC solver (Toro, Riemann Solvers and Numerical
    Methods for Fluid Dynamics, 3rd ed., Sec. 10.4-10.6): the direct
    estimates S_L = min(u_L - c_L, u_R - c_R), S_R = max(u_L + c_L, u_R + c_R),
    S* from the momentum balance of the two star states, species carried as
    passive scalars with the contact;
  * frozen sound speed c^2 = gamma p / rho with gamma = cp/cv of the mixture
    at the face state's T;
  * SSP-RK2 (Heun): U1 = U + dt L(U), U' = (U + U1 + dt L(U1)) / 2;
  * transmissive boundaries: two ghost cells copying the end cells;
  * Strang splitting of one coupled step: flow dt/2, chemistry dt (constant
    rho and e per cell, so only rho Y_k changes), flow dt/2.

Everything is plain numpy float64 with per-cell calls into the oracle's thermo.
"""
from __future__ import annotations

import numpy as np

R = 8.314462618


def prim_from_cons(orc, U, Tguess=None):
    """U [3+ns][n] -> rho, u, p, T, Y [ns][n]."""
    ns = orc.ns
    rho = U[0]
    u = U[1] / rho
    E = U[2] / rho
    Y = U[3:3 + ns] / rho
    e = E - 0.5 * u * u
    n = rho.size
    T = np.empty(n)
    for i in range(n):
        T[i] = orc.T_from_e(e[i], Y[:, i], np.nan if Tguess is None else Tguess[i])
    p = rho * R * T * np.sum(Y / orc.W[:, None], axis=0)
    return rho, u, p, T, Y


def cons_from_prim(orc, rho, u, p, Y):
    """Conserved state from (rho, u, p, Y); T from the ideal-gas law."""
    ns = orc.ns
    Wm = np.sum(Y / orc.W[:, None], axis=0)
    T = p / (rho * R * Wm)
    e = np.array([orc.e_mass(T[i], Y[:, i]) for i in range(rho.size)])
    U = np.empty((3 + ns, rho.size))
    U[0] = rho
    U[1] = rho * u
    U[2] = rho * (e + 0.5 * u * u)
    U[3:] = rho * Y
    return U


def _minmod(a, b):
    return np.where(a * b > 0.0, np.where(np.abs(a) < np.abs(b), a, b), 0.0)


def _face_thermo(orc, rho, p, Y):
    """T, e, sound speed c of face states given (rho, p, Y)."""
    Wm = np.sum(Y / orc.W[:, None], axis=0)
    T = p / (rho * R * Wm)
    n = rho.size
    e = np.empty(n)
    cv = np.empty(n)
    for i in range(n):
        e[i] = orc.e_mass(T[i], Y[:, i])
        cv[i] = orc.cv_mass(T[i], Y[:, i])
    cp = cv + R * Wm
    c = np.sqrt(cp / cv * p / rho)
    return T, e, c


def hllc_flux(orc, rhoL, uL, pL, YL, rhoR, uR, pR, YR):
    """HLLC flux of the multispecies Euler equations for face states L | R."""
    _, eL, cL = _face_thermo(orc, rhoL, pL, YL)
    _, eR, cR = _face_thermo(orc, rhoR, pR, YR)
    EL = rhoL * (eL + 0.5 * uL * uL)
    ER = rhoR * (eR + 0.5 * uR * uR)
    SL = np.minimum(uL - cL, uR - cR)
    SR = np.maximum(uL + cL, uR + cR)
    Ss = (pR - pL + rhoL * uL * (SL - uL) - rhoR * uR * (SR - uR)) / (rhoL * (SL - uL) - rhoR * (SR - uR))

    def flux(rho, u, p, E, Y):
        return np.vstack([rho * u, rho * u * u + p, u * (E + p), rho * u * Y])

    def cons(rho, u, E, Y):
        return np.vstack([rho, rho * u, E, rho * Y])

    def star(rho, u, p, E, Y, S):
        f = rho * (S - u) / (S - Ss)
        return np.vstack([f, f * Ss, f * (E / rho + (Ss - u) * (Ss + p / (rho * (S - u)))), f * Y])

    FL = flux(rhoL, uL, pL, EL, YL)
    FR = flux(rhoR, uR, pR, ER, YR)
    F = np.where(0.0 <= SL, FL,
                 np.where(0.0 <= Ss, FL + SL * (star(rhoL, uL, pL, EL, YL, SL) - cons(rhoL, uL, EL, YL)),
                          np.where(0.0 <= SR, FR + SR * (star(rhoR, uR, pR, ER, YR, SR) - cons(rhoR, uR, ER, YR)),
                                   FR)))
    return F


def rhs_flow(orc, U, dx, T=None):
    """L(U) = -(F_{i+1/2} - F_{i-1/2}) / dx with MUSCL-minmod faces and
    transmissive ends."""
    rho, u, p, T, Y = prim_from_cons(orc, U, T)
    q = np.vstack([rho, u, p, Y])                      # [3+ns][n]
    qg = np.concatenate([q[:, :1], q[:, :1], q, q[:, -1:], q[:, -1:]], axis=1)   # two ghosts per side
    d = np.diff(qg, axis=1)                            # [.., n+3]
    slope = _minmod(d[:, :-1], d[:, 1:])               # cells 1 .. n+2 of qg
    qc = qg[:, 1:-1]                                    # cells -1 .. n
    qL = (qc + 0.5 * slope)[:, :-1]                    # left state at faces -1/2 .. n-1/2
    qR = (qc - 0.5 * slope)[:, 1:]                     # right state at the same faces
    ns = orc.ns
    F = hllc_flux(orc, qL[0], qL[1], qL[2], qL[3:3 + ns], qR[0], qR[1], qR[2], qR[3:3 + ns])
    return -(F[:, 1:] - F[:, :-1]) / dx, T


def flow_step(orc, U, dx, dt):
    """One SSP-RK2 step of the flow."""
    L0, T0 = rhs_flow(orc, U, dx)
    U1 = U + dt * L0
    L1, _ = rhs_flow(orc, U1, dx, T0)
    return 0.5 * (U + U1 + dt * L1)


def strang_step(orc, U, dx, dt, rtol, atol):
    """Flow dt/2, chemistry dt (the oracle's BDF at constant rho and e), flow dt/2."""
    ns = orc.ns
    U = flow_step(orc, U, dx, 0.5 * dt)
    rho, u, p, T, Y = prim_from_cons(orc, U)
    e = U[2] / rho - 0.5 * u * u
    Yo, To, st = orc.integrate(rho, e, Y, dt, rtol, atol, T=T)
    U = U.copy()
    U[3:3 + ns] = rho * Yo
    return flow_step(orc, U, dx, 0.5 * dt), st
