"""The paper's explicit first-order kinetics scheme on the CPU, FP64 (test
infrastructure only: the test suite and the benchmark's CPU legs may use it;
the product library shares no code with it).

Sec. 2.1 and Alg. 2: each cell advances with forward-Euler steps
Y <- Y + dt_i * S, S = dY/dt from Eq. 5 (here from the oracle's own
right-hand side), with the local step chosen so that no mass fraction
changes by more than a set fraction (1-5%) of its current value; the
temperature follows from the fixed internal energy and density by Newton
iteration after every step.  Readings where the paper is silent:

- the limit uses max(|Y_k|, y_floor) (y_floor = 1e-10 by default), so a
  species at or near zero does not force a zero step;
- the last step is shortened to end exactly at dt;
- a cell stops after max_steps steps (status 2) or a failed temperature
  inversion (status 4), keeping its last state.

Each cell is a plain Python loop over its steps: slow, obviously in the
order of the paper's description, and meant for small samples.
"""
from __future__ import annotations

import numpy as np

ST_DONE, ST_KMAX, ST_TINV = 0, 2, 4


def step_size(Y, S, h_left, frac, y_floor):
    """Largest step <= h_left with |S_k| h <= frac max(|Y_k|, y_floor) for all k."""
    h = h_left
    for k in range(Y.size):
        if S[k] != 0.0:
            h = min(h, frac * max(abs(Y[k]), y_floor) / abs(S[k]))
    return h


def integrate_explicit(orc, rho, e, Y, T, dt, frac, y_floor=1e-10, max_steps=10**6):
    """Cells advanced from 0 to dt.  rho, e, T: [n]; Y: [ns][n] (column-major
    by cell).  Returns (Y, T, status, steps)."""
    rho = np.atleast_1d(np.asarray(rho, dtype=np.float64))
    e = np.atleast_1d(np.asarray(e, dtype=np.float64))
    T = np.atleast_1d(np.asarray(T, dtype=np.float64))
    n, ns = rho.size, orc.ns
    Yo = np.array(Y, dtype=np.float64).reshape(ns, n).copy()
    To = T.copy()
    status = np.zeros(n, dtype=np.uint8)
    steps = np.zeros(n, dtype=np.int64)
    for i in range(n):
        y = np.empty(ns + 1)
        y[:ns] = Yo[:, i]
        try:
            y[ns] = orc.T_from_e(e[i], y[:ns], To[i])
        except ValueError:
            status[i] = ST_TINV
            continue
        t, k, st = 0.0, 0, ST_DONE
        while True:
            if k >= max_steps:
                st = ST_KMAX
                break
            S = orc.rhs(rho[i], y)[:ns]
            h = step_size(y[:ns], S, dt - t, frac, y_floor)
            last = h >= dt - t
            y[:ns] = y[:ns] + h * S
            t = dt if last else t + h
            k += 1
            try:
                y[ns] = orc.T_from_e(e[i], y[:ns], y[ns])
            except ValueError:
                st = ST_TINV
                break
            if last:
                break
        Yo[:, i] = y[:ns]
        To[i] = y[ns]
        status[i] = st
        steps[i] = k
    return Yo, To, status, steps
