"""CPU FP64 oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It wraps ``liboracle.so`` (plain C + OpenMP, built from
the sources in this folder) through ctypes.  It shares no code with the
product library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SOURCES = ["omech.c", "okin.c", "obdf.c", "odriver.c"]

ST_DONE, ST_SKIPPED, ST_KMAX, ST_FAIL, ST_TINV = 0, 1, 2, 3, 4


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (-O2, IEEE arithmetic, OpenMP)."""
    if not force and os.path.exists(LIB):
        return LIB
    srcs = [os.path.join(HERE, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
           "-ffp-contract=off", "-Wall", "-Wno-unused-function", "-o", tmp] + srcs + ["-lm"]
    subprocess.run(cmd, check=True, cwd=HERE)
    os.replace(tmp, LIB)
    return LIB


_lib = None
dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
lp = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        vp = C.c_void_p
        L.oracle_last_error.restype = C.c_char_p
        L.oracle_load.restype = vp
        L.oracle_load.argtypes = [C.c_char_p]
        L.oracle_free.argtypes = [vp]
        L.oracle_info.argtypes = [vp, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.oracle_species_name.restype = C.c_char_p
        L.oracle_species_name.argtypes = [vp, C.c_int]
        L.oracle_element_name.restype = C.c_char_p
        L.oracle_element_name.argtypes = [vp, C.c_int]
        L.oracle_species_data.argtypes = [vp, dp, ip]
        L.oracle_thermo.argtypes = [vp, C.c_int, C.c_double, dp]
        L.oracle_e_mass.restype = C.c_double
        L.oracle_e_mass.argtypes = [vp, C.c_double, dp]
        L.oracle_cv_mass.restype = C.c_double
        L.oracle_cv_mass.argtypes = [vp, C.c_double, dp]
        L.oracle_T_from_e.argtypes = [vp, C.c_double, dp, C.c_double, C.POINTER(C.c_double)]
        L.oracle_state_from_TPY.argtypes = [vp, C.c_long, dp, dp, dp, dp, dp]
        L.oracle_rates.argtypes = [vp, C.c_double, dp, dp, dp, dp, dp]
        L.oracle_rhs.argtypes = [vp, C.c_double, dp, dp]
        L.oracle_jac.argtypes = [vp, C.c_double, dp, dp]
        L.oracle_integrate.restype = C.c_long
        L.oracle_integrate.argtypes = [vp, C.c_long, dp, dp, dp, C.c_long, dp, C.c_double,
                                       C.c_double, C.c_double, C.c_long, C.c_int, u8p, vp]
        L.oracle_trajectory.argtypes = [vp, C.c_double, C.c_double, dp, C.c_double, C.c_double,
                                        dp, C.c_int, dp, C.c_double, C.c_double, C.c_long]
        L.oracle_bdf_linear.argtypes = [C.c_int, dp, dp, C.c_double, C.c_double, C.c_double,
                                        C.c_long, vp, C.c_int, vp, lp]
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Oracle:
    """One parsed mechanism plus the oracle's kinetics and integrator."""

    def __init__(self, mech_path: str):
        L = lib()
        self._h = L.oracle_load(mech_path.encode())
        if not self._h:
            raise ValueError("oracle: " + L.oracle_last_error().decode())
        ns, nr, ne = C.c_int(), C.c_int(), C.c_int()
        L.oracle_info(self._h, C.byref(ns), C.byref(nr), C.byref(ne))
        self.ns, self.nr, self.ne = ns.value, nr.value, ne.value
        self.n = self.ns + 1
        self.species = [L.oracle_species_name(self._h, k).decode() for k in range(self.ns)]
        self.elements = [L.oracle_element_name(self._h, e).decode() for e in range(self.ne)]
        self.W = np.zeros(self.ns)
        comp = np.zeros(self.ns * self.ne, dtype=np.int32)
        L.oracle_species_data(self._h, self.W, comp)
        self.comp = comp.reshape(self.ns, self.ne)

    def __del__(self):
        try:
            if self._h:
                lib().oracle_free(self._h)
        except Exception:
            pass

    # thermo
    def thermo(self, k: int, T: float):
        out = np.zeros(4)
        lib().oracle_thermo(self._h, k, float(T), out)
        return out  # cp/R, h/RT, s/R, d(cp/R)/dT

    def e_mass(self, T, Y):
        return lib().oracle_e_mass(self._h, float(T), _f64(Y))

    def cv_mass(self, T, Y):
        return lib().oracle_cv_mass(self._h, float(T), _f64(Y))

    def T_from_e(self, e, Y, Tguess=float("nan")):
        T = C.c_double()
        rc = lib().oracle_T_from_e(self._h, float(e), _f64(Y), float(Tguess), C.byref(T))
        if rc != 0:
            raise ValueError("temperature inversion failed")
        return T.value

    def state_from_TPY(self, T, p, Y):
        """T, p: [n]; Y: [ns][n] column-major.  Returns (rho, e)."""
        T = _f64(np.atleast_1d(T))
        p = _f64(np.broadcast_to(np.asarray(p, dtype=np.float64), T.shape))
        Y = _f64(Y).reshape(self.ns, T.size)
        rho = np.zeros(T.size)
        e = np.zeros(T.size)
        lib().oracle_state_from_TPY(self._h, T.size, T, p, Y, rho, e)
        return rho, e

    def concentrations(self, rho, Y):
        return rho * np.asarray(Y) / self.W

    def rates(self, T, Cc):
        kf, kr, qf, qr = (np.zeros(max(self.nr, 1)) for _ in range(4))
        lib().oracle_rates(self._h, float(T), _f64(Cc), kf, kr, qf, qr)
        return kf[:self.nr], kr[:self.nr], qf[:self.nr], qr[:self.nr]

    def rhs(self, rho, y):
        f = np.zeros(self.n)
        lib().oracle_rhs(self._h, float(rho), _f64(y), f)
        return f

    def jac(self, rho, y):
        J = np.zeros(self.n * self.n)
        lib().oracle_jac(self._h, float(rho), _f64(y), J)
        return J.reshape(self.n, self.n)

    # integration
    def integrate(self, rho, e, Y, dt, rtol, atol, T=None, max_steps=10**7, nthreads=0,
                  with_stats=False):
        """Advance every cell over [0, dt].  Y: [ns][ncell] (copied).
        Returns (Y_out, T_out, status[, stats[ncell,5]])."""
        rho = _f64(rho)
        e = _f64(e)
        ncell = rho.size
        Yo = np.array(Y, dtype=np.float64, copy=True).reshape(self.ns, ncell)
        Yo = np.ascontiguousarray(Yo)
        To = np.full(ncell, np.nan) if T is None else np.array(T, dtype=np.float64, copy=True)
        st = np.zeros(ncell, dtype=np.uint8)
        cs = np.zeros((ncell, 5), dtype=np.int64) if with_stats else None
        lib().oracle_integrate(self._h, ncell, rho, e, Yo, ncell, To, float(dt), float(rtol),
                               float(atol), int(max_steps), int(nthreads), st,
                               cs.ctypes.data if cs is not None else None)
        if with_stats:
            return Yo, To, st, cs
        return Yo, To, st

    def trajectory(self, rho, e, Y0, t1, tout, rtol, atol, Tguess=float("nan"), max_steps=10**7):
        tout = _f64(tout)
        yout = np.zeros((tout.size, self.n))
        st = lib().oracle_trajectory(self._h, float(rho), float(e), _f64(Y0), float(Tguess),
                                     float(t1), tout, tout.size, yout, float(rtol), float(atol),
                                     int(max_steps))
        return yout, st


def bdf_linear(A, y0, t1, rtol, atol, tout=None, max_steps=10**7):
    """Integrate y' = A y from 0 to t1 with the oracle's BDF."""
    A = _f64(A)
    n = A.shape[0]
    y = _f64(y0).copy()
    stats = np.zeros(7, dtype=np.int64)
    if tout is not None:
        tout = _f64(tout)
        yout = np.zeros((tout.size, n))
        st = lib().oracle_bdf_linear(n, A.ravel(), y, float(t1), float(rtol), float(atol),
                                     int(max_steps), tout.ctypes.data, tout.size,
                                     yout.ctypes.data, stats)
        return y, st, stats, yout
    st = lib().oracle_bdf_linear(n, A.ravel(), y, float(t1), float(rtol), float(atol),
                                 int(max_steps), None, 0, None, stats)
    return y, st, stats
