"""Thin Python binding of libchem (ctypes).  Argument marshalling only: every
step of the hot path runs in the library's HIP kernels.  Torch tensors are
used as device memory (their data pointers go through the C ABI) and the
current torch stream is the default context stream.

The library must be built (``python -m paper_2510_23993_amd.build`` or
``__graft_entry__.build()``); importing this module without it raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libchem.so")

CHEM_OK, CHEM_W_INCOMPLETE = 0, 1
ST_DONE, ST_SKIPPED, ST_KMAX, ST_FAIL, ST_TINV, ST_SURR_OK, ST_SURR_REJ = range(7)


class chem_stats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in (
        "ncell", "n_active0", "n_active_after_bulk", "n_bulk_rounds", "n_sparse", "n_incomplete",
        "n_fallback", "steps_total", "attempts_total", "rhs_evals", "jac_evals", "lu_facts",
        "lin_solves", "max_steps_cell")] + [(n, C.c_double) for n in (
        "t_total_ms", "t_screen_ms", "t_bulk_ms", "t_sparse_ms")] + [(n, C.c_int64) for n in (
        "bulk_rhs_evals", "bulk_jac_evals", "bulk_lu_facts", "bulk_lin_solves")] + [
        ("n_surrogate", C.c_int64), ("t_surrogate_ms", C.c_double), ("surr_reject", C.c_int64 * 4),
        ("t_flow_ms", C.c_double), ("flow_bad_cells", C.c_int64)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["surr_reject"] = list(d["surr_reject"])
        return d


class chem_box(C.Structure):
    _fields_ = [("ncell", C.c_int64), ("rho", C.c_void_p), ("e", C.c_void_p), ("Y", C.c_void_p),
                ("ldY", C.c_int64), ("T", C.c_void_p), ("mask", C.c_void_p), ("status", C.c_void_p),
                ("dt", C.c_double), ("level", C.c_int)]


class ChemError(RuntimeError):
    def __init__(self, rc, msg):
        super().__init__(f"libchem error {rc}: {msg}")
        self.rc = rc


_lib = None

EXPORTS = ["chem_load_mechanism", "chem_mech_info", "chem_species_name", "chem_free_mechanism",
           "chem_ctx_create", "chem_ctx_destroy", "chem_set_option", "chem_get_option",
           "chem_load_surrogate", "chem_integrate", "chem_integrate_boxes", "chem_prepare_state",
           "chem_eval_rhs", "chem_synchronize", "chem_last_error", "chem_autotune",
           "chem_mlp_nparams", "chem_mlp_workspace_floats", "chem_mlp_forward", "chem_mlp_backward",
           "chem_mlp_mse", "chem_mlp_adam", "chem_mlp_gather", "chem_mlp_take", "chem_mlp_colstats",
           "chem_mlp_standardize", "chem_mlp_colrange", "chem_surrogate_pairs", "chem_mech_hash",
           "chem_flow_step", "chem_strang_step", "chem_integrate_noalloc",
           "chem_eval_contractions"]


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libchem.so not built ({LIB_PATH}); run paper_2510_23993_amd/build.py")
    # One HIP runtime per process: torch ships its own libamdhip64 (soname
    # libamdhip64.so.7) and its libraries request it by the unversioned name.
    # Loading torch first makes libchem's libamdhip64.so.7 dependency resolve
    # to that already-loaded runtime, so device pointers and streams are shared.
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    vp, i64, dbl = C.c_void_p, C.c_int64, C.c_double
    L.chem_last_error.restype = C.c_char_p
    L.chem_load_mechanism.argtypes = [C.c_char_p, C.POINTER(vp)]
    L.chem_mech_info.argtypes = [vp, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.POINTER(dbl))]
    L.chem_species_name.argtypes = [vp, C.c_int, C.POINTER(C.c_char_p)]
    L.chem_free_mechanism.argtypes = [vp]
    L.chem_free_mechanism.restype = None
    L.chem_ctx_create.argtypes = [vp, C.c_int, vp, C.POINTER(vp)]
    L.chem_ctx_destroy.argtypes = [vp]
    L.chem_ctx_destroy.restype = None
    L.chem_set_option.argtypes = [vp, C.c_char_p, dbl]
    L.chem_get_option.argtypes = [vp, C.c_char_p, C.POINTER(dbl)]
    L.chem_load_surrogate.argtypes = [vp, C.c_char_p]
    L.chem_integrate.argtypes = [vp, i64, vp, vp, vp, i64, vp, vp, vp, dbl, dbl, dbl,
                                 C.POINTER(chem_stats)]
    L.chem_integrate_noalloc.argtypes = [vp, i64, vp, vp, vp, i64, vp, vp, vp, dbl, dbl, dbl]
    L.chem_eval_contractions.argtypes = [vp, i64, vp, vp, vp, C.c_int]
    L.chem_integrate_boxes.argtypes = [vp, C.c_int, C.POINTER(chem_box), dbl, dbl, C.POINTER(chem_stats)]
    L.chem_flow_step.argtypes = [vp, i64, dbl, dbl, vp, i64, vp]
    L.chem_strang_step.argtypes = [vp, i64, dbl, dbl, vp, i64, vp, vp, dbl, dbl, C.POINTER(chem_stats)]
    L.chem_prepare_state.argtypes = [vp, i64, vp, vp, vp, i64, vp, vp]
    L.chem_eval_rhs.argtypes = [vp, i64, vp, vp, vp, vp]
    L.chem_synchronize.argtypes = [vp]
    L.chem_autotune.argtypes = [vp, C.c_int, C.POINTER(chem_box), dbl, dbl, C.c_char_p,
                                C.POINTER(dbl)]
    L.chem_mlp_nparams.restype = i64
    L.chem_mlp_nparams.argtypes = []
    L.chem_mlp_workspace_floats.restype = i64
    L.chem_mlp_workspace_floats.argtypes = [i64]
    L.chem_mlp_forward.argtypes = [vp, i64, vp, vp, vp, vp, C.c_int]
    L.chem_mlp_backward.argtypes = [vp, i64, vp, vp, vp, vp, vp]
    L.chem_mlp_mse.argtypes = [vp, i64, vp, vp, vp, vp]
    L.chem_mlp_adam.argtypes = [vp, i64, vp, vp, vp, vp, dbl, dbl, dbl, dbl, C.c_int]
    L.chem_mlp_gather.argtypes = [vp, i64, vp, vp, i64, C.c_uint64, i64, vp, vp]
    L.chem_mlp_take.argtypes = [vp, i64, vp, vp, vp, vp, vp]
    L.chem_mlp_colstats.argtypes = [vp, i64, C.c_int, vp, vp, vp, vp]
    L.chem_mlp_standardize.argtypes = [vp, i64, C.c_int, vp, vp, vp]
    L.chem_mlp_colrange.argtypes = [vp, i64, C.c_int, vp, vp, vp, vp]
    L.chem_surrogate_pairs.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp, vp]
    L.chem_mech_hash.argtypes = [vp, C.POINTER(C.c_uint64)]
    _lib = L
    return L


def _check(rc):
    if rc < 0:
        raise ChemError(rc, lib().chem_last_error().decode())
    return rc


def _ptr(t):
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


def _check_f64(name, t, shape):
    import torch
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


class Mechanism:
    def __init__(self, path: str):
        h = C.c_void_p()
        _check(lib().chem_load_mechanism(path.encode(), C.byref(h)))
        self._h = h
        ns, nr = C.c_int(), C.c_int()
        W = C.POINTER(C.c_double)()
        _check(lib().chem_mech_info(h, C.byref(ns), C.byref(nr), C.byref(W)))
        self.ns, self.nr = ns.value, nr.value
        self.W = [W[k] for k in range(self.ns)]
        self.species = []
        for k in range(self.ns):
            nm = C.c_char_p()
            _check(lib().chem_species_name(h, k, C.byref(nm)))
            self.species.append(nm.value.decode())

    @property
    def hash(self) -> int:
        h = C.c_uint64()
        _check(lib().chem_mech_hash(self._h, C.byref(h)))
        return h.value

    def __del__(self):
        try:
            if self._h:
                lib().chem_free_mechanism(self._h)
                self._h = None
        except Exception:
            pass


class Context:
    """Device workspace + stream binding for one mechanism."""

    def __init__(self, mech: Mechanism, device: int = 0, stream=None, **options):
        import torch
        self.mech = mech
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = C.c_void_p()
        _check(lib().chem_ctx_create(mech._h, device, C.c_void_p(stream.cuda_stream), C.byref(h)))
        self._h = h
        for k, v in options.items():
            self.set_option(k, v)

    def __del__(self):
        try:
            if self._h:
                lib().chem_ctx_destroy(self._h)
                self._h = None
        except Exception:
            pass

    def set_option(self, key: str, value: float):
        _check(lib().chem_set_option(self._h, key.encode(), float(value)))

    def get_option(self, key: str) -> float:
        v = C.c_double()
        _check(lib().chem_get_option(self._h, key.encode(), C.byref(v)))
        return v.value

    def integrate(self, rho, e, Y, T, dt, rtol, atol, mask=None, status=None, stats=True):
        """rho, e, T: [n] float64 device tensors; Y: [ns, n] (column-major per
        species, i.e. a contiguous [ns][n] tensor).  Y and T are updated in
        place.  Returns the stats dict (synchronising) or None."""
        n = rho.shape[0]
        _check_f64("rho", rho, (n,))
        _check_f64("e", e, (n,))
        _check_f64("T", T, (n,))
        _check_f64("Y", Y, (self.mech.ns, n))
        st = chem_stats() if stats else None
        rc = _check(lib().chem_integrate(self._h, n, _ptr(rho), _ptr(e), _ptr(Y), n, _ptr(T),
                                         _ptr(mask), _ptr(status), float(dt), float(rtol),
                                         float(atol), C.byref(st) if st is not None else None))
        if st is None:
            return None
        d = st.as_dict()
        d["rc"] = rc
        return d

    def integrate_noalloc(self, rho, e, Y, T, dt, rtol, atol, mask=None, status=None):
        """chem_integrate_noalloc: as integrate() without statistics, on the
        library's fixed device scratch (no allocation; at most 2^20 cells)."""
        n = rho.shape[0]
        _check_f64("rho", rho, (n,))
        _check_f64("e", e, (n,))
        _check_f64("T", T, (n,))
        _check_f64("Y", Y, (self.mech.ns, n))
        return _check(lib().chem_integrate_noalloc(self._h, n, _ptr(rho), _ptr(e), _ptr(Y), n, _ptr(T),
                                                   _ptr(mask), _ptr(status), float(dt), float(rtol),
                                                   float(atol)))

    def flow_step(self, U, T, dx, dt):
        """One SSP-RK2 step of the 1-D flow: U [3+ns, n], T [n] (in: guess,
        out: T of the new state); synchronises."""
        n = T.shape[0]
        _check_f64("T", T, (n,))
        _check_f64("U", U, (3 + self.mech.ns, n))
        _check(lib().chem_flow_step(self._h, n, float(dx), float(dt), _ptr(U), n, _ptr(T)))

    def strang_step(self, U, T, dx, dt, rtol, atol, status=None, stats=True):
        """Flow dt/2, chemistry dt, flow dt/2 (U, T as flow_step)."""
        n = T.shape[0]
        _check_f64("T", T, (n,))
        _check_f64("U", U, (3 + self.mech.ns, n))
        st = chem_stats() if stats else None
        rc = _check(lib().chem_strang_step(self._h, n, float(dx), float(dt), _ptr(U), n, _ptr(T), _ptr(status),
                                           float(rtol), float(atol), C.byref(st) if st is not None else None))
        if st is None:
            return None
        d = st.as_dict()
        d["rc"] = rc
        return d

    def integrate_boxes(self, boxes: Sequence[dict], rtol, atol, stats=True):
        """boxes: dicts with rho, e, Y ([ns, n]), T, dt and optional mask,
        status, level."""
        arr = self._box_array(boxes)
        st = chem_stats() if stats else None
        rc = _check(lib().chem_integrate_boxes(self._h, len(boxes), arr, float(rtol), float(atol),
                                               C.byref(st) if st is not None else None))
        if st is None:
            return None
        d = st.as_dict()
        d["rc"] = rc
        return d

    def _box_array(self, boxes):
        arr = (chem_box * len(boxes))()
        for i, b in enumerate(boxes):
            n = b["rho"].shape[0]
            for k in ("rho", "e", "T"):
                _check_f64(k, b[k], (n,))
            _check_f64("Y", b["Y"], (self.mech.ns, n))
            arr[i] = chem_box(n, _ptr(b["rho"]), _ptr(b["e"]), _ptr(b["Y"]), n, _ptr(b["T"]),
                              _ptr(b.get("mask")), _ptr(b.get("status")), float(b["dt"]),
                              int(b.get("level", 0)))
        return arr

    def autotune(self, boxes: Sequence[dict], rtol, atol, cache_path: Optional[str] = None):
        """Pick the fastest schedule for these boxes; returns (options, ms)."""
        arr = self._box_array(boxes)
        ms = C.c_double()
        _check(lib().chem_autotune(self._h, len(boxes), arr, float(rtol), float(atol),
                                   cache_path.encode() if cache_path else None, C.byref(ms)))
        opts = {k: self.get_option(k) for k in ("group", "max_rounds", "nactive_star",
                                                 "kmax_bulk", "grid_waves")}
        return opts, ms.value

    def prepare_state(self, T, p, Y, rho, e):
        n = T.shape[0]
        _check(lib().chem_prepare_state(self._h, n, _ptr(T), _ptr(p), _ptr(Y), n, _ptr(rho), _ptr(e)))

    def eval_rhs(self, rho, y, f, J=None):
        n = rho.shape[0]
        _check(lib().chem_eval_rhs(self._h, n, _ptr(rho), _ptr(y), _ptr(f), _ptr(J)))

    def eval_contractions(self, lnC, zf, zr, precision=0):
        """chem_eval_contractions: zf = nu'^T lnC and zr = nu''^T lnC for n
        states; lnC [ns, n], zf and zr [nr, n] float64 device tensors."""
        n = lnC.shape[1]
        _check_f64("lnC", lnC, (self.mech.ns, n))
        _check_f64("zf", zf, (self.mech.nr, n))
        _check_f64("zr", zr, (self.mech.nr, n))
        _check(lib().chem_eval_contractions(self._h, n, _ptr(lnC), _ptr(zf), _ptr(zr), int(precision)))

    def synchronize(self):
        _check(lib().chem_synchronize(self._h))

    def load_surrogate(self, path: str):
        _check(lib().chem_load_surrogate(self._h, path.encode()))

    def surrogate_pairs(self, rho, Y0, T0, Y1, T1, dt, X, targets):
        """Raw float32 features [n][12] and targets [n][10] of increments."""
        n = rho.shape[0]
        _check(lib().chem_surrogate_pairs(self._h, n, _ptr(rho), _ptr(Y0), _ptr(T0), _ptr(Y1), _ptr(T1),
                                          _ptr(dt), _ptr(X), _ptr(targets)))


def _stream_handle(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class MLP:
    """The surrogate network's kernels on float32 device tensors (parameters
    in the flat layout of chem_mlp_forward)."""

    NIN, NOUT = 12, 10

    @staticmethod
    def nparams() -> int:
        return lib().chem_mlp_nparams()

    @staticmethod
    def workspace(batch, device="cuda"):
        import torch
        return torch.empty(int(lib().chem_mlp_workspace_floats(batch)), dtype=torch.float32, device=device)

    @staticmethod
    def forward(params, X, out, ws, mode=0, stream=None):
        _check(lib().chem_mlp_forward(_stream_handle(stream), X.shape[0], _ptr(params), _ptr(X), _ptr(out),
                                      _ptr(ws), int(mode)))

    @staticmethod
    def backward(params, X, ws, dout, grads, stream=None):
        _check(lib().chem_mlp_backward(_stream_handle(stream), X.shape[0], _ptr(params), _ptr(X), _ptr(ws),
                                       _ptr(dout), _ptr(grads)))

    @staticmethod
    def mse(out, target, dout, loss=None, stream=None):
        _check(lib().chem_mlp_mse(_stream_handle(stream), out.numel(), _ptr(out), _ptr(target), _ptr(dout),
                                  _ptr(loss)))

    @staticmethod
    def adam(params, grads, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        _check(lib().chem_mlp_adam(_stream_handle(stream), params.numel(), _ptr(params), _ptr(grads), _ptr(m),
                                   _ptr(v), float(lr), float(beta1), float(beta2), float(eps), int(step)))

    @staticmethod
    def gather(X, T, batch, seed, step, Xb, Tb, stream=None):
        _check(lib().chem_mlp_gather(_stream_handle(stream), X.shape[0], _ptr(X), _ptr(T), int(batch),
                                     int(seed) & 0xFFFFFFFFFFFFFFFF, int(step), _ptr(Xb), _ptr(Tb)))

    @staticmethod
    def take(idx, X, T, Xo, To, stream=None):
        """Rows idx (int64 device tensor) of X and T into Xo and To."""
        if idx.element_size() != 8 or idx.is_floating_point():
            raise TypeError("idx must be int64")
        _check(lib().chem_mlp_take(_stream_handle(stream), idx.numel(), _ptr(idx), _ptr(X), _ptr(T), _ptr(Xo),
                                   _ptr(To)))

    @staticmethod
    def colstats(data, acc, mean, sd, stream=None):
        _check(lib().chem_mlp_colstats(_stream_handle(stream), data.shape[0], data.shape[1], _ptr(data),
                                       _ptr(acc), _ptr(mean), _ptr(sd)))

    @staticmethod
    def colrange(data, scratch, lo, hi, stream=None):
        _check(lib().chem_mlp_colrange(_stream_handle(stream), data.shape[0], data.shape[1], _ptr(data),
                                       _ptr(scratch), _ptr(lo), _ptr(hi)))

    @staticmethod
    def standardize(data, mean, sd, stream=None):
        _check(lib().chem_mlp_standardize(_stream_handle(stream), data.shape[0], data.shape[1], _ptr(data),
                                          _ptr(mean), _ptr(sd)))
