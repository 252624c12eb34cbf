"""The library's one-lane BDF stepper compiled for the CPU (a test harness
in tests/host_stepper/, never part of the library): its step-size control
checked on the CPU against the oracle, against an emulation of the bare FP32
hardware log2/exp2 instructions in the controllers' power, and the last-step
rule on the case where t + (t_end - t) rounds below t_end."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from synth import fields

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
P = ctypes.POINTER(ctypes.c_double)


@pytest.fixture(scope="module")
def hs(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    from paper_2510_23993_amd import build
    build.generate()   # the compiled mechanism's structure header
    out = str(tmp_path_factory.mktemp("hs") / "libhs.so")
    cmd = [HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O2", "-std=c++17", "-fPIC", "-shared",
           "-ffp-contract=on", "-I", os.path.join(ROOT, "paper_2510_23993_amd", "csrc"), "-o", out,
           os.path.join(ROOT, "tests", "host_stepper", "harness.cpp")]
    subprocess.run(cmd, check=True, capture_output=True)
    lib = ctypes.CDLL(out)
    lib.hs_next_step.argtypes = [ctypes.c_double] * 4 + [P, P]
    return lib


def integrate(lib, mode, rho, Y, T, dt, rtol, atol, kmax=100000):
    n = rho.size
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    Y = np.ascontiguousarray(Y, dtype=np.float64).copy()
    T = np.ascontiguousarray(T, dtype=np.float64).copy()
    st = np.zeros(n, np.uint8)
    att = np.zeros(n, np.int64)
    rc = lib.hs_integrate(fields.M9_PATH.encode(), mode, ctypes.c_int64(n), rho.ctypes.data_as(P),
                          Y.ctypes.data_as(P), T.ctypes.data_as(P), ctypes.c_double(dt), ctypes.c_double(rtol),
                          ctypes.c_double(atol), kmax, st.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                          att.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    assert rc == 0
    return Y, T, st, att


@pytest.mark.parametrize("mode", [0, 1, 2, 3])
def test_host_stepper_matches_oracle(hs, m9, mode):
    # 1e-6 relative on species above 1e-10 and 1e-3 K, as the GPU parity
    # tests, with every controller power (library FP32, bare-instruction
    # emulation, FP64 pow, and results moved by up to 2 ulp)
    c = fields.c1_cells(300, seed=1001)
    rho, e = m9.state_from_TPY(c.T, c.p, c.Y)
    T0 = np.array([m9.T_from_e(e[i], c.Y[:, i]) for i in range(rho.size)])
    Yh, Th, st, att = integrate(hs, mode, rho, c.Y, T0, c.dt, 1e-8, 1e-20)
    assert np.all(st == 0)
    Yr, Tr, so = m9.integrate(rho, e, c.Y, c.dt, 1e-12, 1e-20, T=c.T)
    big = Yr > 1e-10
    rel = np.max(np.where(big, np.abs(Yh - Yr) / np.where(big, Yr, 1.0), 0.0))
    assert rel <= 1e-6 and np.max(np.abs(Th - Tr)) <= 1e-3


def test_retry_at_the_clamped_size_is_the_last_step(hs):
    # after a clamp h = t_end - t, an attempt retried at that size (a Newton
    # failure with a stale Jacobian keeps the step) must again be flagged as
    # the last one and land exactly on t_end; also for t far below t_end,
    # where t_end - t is rounded (t + fl(t_end - t) still rounds to t_end)
    rng = np.random.default_rng(3)
    for tend in (5e-9, 1e-8, 2e-8, 4e-8, 1e-7):
        for t0 in np.concatenate([rng.uniform(0.0, tend, 2000), tend * rng.uniform(0.0, 1.0, 2000) ** 12]):
            h = tend - t0
            hn, fac = ctypes.c_double(), ctypes.c_double()
            last = hs.hs_next_step(t0, h, tend, 1.0, ctypes.byref(hn), ctypes.byref(fac))
            assert last == 1 and hn.value == tend - t0 and t0 + hn.value == tend
            # a step that falls short is not flagged, one beyond is clamped
            last = hs.hs_next_step(t0, 0.5 * h, tend, 1.0, ctypes.byref(hn), ctypes.byref(fac))
            assert (last == 1) == (t0 + 0.5 * h >= tend or 0.5 * h >= tend - t0)
            last = hs.hs_next_step(t0, h, tend, 3.0, ctypes.byref(hn), ctypes.byref(fac))
            assert last == 1 and hn.value == tend - t0 and fac.value == (tend - t0) / h


def test_amr_cells_finish_with_the_bare_instruction_power(hs, m9):
    # every active cell of nine AMR boxes (three per level, all three dt)
    # finishes with the emulated FP32 instructions in the controllers' power
    boxes = fields.c3_boxes()
    pick = []
    for lev in range(3):
        pick += [i for i, b in enumerate(boxes) if b.level == lev and np.prod(b.shape) <= 8192][:3]
    total = 0
    for i in pick:
        c = fields.c3_box_state(boxes[i], box_id=i)
        act = c.T >= 500.0
        rho, _ = m9.state_from_TPY(c.T[act], c.p[act], c.Y[:, act])
        for mode in (1, 3):
            Yh, Th, st, att = integrate(hs, mode, rho, c.Y[:, act], c.T[act], c.dt, 1e-8, 1e-20)
            assert np.all(st == 0), (i, mode, np.bincount(st))
        total += int(act.sum())
    assert total > 20000


@pytest.mark.parametrize("n", [1, 2, 3, 5, 9, 10, 16])
def test_library_lu_against_numpy(hs, n):
    # the one-lane kernel's dense LU and solve (compiled for the CPU) against
    # numpy's LAPACK solve: random systems, systems that need row exchanges
    # (zero leading diagonal), and singular or non-finite ones reported
    rng = np.random.default_rng(7 + n)
    hs.hs_lu.argtypes = [ctypes.c_int, P, P]
    for trial in range(40):
        A = rng.normal(size=(n, n))
        if trial % 4 == 1 and n > 1:   # a permuted diagonal-heavy matrix: every pivot needs an exchange
            A = np.roll(np.eye(n) * 3.0 + 0.1 * rng.normal(size=(n, n)), 1, axis=0)
        if trial % 4 == 2:             # Newton-like matrices I - c J
            A = np.eye(n) - rng.uniform(1e-3, 1e3) * rng.normal(size=(n, n))
        b = rng.normal(size=n)
        x = b.copy()
        Ac = np.ascontiguousarray(A)
        assert hs.hs_lu(n, Ac.ctypes.data_as(P), x.ctypes.data_as(P)) == 1
        ref = np.linalg.solve(A, b)
        tol = 1e-13 * np.linalg.cond(A) * max(1.0, np.max(np.abs(ref)))
        assert np.max(np.abs(x - ref)) <= tol, (n, trial)
    if n > 1:
        A = rng.normal(size=(n, n))
        A[:, n // 2] = 0.0             # exactly singular: a zero pivot
        x = rng.normal(size=n)
        assert hs.hs_lu(n, np.ascontiguousarray(A).ctypes.data_as(P), x.ctypes.data_as(P)) == 0
    A = rng.normal(size=(n, n))
    A[n - 1, n - 1] = np.nan
    x = rng.normal(size=n)
    assert hs.hs_lu(n, np.ascontiguousarray(A).ctypes.data_as(P), x.ctypes.data_as(P)) == 0
