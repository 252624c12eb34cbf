"""The CPU oracle built with AddressSanitizer, LeakSanitizer and
UndefinedBehaviorSanitizer (gcc, host code only) and run through a small C
driver (tests/oracle_sanitize/driver.c) on cells of both mechanisms: no
sanitizer report, and every result equal to the regular build's (the same
arithmetic: no fast-math, no contraction, in both builds)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import Oracle
from synth import fields

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    out = str(tmp_path_factory.mktemp("osan") / "driver")
    srcs = [os.path.join(ORACLE, s) for s in ("omech.c", "okin.c", "obdf.c", "odriver.c")]
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fno-omit-frame-pointer", "-fno-fast-math", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-I", ORACLE, "-o", out,
           os.path.join(ROOT, "tests", "oracle_sanitize", "driver.c")] + srcs + ["-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "sanitize" in r.stderr and "cannot find" in r.stderr:
        pytest.skip("sanitizer runtime not installed")
    assert r.returncode == 0, r.stderr[-2000:]
    return out


def _run(driver, tmp_path, path, cells, dt, rtol):
    ns = cells.Y.shape[0]
    f = tmp_path / "cells.txt"
    with open(f, "w") as fh:
        fh.write(f"{cells.T.size} {ns}\n")
        for i in range(cells.T.size):
            fh.write(" ".join(repr(float(v)) for v in [cells.T[i], cells.p[i], *cells.Y[:, i]]) + "\n")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([driver, path, str(f), repr(dt), repr(rtol)], capture_output=True, text=True, env=env,
                       timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-3000:]
    lines = r.stdout.strip().splitlines()
    n = cells.T.size
    out = np.array([[float(v) for v in ln.split()] for ln in lines[:n]])
    rhs = np.array([float(v) for v in lines[n].split()])
    J = np.array([float(v) for v in lines[n + 1].split()])
    return out, rhs, J


@pytest.mark.parametrize("mech", ["m9", "m53"])
def test_sanitized_oracle_matches_regular_build(driver, tmp_path, mech):
    if mech == "m9":
        path, cells, rtol = fields.M9_PATH, fields.c1_cells(6, seed=1001), 1e-8
        dt = cells.dt
    else:
        path, cells, rtol = fields.M53_PATH, fields.c4_cells(2, seed=1004), 1e-7
        dt = 1e-8
    out, rhs, J = _run(driver, tmp_path, path, cells, dt, rtol)
    o = Oracle(path)
    rho, e = o.state_from_TPY(cells.T, cells.p, cells.Y)
    T0 = np.array([o.T_from_e(e[i], cells.Y[:, i], cells.T[i] + 300.0) for i in range(rho.size)])
    y0 = np.concatenate([cells.Y[:, 0], [T0[0]]])
    assert np.allclose(rhs, o.rhs(rho[0], y0), rtol=1e-12, atol=0)
    assert np.allclose(J, o.jac(rho[0], y0).ravel(), rtol=1e-12, atol=0)
    Y1, T1, st = o.integrate(rho, e, cells.Y, dt, rtol, 1e-20, T=T0, max_steps=200000, nthreads=1)
    assert np.array_equal(out[:, 1].astype(int), st)
    assert np.allclose(out[:, 0], T1, rtol=1e-12, atol=0)
    assert np.allclose(out[:, 2:].T, Y1, rtol=1e-10, atol=1e-22)
