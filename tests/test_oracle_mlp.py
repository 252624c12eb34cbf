"""Pins of the CPU FP64 surrogate network: GELU against normal-CDF values,
derivatives against finite differences, the backward pass against finite
differences of the loss, closed forms of degenerate networks, one Adam step
in closed form, and the feature/target transforms against their inverses."""
import math

import numpy as np
import pytest

from oracle import omlp

SMALL = (5, 7, 6, 4, 3)


def test_parameter_count():
    # 12*256 + 256 + 2 (256*256 + 256) + 256*10 + 10
    assert omlp.n_params() == 137482
    lay = omlp.layout()
    assert lay[0][0] == 0 and lay[0][1] == (256, 12) and lay[-1][1] == (10, 256)


def test_gelu_normal_cdf_values():
    # z Phi(z) with tabulated standard normal CDF values
    for z, Phi in ((1.0, 0.8413447460685429), (-1.0, 0.15865525393145707),
                   (2.0, 0.9772498680518208), (-0.5, 0.3085375387259869)):
        assert omlp.gelu(np.array(z)) == pytest.approx(z * Phi, rel=1e-14, abs=1e-16)
    assert omlp.gelu(np.array(0.0)) == 0.0
    # far tails: identity and zero
    assert omlp.gelu(np.array(40.0)) == 40.0
    assert abs(omlp.gelu(np.array(-40.0))) < 1e-300


def test_gelu_prime_vs_finite_differences():
    z = np.linspace(-6, 6, 97)
    h = 1e-3
    # Richardson-extrapolated central difference, O(h^4)
    d1 = (omlp.gelu(z + h) - omlp.gelu(z - h)) / (2 * h)
    d2 = (omlp.gelu(z + h / 2) - omlp.gelu(z - h / 2)) / h
    fd = (4 * d2 - d1) / 3
    assert np.max(np.abs(omlp.gelu_prime(z) - fd)) < 1e-11
    assert omlp.gelu_prime(np.array(0.0)) == 0.5


def test_backward_vs_finite_differences():
    rng = np.random.default_rng(3)
    p = omlp.init_params(rng, SMALL)
    X = rng.normal(size=(11, SMALL[0]))
    T = rng.normal(size=(11, SMALL[-1]))
    loss, g = omlp.loss_and_grad(p, X, T, SMALL)
    assert loss == pytest.approx(omlp.mse(omlp.forward(p, X, SMALL)[0], T))
    h = 1e-5
    for j in range(p.size):
        e = np.zeros_like(p)
        e[j] = h
        fd = (omlp.loss_and_grad(p + e, X, T, SMALL)[0] - omlp.loss_and_grad(p - e, X, T, SMALL)[0]) / (2 * h)
        assert g[j] == pytest.approx(fd, rel=1e-6, abs=1e-10), j


def test_constant_network_closed_form():
    # all weights zero: the output is b4 for every input, and the gradient of
    # the mean squared error is 2 (b4 - mean T) / n_out on b4, zero on W4
    rng = np.random.default_rng(4)
    p = np.zeros(omlp.n_params(SMALL))
    w4, (o, i), b4, n = omlp.layout(SMALL)[-1]
    p[b4:b4 + n] = rng.normal(size=n)
    X = rng.normal(size=(9, SMALL[0]))
    T = rng.normal(size=(9, SMALL[-1]))
    out, _ = omlp.forward(p, X, SMALL)
    assert np.array_equal(out, np.broadcast_to(p[b4:b4 + n], out.shape))
    loss, g = omlp.loss_and_grad(p, X, T, SMALL)
    assert np.allclose(g[b4:b4 + n], 2 * (p[b4:b4 + n] - T.mean(axis=0)) / n, rtol=1e-14, atol=1e-15)
    assert np.all(g[w4:w4 + o * i] == 0.0)          # hidden activations gelu(0) = 0


def test_adam_first_step_is_signed_lr():
    # from zero moments the bias-corrected first step is lr * g / (|g| + eps)
    rng = np.random.default_rng(5)
    g = rng.normal(size=50)
    p = rng.normal(size=50)
    p1, m, v = omlp.adam_step(p, g, np.zeros(50), np.zeros(50), 1, 1e-3)
    assert np.allclose(p - p1, 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_features_and_target_transform():
    rng = np.random.default_rng(6)
    n = 20
    T = rng.uniform(300, 3000, n)
    p = rng.uniform(0.5, 40, n) * omlp.ATM
    Y = rng.dirichlet(np.ones(9), n).T
    Y[3, :5] = 0.0
    X = omlp.features(T, p, Y, 5e-9)
    assert np.allclose(X[:, 1], np.log(p / 101325.0))
    assert np.all(X[:5, 5] == math.log(1e-20))
    assert np.all(X[:, 11] == math.log(5e-9))
    Y1 = Y + rng.normal(size=Y.shape) * 1e-5
    T1 = T + rng.normal(size=n)
    raw = omlp.targets(Y, T, Y1, T1)
    dY, dT = omlp.decode(Y, T, raw)
    assert np.allclose(dY, Y1 - Y, rtol=1e-12, atol=1e-22)
    assert np.allclose(dT, T1 - T, rtol=1e-12, atol=1e-12)
    # small increments stay linear: asinh(x) ~ x
    small = omlp.targets(Y, T, Y + 1e-9 * (1e-4 * Y + 1e-14), T)
    assert np.allclose(small[:, :9], 1e-9, rtol=1e-6)
