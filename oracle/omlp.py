"""CPU FP64 reference of the chemistry surrogate network (test infrastructure
only: the test suite, the smoke check and the benchmark's CPU-baseline leg may
import it; the product library shares no code with it).

The network maps a reactor state and a timestep to the state increment over
that timestep (the learned-surrogate addition to the chemistry substep of
Sec. 2.1): a multilayer perceptron 12 -> 256 -> 256 -> 256 -> 10 with GELU
activations after the three hidden layers and a linear output layer.

Readings fixed here (the paper defines no surrogate):
  * GELU is the exact form z * Phi(z) = z/2 (1 + erf(z / sqrt 2)).
  * The loss is the mean squared error over the batch and the 10 outputs.
  * Adam with bias correction (first and second moments, step counted from 1).
  * Parameters are one flat vector: W1 [256][12], b1 [256], W2 [256][256],
    b2 [256], W3 [256][256], b3 [256], W4 [10][256], b4 [10]; W[out][in].
  * Features of a state (T, p, Y, dt): T [K], ln(p / 1 atm), ln max(Y_k, 1e-20)
    for the 9 species, ln dt; each then z-scored with the training mean/std.
  * Targets: asinh(dY_k / s_k) with s_k = 1e-4 |Y_k| + 1e-14 and
    asinh(dT / s_T) with s_T = 1e-4 T, then z-scored; asinh keeps small
    increments in relative terms and compresses large ones.

Everything is written out plainly in numpy float64.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

SIZES = (12, 256, 256, 256, 10)
ATM = 101325.0
Y_CLIP = 1e-20
S_REL, S_ABS_Y = 1e-4, 1e-14


def layout(sizes=SIZES):
    """[(W offset, (out, in), b offset, out)] per layer."""
    out, off = [], 0
    for a, b in zip(sizes[:-1], sizes[1:]):
        w = off
        off += a * b
        out.append((w, (b, a), off, b))
        off += b
    return out


def n_params(sizes=SIZES) -> int:
    w, (o, i), b, n = layout(sizes)[-1]
    return b + n


def unpack(params, sizes=SIZES):
    return [(params[w:w + o * i].reshape(o, i), params[b:b + n]) for w, (o, i), b, n in layout(sizes)]


def init_params(rng, sizes=SIZES):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases."""
    p = np.zeros(n_params(sizes))
    for w, (o, i), b, n in layout(sizes):
        lim = 1.0 / math.sqrt(i)
        p[w:w + o * i] = rng.uniform(-lim, lim, o * i)
        p[b:b + n] = rng.uniform(-lim, lim, n)
    return p


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_prime(z):
    """d/dz [z Phi(z)] = Phi(z) + z phi(z)."""
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def forward(params, X, sizes=SIZES):
    """X [batch][12] -> out [batch][10]; also the pre-activations and
    activations of every layer (for the backward pass)."""
    h = np.asarray(X, dtype=np.float64)
    hs, zs = [h], []
    layers = unpack(np.asarray(params, dtype=np.float64), sizes)
    for li, (W, b) in enumerate(layers):
        z = h @ W.T + b
        zs.append(z)
        h = gelu(z) if li < len(layers) - 1 else z
        hs.append(h)
    return h, (hs, zs)


def mse(out, T):
    d = out - T
    return float(np.mean(d * d))


def loss_and_grad(params, X, T, sizes=SIZES):
    """Mean squared error over batch and outputs, and its gradient with
    respect to the flat parameter vector (chain rule, layer by layer)."""
    out, (hs, zs) = forward(params, X, sizes)
    B, n_out = out.shape
    loss = mse(out, T)
    g = np.zeros(n_params(sizes))
    lay = layout(sizes)
    dz = 2.0 * (out - T) / (B * n_out)            # d loss / d z of the output layer
    layers = unpack(np.asarray(params, dtype=np.float64), sizes)
    for li in range(len(lay) - 1, -1, -1):
        w, (o, i), b, n = lay[li]
        g[w:w + o * i] = (dz.T @ hs[li]).reshape(-1)  # dW = dz^T h_in
        g[b:b + n] = dz.sum(axis=0)
        if li > 0:
            dh = dz @ layers[li][0]                 # d loss / d h_in
            dz = dh * gelu_prime(zs[li - 1])
    return loss, g


def adam_step(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counted from 1); returns new (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def features(T, p, Y, dt):
    """Raw (not yet standardised) features, [n][12]: T, ln(p/atm), ln max(Y,
    1e-20) for each species, ln dt.  Y is [9][n]."""
    T = np.asarray(T, dtype=np.float64)
    n = T.size
    X = np.empty((n, 12))
    X[:, 0] = T
    X[:, 1] = np.log(np.asarray(p, dtype=np.float64) / ATM)
    X[:, 2:11] = np.log(np.maximum(np.asarray(Y, dtype=np.float64), Y_CLIP)).T
    X[:, 11] = np.log(np.broadcast_to(np.asarray(dt, dtype=np.float64), (n,)))
    return X


def targets(Y0, T0, Y1, T1):
    """Raw (not yet standardised) targets, [n][10]."""
    Y0, Y1 = np.asarray(Y0, dtype=np.float64), np.asarray(Y1, dtype=np.float64)
    T0, T1 = np.asarray(T0, dtype=np.float64), np.asarray(T1, dtype=np.float64)
    sY = S_REL * np.abs(Y0) + S_ABS_Y
    sT = S_REL * T0
    out = np.empty((T0.size, 10))
    out[:, :9] = np.arcsinh((Y1 - Y0) / sY).T
    out[:, 9] = np.arcsinh((T1 - T0) / sT)
    return out


def decode(Y0, T0, raw_targets):
    """Inverse of targets(): increments (dY [9][n], dT [n]) from raw targets."""
    Y0, T0 = np.asarray(Y0, dtype=np.float64), np.asarray(T0, dtype=np.float64)
    sY = S_REL * np.abs(Y0) + S_ABS_Y
    dY = np.sinh(raw_targets[:, :9].T) * sY
    dT = np.sinh(raw_targets[:, 9]) * S_REL * T0
    return dY, dT
