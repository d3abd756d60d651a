"""FP64 reference of the QED-rate surrogate network (test infrastructure only).

A 4 -> 64 -> 64 -> 2 perceptron with tanh hidden activations and a linear
output:  h1 = tanh(x W1 + b1),  h2 = tanh(h1 W2 + b2),  y = h2 W3 + b3.
Loss = sum over batch rows b and outputs o of w_o (y_bo - t_bo)^2 / (2 B) with
w = (RATE_WEIGHT, 1): output 0 is the rate, output 1 the sampled fraction.
Forward and backward are written out with plain matrix products in FP64
(the paper does not use a network; this is the surrogate of its Monte-Carlo
rates, Sec. IV Eqs. 23-24).  Weights are passed as given: when checking the
GPU kernels the caller passes the weights the GPU network holds (the sum of
its hi and lo BF16 terms, or the hi terms alone for its backward pass).
"""
from __future__ import annotations

import numpy as np

SIZES = (4, 64, 64, 2)
RATE_WEIGHT = 10.0
OUT_WEIGHT = np.array([RATE_WEIGHT, 1.0])


def init_params(rng: np.random.Generator):
    p = {}
    for li, (a, b) in enumerate(zip(SIZES[:-1], SIZES[1:]), start=1):
        p[f"W{li}"] = rng.standard_normal((a, b)) / np.sqrt(a)
        p[f"b{li}"] = np.zeros(b)
    return p


def forward(p, X):
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ p["W1"] + p["b1"]
    h1 = np.tanh(z1)
    z2 = h1 @ p["W2"] + p["b2"]
    h2 = np.tanh(z2)
    y = h2 @ p["W3"] + p["b3"]
    return y, (X, h1, h2)


def loss(p, X, T):
    y, _ = forward(p, X)
    return float(np.sum(OUT_WEIGHT * (y - T) ** 2) / (2.0 * len(X)))


def backward(p, X, T):
    """Gradients of `loss` with respect to every parameter (chain rule)."""
    y, (X, h1, h2) = forward(p, X)
    B = len(X)
    dy = OUT_WEIGHT * (y - T) / B
    g = {"W3": h2.T @ dy, "b3": dy.sum(0)}
    dh2 = dy @ p["W3"].T
    dz2 = dh2 * (1.0 - h2 ** 2)
    g["W2"] = h1.T @ dz2
    g["b2"] = dz2.sum(0)
    dh1 = dz2 @ p["W2"].T
    dz1 = dh1 * (1.0 - h1 ** 2)
    g["W1"] = X.T @ dz1
    g["b1"] = dz1.sum(0)
    return g
