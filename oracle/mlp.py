"""fp64 oracle of the cost-model MLP -- TEST INFRASTRUCTURE ONLY.

The paper derives configurations for unseen (computation, workload) pairs by
interpolating over past profiles (Sec. 3.2, "Configuration Derivation": radial
basis functions for 1-3 dimensions, Euclidean nearest neighbour above).  This
build replaces that interpolator with a small learned model; the oracle below
fixes what that model computes:

* network: 24 -> 64 -> 64 -> 1, ReLU after the two hidden layers, linear output;
* loss: mean squared error between the output and the target log-runtime;
* optimiser: Adam (lr 1e-3, beta1 0.9, beta2 0.999, eps 1e-8), bias-corrected.

Parameters are one flat fp64 vector in the order W1 [64, 24] (row-major,
[out, in]), b1 [64], W2 [64, 64], b2 [64], W3 [1, 64], b3 [1]: 5825 values.
A matmul is used as a library primitive; nothing is fused or reordered.
"""
from __future__ import annotations

import numpy as np

N_IN, N_H1, N_H2 = 24, 64, 64
SHAPES = [(N_H1, N_IN), (N_H1,), (N_H2, N_H1), (N_H2,), (1, N_H2), (1,)]
N_PARAMS = sum(int(np.prod(s)) for s in SHAPES)


def unpack(theta: np.ndarray):
    theta = np.asarray(theta, dtype=np.float64)
    out, off = [], 0
    for s in SHAPES:
        n = int(np.prod(s))
        out.append(theta[off:off + n].reshape(s))
        off += n
    assert off == theta.size == N_PARAMS
    return out


def forward(theta: np.ndarray, X: np.ndarray):
    """Returns (y [n], cache) for inputs X [n, 24]."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    y = (h2 @ W3.T + b3)[:, 0]
    return y, (X, z1, h1, z2, h2)


def loss(theta, X, t) -> float:
    y, _ = forward(theta, X)
    return float(np.mean((y - np.asarray(t, np.float64)) ** 2))


def loss_and_grad(theta, X, t):
    """Mean-squared-error loss and its gradient with respect to every parameter,
    by the chain rule through the three layers."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    y, (X, z1, h1, z2, h2) = forward(theta, X)
    n = X.shape[0]
    r = y - np.asarray(t, np.float64)
    L = float(np.mean(r ** 2))
    dy = (2.0 / n) * r                      # dL/dy           [n]
    gW3 = dy[None, :] @ h2                  # [1, 64]
    gb3 = np.array([dy.sum()])
    dh2 = dy[:, None] @ W3                  # [n, 64]
    dz2 = dh2 * (z2 > 0)
    gW2 = dz2.T @ h1                        # [64, 64]
    gb2 = dz2.sum(axis=0)
    dh1 = dz2 @ W2                          # [n, 64]
    dz1 = dh1 * (z1 > 0)
    gW1 = dz1.T @ X                         # [64, 24]
    gb1 = dz1.sum(axis=0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return L, g


def adam_step(theta, g, m, v, step: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    theta = theta - lr * mhat / (np.sqrt(vhat) + eps)
    return theta, m, v


def train(theta, X, t, epochs: int, batch: int, perms, lr=1e-3):
    """Mini-batch Adam; ``perms[e]`` is the sample order of epoch e (drawn by the
    caller).  Returns (theta, per-epoch mean loss)."""
    theta = np.array(theta, np.float64)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    step = 0
    hist = []
    n = X.shape[0]
    for e in range(epochs):
        tot = 0.0
        for s in range(0, n, batch):
            idx = perms[e][s:s + batch]
            L, g = loss_and_grad(theta, X[idx], t[idx])
            step += 1
            theta, m, v = adam_step(theta, g, m, v, step, lr=lr)
            tot += L * len(idx)
        hist.append(tot / n)
    return theta, hist
