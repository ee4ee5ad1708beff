"""Per-block damping network (test infrastructure only).

The paper damps every additive Schwarz block with one global factor (the
damping discussion after eq:applyCS); per-block weights are an extension.
Their network is a plain multilayer perceptron

    h1 = relu(W1 x + b1),  h2 = relu(W2 h1 + b2),  o = w3 . h2 + b3,
    omega_j = gamma * exp(clip(o_j, -OCLIP, OCLIP)),

with 16 inputs (block features), two hidden layers of 64 units and one
output, 5313 parameters stored flat in the order W1 (64 x 16, row-major),
b1, W2 (64 x 64, row-major), b2, w3, b3.  Training regresses o on
t = log(omega* / gamma) with the mean squared error and Adam.

Everything here is FP64 NumPy written from these definitions.
"""
from __future__ import annotations

import numpy as np

NFEAT = 16
HIDDEN = 64
NPARAM = NFEAT * HIDDEN + HIDDEN + HIDDEN * HIDDEN + HIDDEN + HIDDEN + 1  # 5313
OCLIP = 3.0


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.shape == (NPARAM,)
    k = 0

    def take(n, shape):
        nonlocal k
        out = theta[k:k + n].reshape(shape)
        k += n
        return out

    W1 = take(NFEAT * HIDDEN, (HIDDEN, NFEAT))
    b1 = take(HIDDEN, (HIDDEN,))
    W2 = take(HIDDEN * HIDDEN, (HIDDEN, HIDDEN))
    b2 = take(HIDDEN, (HIDDEN,))
    w3 = take(HIDDEN, (HIDDEN,))
    b3 = take(1, (1,))
    return W1, b1, W2, b2, w3, b3


def pack(W1, b1, W2, b2, w3, b3):
    return np.concatenate([np.ravel(W1), np.ravel(b1), np.ravel(W2), np.ravel(b2), np.ravel(w3), np.ravel(b3)])


def init(rng):
    """He-scaled normal weights, zero biases (draws passed in through rng)."""
    W1 = rng.standard_normal((HIDDEN, NFEAT)) * np.sqrt(2.0 / NFEAT)
    W2 = rng.standard_normal((HIDDEN, HIDDEN)) * np.sqrt(2.0 / HIDDEN)
    w3 = rng.standard_normal(HIDDEN) * np.sqrt(1.0 / HIDDEN)
    return pack(W1, np.zeros(HIDDEN), W2, np.zeros(HIDDEN), w3, np.zeros(1))


def forward(theta, X):
    """Network output o (before the clip) for every row of X (n x 16)."""
    W1, b1, W2, b2, w3, b3 = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    a1 = X @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    return h2 @ w3 + b3[0]


def weights(theta, X, gamma):
    return gamma * np.exp(np.clip(forward(theta, X), -OCLIP, OCLIP))


def loss_and_grad(theta, X, t):
    """L = mean((o - t)^2) and dL/dtheta by backpropagation."""
    W1, b1, W2, b2, w3, b3 = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    n = X.shape[0]
    a1 = X @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    o = h2 @ w3 + b3[0]
    e = o - t
    L = float(np.mean(e * e))
    do = 2.0 * e / n                       # dL/do
    gw3 = h2.T @ do
    gb3 = np.array([do.sum()])
    dh2 = np.outer(do, w3)
    da2 = dh2 * (a2 > 0.0)
    gW2 = da2.T @ h1
    gb2 = da2.sum(axis=0)
    dh1 = da2 @ W2
    da1 = dh1 * (a1 > 0.0)
    gW1 = da1.T @ X
    gb1 = da1.sum(axis=0)
    return L, pack(gW1, gb1, gW2, gb2, gw3, gb3)


def adam_step(theta, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba) with bias correction; step counts from 1."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
