"""FP64 reference of the scheduler's cost model (test infrastructure only).

Two tanh hidden layers and a linear output, trained on the mean squared error:

    z1 = W1 x + b1,  h1 = tanh(z1)
    z2 = W2 h1 + b2, h2 = tanh(z2)
    y  = w3 . h2 + b3,   loss = mean_i (y_i - t_i)^2

Parameters are one flat vector laid out W1[H][F], b1[H], W2[H][H], b2[H], w3[H], b3.
The gradient is back-propagation written out with plain numpy products; it is
pinned against central finite differences of ``loss`` in the CPU tests.
"""
from __future__ import annotations

import numpy as np


def n_params(F: int, H: int) -> int:
    return H * F + H + H * H + H + H + 1


def unpack(p, F, H):
    p = np.asarray(p, np.float64)
    assert p.shape == (n_params(F, H),)
    o = 0
    W1 = p[o:o + H * F].reshape(H, F); o += H * F
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    w3 = p[o:o + H]; o += H
    b3 = p[o]
    return W1, b1, W2, b2, w3, b3


def forward(p, X, F, H):
    W1, b1, W2, b2, w3, b3 = unpack(p, F, H)
    X = np.asarray(X, np.float64).reshape(-1, F)
    h1 = np.tanh(X @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    return h2 @ w3 + b3, h1, h2


def loss(p, X, t, F, H):
    y, _, _ = forward(p, X, F, H)
    r = y - np.asarray(t, np.float64)
    return float(np.mean(r * r))


def loss_grad(p, X, t, F, H):
    """(loss, d loss / d p) by the chain rule through the three layers."""
    W1, b1, W2, b2, w3, b3 = unpack(p, F, H)
    X = np.asarray(X, np.float64).reshape(-1, F)
    n = X.shape[0]
    y, h1, h2 = forward(p, X, F, H)
    r = y - np.asarray(t, np.float64)
    dy = 2.0 * r / n                       # d loss / d y_i
    g_b3 = dy.sum()
    g_w3 = h2.T @ dy
    d2 = np.outer(dy, w3) * (1.0 - h2 * h2)  # d loss / d z2
    g_W2 = d2.T @ h1
    g_b2 = d2.sum(axis=0)
    d1 = (d2 @ W2) * (1.0 - h1 * h1)         # d loss / d z1
    g_W1 = d1.T @ X
    g_b1 = d1.sum(axis=0)
    g = np.concatenate([g_W1.ravel(), g_b1, g_W2.ravel(), g_b2, g_w3, [g_b3]])
    return float(np.mean(r * r)), g


def init(F, H, seed):
    """Seeded initial parameters (uniform, scaled by fan-in)."""
    rng = np.random.default_rng(seed)
    p = np.zeros(n_params(F, H))
    W1, b1, W2, b2, w3, b3 = unpack(p, F, H)
    o = 0
    p[o:o + H * F] = rng.uniform(-1, 1, H * F) / np.sqrt(F); o += H * F + H
    p[o:o + H * H] = rng.uniform(-1, 1, H * H) / np.sqrt(H); o += H * H + H
    p[o:o + H] = rng.uniform(-1, 1, H) / np.sqrt(H)
    return p
