"""FP64 reference of the scheduler's model (test infrastructure only).

Two tanh hidden layers and O linear outputs, trained on the squared error:

    z1 = W1 x + b1,  h1 = tanh(z1)
    z2 = W2 h1 + b2, h2 = tanh(z2)
    y  = W3 h2 + b3,   loss = mean_i sum_o (y_io - t_io)^2

Parameters are one flat vector laid out W1[H][F], b1[H], W2[H][H], b2[H], W3[O][H], b3[O].
The gradient is back-propagation written out with plain numpy products; it is
pinned against central finite differences of ``loss`` in the CPU tests.
"""
from __future__ import annotations

import numpy as np


def n_params(F: int, H: int, O: int = 1) -> int:
    return H * F + H + H * H + H + O * H + O


def unpack(p, F, H, O=1):
    p = np.asarray(p, np.float64)
    assert p.shape == (n_params(F, H, O),)
    o = 0
    W1 = p[o:o + H * F].reshape(H, F); o += H * F
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    W3 = p[o:o + O * H].reshape(O, H); o += O * H
    b3 = p[o:o + O]
    return W1, b1, W2, b2, W3, b3


def forward(p, X, F, H, O=1):
    """(y [n, O], h1, h2); y is [n] when O = 1."""
    W1, b1, W2, b2, W3, b3 = unpack(p, F, H, O)
    X = np.asarray(X, np.float64).reshape(-1, F)
    h1 = np.tanh(X @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    y = h2 @ W3.T + b3
    return (y[:, 0] if O == 1 else y), h1, h2


def _residual(p, X, t, F, H, O):
    y, h1, h2 = forward(p, X, F, H, O)
    y = y.reshape(-1, O)
    return y - np.asarray(t, np.float64).reshape(-1, O), h1, h2


def loss(p, X, t, F, H, O=1):
    r, _, _ = _residual(p, X, t, F, H, O)
    return float(np.mean(np.sum(r * r, axis=1)))


def loss_grad(p, X, t, F, H, O=1):
    """(loss, d loss / d p) by the chain rule through the three layers."""
    W1, b1, W2, b2, W3, b3 = unpack(p, F, H, O)
    X = np.asarray(X, np.float64).reshape(-1, F)
    n = X.shape[0]
    r, h1, h2 = _residual(p, X, t, F, H, O)
    dy = 2.0 * r / n                          # d loss / d y_io
    g_b3 = dy.sum(axis=0)
    g_W3 = dy.T @ h2
    d2 = (dy @ W3) * (1.0 - h2 * h2)          # d loss / d z2
    g_W2 = d2.T @ h1
    g_b2 = d2.sum(axis=0)
    d1 = (d2 @ W2) * (1.0 - h1 * h1)          # d loss / d z1
    g_W1 = d1.T @ X
    g_b1 = d1.sum(axis=0)
    g = np.concatenate([g_W1.ravel(), g_b1, g_W2.ravel(), g_b2, g_W3.ravel(), g_b3])
    return float(np.mean(np.sum(r * r, axis=1))), g


def init(F, H, seed, O=1):
    """Seeded initial parameters (uniform, scaled by fan-in)."""
    rng = np.random.default_rng(seed)
    p = np.zeros(n_params(F, H, O))
    o = 0
    p[o:o + H * F] = rng.uniform(-1, 1, H * F) / np.sqrt(F); o += H * F + H
    p[o:o + H * H] = rng.uniform(-1, 1, H * H) / np.sqrt(H); o += H * H + H
    p[o:o + O * H] = rng.uniform(-1, 1, O * H) / np.sqrt(H)
    return p
