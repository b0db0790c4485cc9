"""Pins of the FP64 reference of the scheduler's cost model."""
import numpy as np
import pytest

from oracle import mlp


@pytest.mark.parametrize("F,H,O,n", [(8, 16, 1, 37), (3, 5, 1, 4), (1, 1, 1, 1), (10, 12, 2, 23), (2, 3, 4, 5)])
def test_gradient_matches_central_differences(F, H, O, n):
    rng = np.random.default_rng(F * 100 + H + 7 * O)
    p = mlp.init(F, H, seed=F + H, O=O) + rng.normal(0, 0.1, mlp.n_params(F, H, O))
    X = rng.normal(size=(n, F))
    t = rng.normal(size=(n, O))
    L, g = mlp.loss_grad(p, X, t, F, H, O)
    assert abs(L - mlp.loss(p, X, t, F, H, O)) <= 1e-15 * max(1.0, L)
    h = 1e-6
    fd = np.empty_like(p)
    for k in range(p.size):
        e = np.zeros_like(p)
        e[k] = h
        fd[k] = (mlp.loss(p + e, X, t, F, H, O) - mlp.loss(p - e, X, t, F, H, O)) / (2 * h)
    assert np.max(np.abs(fd - g)) <= 1e-7 * max(1.0, np.max(np.abs(g)))


def test_outputs_are_independent_heads():
    """Output o depends only on row o of W3 and on b3[o], and the loss is the sum of the
    per-output losses: a two-output model equals two one-output models sharing the hidden
    layers."""
    F, H, n = 5, 7, 11
    rng = np.random.default_rng(3)
    p2 = mlp.init(F, H, seed=4, O=2) + rng.normal(0, 0.1, mlp.n_params(F, H, 2))
    X = rng.normal(size=(n, F))
    t = rng.normal(size=(n, 2))
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p2, F, H, 2)
    shared = np.concatenate([W1.ravel(), b1, W2.ravel(), b2])
    heads = [np.concatenate([shared, W3[o], [b3[o]]]) for o in range(2)]
    y2, _, _ = mlp.forward(p2, X, F, H, 2)
    for o in range(2):
        y1, _, _ = mlp.forward(heads[o], X, F, H)
        assert np.allclose(y2[:, o], y1, rtol=0, atol=1e-15)
    L2 = mlp.loss(p2, X, t, F, H, 2)
    assert abs(L2 - sum(mlp.loss(heads[o], X, t[:, o], F, H) for o in range(2))) <= 1e-14 * L2


def test_linear_special_case():
    """With W1 = 0 and W2 = 0 the model is the constant w3.tanh(b2) + b3: the loss is a
    quadratic in b3 minimised at mean(t) - w3.tanh(b2)."""
    F, H = 4, 3
    p = np.zeros(mlp.n_params(F, H))
    W1, b1, W2, b2, w3, b3 = mlp.unpack(p, F, H)
    off_b2 = H * F + H + H * H
    p[off_b2:off_b2 + H] = [0.3, -0.2, 0.5]
    p[off_b2 + H:off_b2 + 2 * H] = [1.0, 2.0, -1.0]
    X = np.random.default_rng(0).normal(size=(10, F))
    t = np.arange(10.0)
    c = float(np.dot([1.0, 2.0, -1.0], np.tanh([0.3, -0.2, 0.5])))
    y, _, _ = mlp.forward(p, X, F, H)
    assert np.allclose(y, c)
    p[-1] = t.mean() - c
    L, g = mlp.loss_grad(p, X, t, F, H)
    assert abs(g[-1]) < 1e-12
    assert abs(L - np.var(t)) < 1e-12
