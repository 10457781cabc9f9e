"""Pins of the cost-model reference: finite differences, least squares and the
published form of Adam's first step."""
import numpy as np

from oracle import mlp
from paper_2007_01277_amd import inputs


def _params(d, seed, hidden=mlp.HIDDEN):
    g = inputs.rng(seed)
    parts = []
    for a, b in mlp.layer_shapes(d, hidden):
        lim = np.sqrt(6.0 / a)
        parts += [g.uniform(-lim, lim, a * b), g.uniform(-0.1, 0.1, b)]
    return np.concatenate(parts)


def test_layout_size():
    assert mlp.n_params(28) == 28 * 64 + 64 + 2 * (64 * 64 + 64) + 64 + 1


def test_gradient_matches_central_differences():
    d, n = 7, 23
    g = inputs.rng(1)
    X = g.standard_normal((n, d))
    y = g.standard_normal(n)
    p = _params(d, 2)
    _, gr = mlp.grad(p, X, y)
    h = 1e-6
    idx = inputs.rng(3).choice(p.size, 200, replace=False)
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (mlp.loss(p + e, X, y) - mlp.loss(p - e, X, y)) / (2 * h)
        assert abs(fd - gr[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, (i, fd, gr[i])


def test_linear_model_trained_with_adam_reaches_least_squares():
    # no hidden layer: yhat = X w + b; Adam on the MSE converges to lstsq
    d, n = 5, 200
    g = inputs.rng(4)
    X = g.standard_normal((n, d))
    y = X @ g.standard_normal(d) + 0.3 + 0.05 * g.standard_normal(n)
    p = np.zeros(mlp.n_params(d, ()))
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    for t in range(1, 6001):
        _, gr = mlp.grad(p, X, y, ())
        p, m, v = mlp.adam_step(p, gr, m, v, t, lr=0.01)
    A = np.hstack([X, np.ones((n, 1))])
    ref = np.linalg.lstsq(A, y, rcond=None)[0]
    np.testing.assert_allclose(p, ref, rtol=0, atol=1e-6)


def test_adam_first_step_is_lr_times_sign():
    # with zero moments, the bias-corrected first step is lr * g / (|g| + eps)
    p = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -4.0, 1e-3])
    p1, m, v = mlp.adam_step(p, g, np.zeros(3), np.zeros(3), 1, lr=0.1)
    np.testing.assert_allclose(p1, p - 0.1 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_relu_blocks_gradient():
    # a layer whose pre-activations are all negative passes no gradient below it
    d = 3
    p = _params(d, 5)
    layers = mlp.unpack(p, d)
    layers[0][1][:] = -1e3  # b_1 very negative: h_1 = 0
    X = inputs.rng(6).standard_normal((10, d))
    _, gr = mlp.grad(p, X, np.ones(10))
    assert np.all(gr[: d * 64 + 64] == 0.0)
