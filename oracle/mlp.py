"""Reference maths of the learned cost model -- TEST INFRASTRUCTURE ONLY.

The tuner's cost model is a multilayer perceptron with three hidden layers of
64 ReLU units and one linear output, trained with Adam on the mean squared
error.  The paper has no learned component; this is the reading of "MLP 3x64":

  h_1 = relu(x W_1 + b_1), h_2 = relu(h_1 W_2 + b_2), h_3 = relu(h_2 W_3 + b_3),
  yhat = h_3 W_4 + b_4,   L = (1/n) sum_i (yhat_i - y_i)^2,
  Adam (Kingma & Ba, 2015): m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
  p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).

Parameters are one flat float vector laid out as W_1[d][64], b_1[64],
W_2[64][64], b_2[64], W_3[64][64], b_3[64], W_4[64][1], b_4[1] (row-major,
W[in][out]).  Everything here is float64 numpy; the layer list is generic so the
tests can also check a single linear layer against least squares.
"""
from __future__ import annotations

import numpy as np

HIDDEN = (64, 64, 64)


def layer_shapes(d_in: int, hidden=HIDDEN):
    dims = [d_in] + list(hidden) + [1]
    return [(dims[i], dims[i + 1]) for i in range(len(dims) - 1)]


def n_params(d_in: int, hidden=HIDDEN) -> int:
    return sum(a * b + b for a, b in layer_shapes(d_in, hidden))


def unpack(p: np.ndarray, d_in: int, hidden=HIDDEN):
    out, o = [], 0
    for a, b in layer_shapes(d_in, hidden):
        W = p[o:o + a * b].reshape(a, b)
        o += a * b
        bias = p[o:o + b]
        o += b
        out.append((W, bias))
    assert o == p.size
    return out


def forward(p, X, hidden=HIDDEN):
    """Returns (yhat[n], activations) with activations[0] = X and the
    pre-activations of every layer, for the backward pass."""
    X = np.asarray(X, np.float64)
    layers = unpack(np.asarray(p, np.float64), X.shape[1], hidden)
    acts, pres = [X], []
    h = X
    for li, (W, b) in enumerate(layers):
        z = h @ W + b
        pres.append(z)
        h = np.maximum(z, 0.0) if li < len(layers) - 1 else z
        acts.append(h)
    return h[:, 0], (acts, pres)


def loss(p, X, y, hidden=HIDDEN) -> float:
    yhat, _ = forward(p, X, hidden)
    return float(np.mean((yhat - np.asarray(y, np.float64)) ** 2))


def grad(p, X, y, hidden=HIDDEN):
    """(loss, gradient) by the chain rule, layer by layer from the output."""
    yhat, (acts, pres) = forward(p, X, hidden)
    y = np.asarray(y, np.float64)
    n = y.size
    layers = unpack(np.asarray(p, np.float64), acts[0].shape[1], hidden)
    dz = (2.0 / n) * (yhat - y)[:, None]  # dL/dz of the output layer
    grads = [None] * len(layers)
    for li in reversed(range(len(layers))):
        W, _ = layers[li]
        grads[li] = (acts[li].T @ dz, dz.sum(axis=0))
        if li > 0:
            dz = (dz @ W.T) * (pres[li - 1] > 0.0)
    g = np.concatenate([np.concatenate([gw.ravel(), gb]) for gw, gb in grads])
    return float(np.mean((yhat - y) ** 2)), g


def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update at step t >= 1; returns new (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
