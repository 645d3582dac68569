"""FP64 reference for the small mu / expansion-order predictor network.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The network is a plain multilayer perceptron: L affine layers with tanh
between them and a linear output,
    h_0 = x,  h_j = tanh(W_j h_{j-1} + b_j) (j < L),  y = W_L h_{L-1} + b_L,
trained on the mean squared error  loss = mean((y - t)^2)  with Adam
(Kingma & Ba 2015: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
w -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)).

Weights are stored as W_j with shape (out, in), activations row-major
(batch, features).  Gradients are written out by the chain rule below; the
tests pin them with central finite differences.
"""
from __future__ import annotations

import numpy as np

__all__ = ["init_params", "forward", "loss", "backward", "adam_step"]


def init_params(sizes, seed=0):
    """Uniform(-1/sqrt(in), 1/sqrt(in)) weights and zero biases, FP64."""
    rng = np.random.default_rng(seed)
    params = []
    for i in range(len(sizes) - 1):
        lim = 1.0 / np.sqrt(sizes[i])
        W = rng.uniform(-lim, lim, size=(sizes[i + 1], sizes[i]))
        b = np.zeros(sizes[i + 1])
        params.append((W, b))
    return params


def forward(params, x):
    """Returns (y, hs) with hs the list of layer inputs h_0 .. h_{L-1}."""
    hs = [np.asarray(x, dtype=np.float64)]
    h = hs[0]
    for j, (W, b) in enumerate(params):
        z = h @ W.T + b
        if j < len(params) - 1:
            h = np.tanh(z)
            hs.append(h)
        else:
            h = z
    return h, hs


def loss(params, x, t):
    y, _ = forward(params, x)
    return float(np.mean((y - t) ** 2))


def backward(params, x, t):
    """Gradients [(dW_j, db_j)] of the mean squared error loss."""
    y, hs = forward(params, x)
    n = y.size
    g = 2.0 * (y - t) / n  # d loss / d y
    grads = [None] * len(params)
    for j in range(len(params) - 1, -1, -1):
        W, _ = params[j]
        h_in = hs[j]
        grads[j] = (g.T @ h_in, g.sum(axis=0))
        if j > 0:
            g = (g @ W) * (1.0 - h_in ** 2)  # h_in = tanh(z_{j-1})
    return grads


def adam_step(params, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update in place; state = dict(t=int, m=[...], v=[...])."""
    if not state:
        state["t"] = 0
        state["m"] = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
        state["v"] = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
    state["t"] += 1
    t = state["t"]
    new = []
    for j, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
        out = []
        for k, (w, gw) in enumerate(((W, gW), (b, gb))):
            m = state["m"][j][k]
            v = state["v"][j][k]
            m[...] = b1 * m + (1.0 - b1) * gw
            v[...] = b2 * v + (1.0 - b2) * gw * gw
            mh = m / (1.0 - b1 ** t)
            vh = v / (1.0 - b2 ** t)
            out.append(w - lr * mh / (np.sqrt(vh) + eps))
        new.append(tuple(out))
    return new
