"""Pins for the FP64 network reference: analytic gradients against central
finite differences, and Adam's first step against its closed form."""
import numpy as np

from oracle import mlp_oracle as M


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    sizes = [7, 16, 16, 16, 2]
    params = M.init_params(sizes, seed=1)
    x = rng.normal(size=(5, 7))
    t = rng.normal(size=(5, 2))
    grads = M.backward(params, x, t)
    h = 1e-6
    for j, (W, b) in enumerate(params):
        for arr, g in ((W, grads[j][0]), (b, grads[j][1])):
            flat = arr.reshape(-1)
            gflat = g.reshape(-1)
            for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
                old = flat[idx]
                flat[idx] = old + h
                lp = M.loss(params, x, t)
                flat[idx] = old - h
                lm = M.loss(params, x, t)
                flat[idx] = old
                fd = (lp - lm) / (2 * h)
                assert abs(fd - gflat[idx]) <= 1e-7 * max(1.0, abs(fd))


def test_adam_first_step_closed_form():
    # after one step m_hat = g, v_hat = g^2: w -= lr * g / (|g| + eps)
    params = [(np.array([[1.0, -2.0]]), np.array([0.5]))]
    grads = [(np.array([[0.3, -4.0]]), np.array([1e-3]))]
    state = {}
    new = M.adam_step(params, grads, state, lr=0.01)
    assert np.allclose(new[0][0], [[1.0 - 0.01 * 0.3 / (0.3 + 1e-8), -2.0 + 0.01 * 4.0 / (4.0 + 1e-8)]])
    assert np.allclose(new[0][1], [0.5 - 0.01 * 1e-3 / (1e-3 + 1e-8)])
    assert state["t"] == 1


def test_training_reduces_loss():
    rng = np.random.default_rng(3)
    x = rng.normal(size=(64, 4))
    t = np.stack([np.sin(x[:, 0]) + 0.5 * x[:, 1], x[:, 2] * x[:, 3]], axis=1)
    params = M.init_params([4, 32, 32, 2], seed=0)
    state = {}
    l0 = M.loss(params, x, t)
    for _ in range(300):
        params = M.adam_step(params, M.backward(params, x, t), state, lr=3e-3)
    assert M.loss(params, x, t) < 0.2 * l0
