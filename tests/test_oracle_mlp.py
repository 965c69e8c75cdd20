"""Pins of the FP64 reference MLP: gradients against central finite
differences, GELU against its closed form and special values."""
import math

import numpy as np

from oracle import mlp


def _params(rs, sizes):
    return [(rs.normal(size=(o, i)) / math.sqrt(i), rs.normal(size=o) * 0.1)
            for i, o in zip(sizes[:-1], sizes[1:])]


def test_gelu_values():
    z = np.array([-3.0, -1.0, 0.0, 0.5, 2.0])
    ref = [0.5 * v * (1 + math.erf(v / math.sqrt(2))) for v in z]
    assert np.allclose(mlp.gelu(z), ref, rtol=0, atol=1e-15)
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    # derivative by central differences
    h = 1e-6
    num = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    assert np.allclose(mlp.gelu_grad(z), num, rtol=1e-8, atol=1e-9)


def test_backward_matches_finite_differences():
    rs = np.random.default_rng(0)
    sizes = [12, 8, 8, 8, 5]
    params = _params(rs, sizes)
    x = rs.normal(size=(7, 12))
    t = rs.normal(size=(7, 5))
    grads = mlp.backward(params, x, t)
    h = 1e-6
    for li, (W, b) in enumerate(params):
        for arr, g in ((W, grads[li][0]), (b, grads[li][1])):
            flat = arr.reshape(-1)
            gflat = g.reshape(-1)
            for idx in rs.choice(flat.size, size=min(6, flat.size), replace=False):
                old = flat[idx]
                flat[idx] = old + h
                lp = mlp.loss(params, x, t)
                flat[idx] = old - h
                lm = mlp.loss(params, x, t)
                flat[idx] = old
                num = (lp - lm) / (2 * h)
                assert abs(num - gflat[idx]) <= 1e-7 * max(1.0, abs(num)), (li, idx, num, gflat[idx])


def test_linear_network_reduces_to_least_squares_gradient():
    """With one layer the gradient is the textbook 2 (XW^T + b - T)^T X / (B n)."""
    rs = np.random.default_rng(1)
    W, b = rs.normal(size=(3, 4)), rs.normal(size=3)
    x, t = rs.normal(size=(5, 4)), rs.normal(size=(5, 3))
    (dW, db), = mlp.backward([(W, b)], x, t)
    r = x @ W.T + b - t
    assert np.allclose(dW, 2 * r.T @ x / r.size, rtol=1e-14, atol=1e-15)
    assert np.allclose(db, 2 * r.sum(0) / r.size, rtol=1e-14, atol=1e-15)
