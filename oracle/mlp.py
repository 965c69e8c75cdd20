"""Oracle: FP64 reference of the per-column corrector network.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

A multilayer perceptron y = W4 g(W3 g(W2 g(W1 x + b1) + b2) + b3) + b4 with
g the Gauss error linear unit g(z) = z (1 + erf(z / sqrt 2)) / 2, and the
mean-squared loss over a batch, L = sum (y - t)^2 / (B n_out).  Backward by
the chain rule, layer by layer.  Weights are stored W[out, in] (row-major),
as the GPU kernels store them.
"""
import math

import numpy as np

_ERF = np.vectorize(math.erf, otypes=[np.float64])


def gelu(z):
    return 0.5 * z * (1.0 + _ERF(z / math.sqrt(2.0)))


def gelu_grad(z):
    cdf = 0.5 * (1.0 + _ERF(z / math.sqrt(2.0)))
    pdf = np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)
    return cdf + z * pdf


def forward(params, x):
    """params: list of (W, b); returns (y, cache of pre-activations)."""
    h = x
    zs, hs = [], [x]
    for i, (W, b) in enumerate(params):
        z = h @ W.T + b
        zs.append(z)
        h = gelu(z) if i + 1 < len(params) else z
        hs.append(h)
    return h, (zs, hs)


def loss(params, x, t):
    y, _ = forward(params, x)
    return float(np.sum((y - t) ** 2) / y.size)


def backward(params, x, t):
    """Gradients of the mean-squared loss: list of (dW, db)."""
    y, (zs, hs) = forward(params, x)
    dh = 2.0 * (y - t) / y.size
    grads = [None] * len(params)
    for i in range(len(params) - 1, -1, -1):
        dz = dh if i + 1 == len(params) else dh * gelu_grad(zs[i])
        W, _ = params[i]
        grads[i] = (dz.T @ hs[i], dz.sum(axis=0))
        dh = dz @ W
    return grads
