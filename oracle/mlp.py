"""Float64 reference of the schedule cost model -- TEST INFRASTRUCTURE ONLY.

The network is not in the paper; it only chooses which exact intersection
kernel runs a bucket of work, so it never changes a count.  Its definition:

    a1 = relu(W1 x + b1)        W1: [H, 3]
    a2 = relu(W2 a1 + b2)       W2: [H, H]
    y  = W3 a2 + b3             W3: [K, H]     (one predicted cost per candidate)

A training row is (x, c, t): features x, candidate index c, measured target t.
The loss over a batch of B rows is  (1/B) * sum_i 0.5 * (y_i[c_i] - t_i)^2.
The optimiser is Adam (Kingma and Ba, 2015) with bias correction.
Parameters are stored row-major as float arrays in the order
W1, b1, W2, b2, W3, b3.
"""
from __future__ import annotations

import numpy as np

H_DEFAULT = 32
IN_DIM = 3


def param_shapes(K: int, H: int = H_DEFAULT):
    return [(H, IN_DIM), (H,), (H, H), (H,), (K, H), (K,)]


def init_params(K: int, H: int = H_DEFAULT, seed: int = 0):
    """He-style init from numpy's PCG64 (only used by the tests' float64 path)."""
    rng = np.random.default_rng(seed)
    ps = []
    for shp in param_shapes(K, H):
        if len(shp) == 2:
            ps.append(rng.standard_normal(shp) * np.sqrt(2.0 / shp[1]))
        else:
            ps.append(np.zeros(shp))
    return ps


def forward(params, X):
    """Returns y [B, K] and the cache needed by :func:`backward`."""
    W1, b1, W2, b2, W3, b3 = params
    z1 = X @ W1.T + b1
    a1 = np.maximum(z1, 0.0)
    z2 = a1 @ W2.T + b2
    a2 = np.maximum(z2, 0.0)
    y = a2 @ W3.T + b3
    return y, (X, z1, a1, z2, a2)


def loss(params, X, c, t):
    y, _ = forward(params, X)
    B = X.shape[0]
    r = y[np.arange(B), c] - t
    return 0.5 * float(np.mean(r * r))


def loss_and_grad(params, X, c, t):
    """Loss and gradients (same order as ``params``) by backpropagation."""
    W1, b1, W2, b2, W3, b3 = params
    y, (X, z1, a1, z2, a2) = forward(params, X)
    B = X.shape[0]
    r = y[np.arange(B), c] - t
    L = 0.5 * float(np.mean(r * r))
    dy = np.zeros_like(y)
    dy[np.arange(B), c] = r / B
    gW3 = dy.T @ a2
    gb3 = dy.sum(axis=0)
    da2 = dy @ W3
    dz2 = da2 * (z2 > 0)
    gW2 = dz2.T @ a1
    gb2 = dz2.sum(axis=0)
    da1 = dz2 @ W2
    dz1 = da1 * (z1 > 0)
    gW1 = dz1.T @ X
    gb1 = dz1.sum(axis=0)
    return L, [gW1, gb1, gW2, gb2, gW3, gb3]


def adam_step(params, grads, m_state, v_state, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update in place; ``step`` counts from 1."""
    for p, g, m, v in zip(params, grads, m_state, v_state):
        m *= beta1
        m += (1.0 - beta1) * g
        v *= beta2
        v += (1.0 - beta2) * g * g
        mhat = m / (1.0 - beta1 ** step)
        vhat = v / (1.0 - beta2 ** step)
        p -= lr * mhat / (np.sqrt(vhat) + eps)


def flatten(params) -> np.ndarray:
    return np.concatenate([p.ravel() for p in params])


def unflatten(flat, K: int, H: int = H_DEFAULT):
    out, off = [], 0
    for shp in param_shapes(K, H):
        sz = int(np.prod(shp))
        out.append(np.asarray(flat[off:off + sz], dtype=np.float64).reshape(shp))
        off += sz
    return out
