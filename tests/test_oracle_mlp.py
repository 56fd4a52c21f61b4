"""Pins of the float64 scheduler-network reference: central finite
differences for every parameter, a hand-checked tiny case, and Adam's
first step (whose size is lr * sign(g) by construction of the method)."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import mlp


def batch(K, B=17, seed=0):
    rng = np.random.default_rng(seed)
    X = np.column_stack([rng.uniform(0, 16, B), rng.uniform(0, 16, B), rng.integers(0, 2, B)])
    c = rng.integers(0, K, B)
    t = rng.normal(0, 3, B)
    return X, c, t


@pytest.mark.parametrize("K,H,weighted", [(4, 8, False), (6, 32, False), (4, 8, True)])
def test_gradients_match_finite_differences(K, H, weighted):
    params = mlp.init_params(K, H, seed=K)
    X, c, t = batch(K)
    w = np.random.default_rng(5).uniform(0, 2, len(t)) if weighted else None
    _, grads = mlp.loss_and_grad(params, X, c, t, w)
    h = 1e-6
    for p, g in zip(params, grads):
        flat, gflat = p.reshape(-1), g.reshape(-1)
        for i in range(0, flat.size, max(1, flat.size // 40)):
            old = flat[i]
            flat[i] = old + h
            lp = mlp.loss(params, X, c, t, w)
            flat[i] = old - h
            lm = mlp.loss(params, X, c, t, w)
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - gflat[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, gflat[i])


def test_tiny_forward_by_hand():
    # H = 1, K = 2: y = W3 * relu(W2 * relu(W1 x + b1) + b2) + b3
    params = [np.array([[1.0, -2.0, 0.5]]), np.array([0.25]), np.array([[3.0]]), np.array([-1.0]),
              np.array([[2.0], [-1.0]]), np.array([0.5, 1.0])]
    X = np.array([[2.0, 0.5, 1.0], [0.0, 1.0, 0.0]])
    y, _ = mlp.forward(params, X)
    # row 0: z1 = 2 - 1 + 0.5 + 0.25 = 1.75; z2 = 5.25 - 1 = 4.25 -> y = (9.0, -3.25)
    # row 1: z1 = -2 + 0.25 < 0 -> a1 = 0; z2 = -1 -> a2 = 0 -> y = b3
    assert np.allclose(y, [[9.0, -3.25], [0.5, 1.0]])
    L = mlp.loss(params, X, np.array([0, 1]), np.array([8.0, 2.0]))
    assert np.isclose(L, 0.5 * (1.0 + 1.0) / 2)


def test_adam_first_step_is_lr_times_sign():
    params = mlp.init_params(3, 8, seed=1)
    X, c, t = batch(3)
    _, grads = mlp.loss_and_grad(params, X, c, t)
    before = [p.copy() for p in params]
    ms = [np.zeros_like(p) for p in params]
    vs = [np.zeros_like(p) for p in params]
    mlp.adam_step(params, grads, ms, vs, step=1, lr=0.01, eps=1e-300)
    for b, a, g in zip(before, params, grads):
        nz = g != 0
        assert np.allclose((b - a)[nz], 0.01 * np.sign(g[nz]))
        assert np.array_equal(a[~nz], b[~nz])


def test_weights_scale_free_and_equal_to_duplicated_rows():
    params = mlp.init_params(4, 8, seed=2)
    X, c, t = batch(4, B=9)
    L1, g1 = mlp.loss_and_grad(params, X, c, t)
    L2, g2 = mlp.loss_and_grad(params, X, c, t, np.full(9, 3.5))        # a constant weight changes nothing
    assert np.isclose(L1, L2) and all(np.allclose(a, b) for a, b in zip(g1, g2))
    w = np.array([2, 1, 1, 1, 1, 1, 1, 1, 0], dtype=np.float64)          # weight 2 = the row twice, 0 = dropped
    Lw, gw = mlp.loss_and_grad(params, X, c, t, w)
    idx = [0, 0, 1, 2, 3, 4, 5, 6, 7]
    Ld, gd = mlp.loss_and_grad(params, X[idx], c[idx], t[idx])
    assert np.isclose(Lw, Ld) and all(np.allclose(a, b) for a, b in zip(gw, gd))
