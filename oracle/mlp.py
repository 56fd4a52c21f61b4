"""Float64 reference of the schedule cost model -- TEST INFRASTRUCTURE ONLY.

The network is not in the paper; it only chooses which exact intersection
kernel runs a bucket of work, so it never changes a count.  Its definition:

    a1 = relu(W1 x + b1)        W1: [H, 3]
    a2 = relu(W2 a1 + b2)       W2: [H, H]
    y  = W3 a2 + b3             W3: [K, H]     (one predicted cost per candidate)

A training row is (x, c, t, w): features x, candidate index c, measured
target t, weight w >= 0 (1 when no weights are given).  The loss over a
batch is  sum_i w_i * 0.5 * (y_i[c_i] - t_i)^2 / sum_i w_i.
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


def _weights(w, B):
    return np.ones(B) if w is None else np.asarray(w, dtype=np.float64)


def loss(params, X, c, t, w=None):
    y, _ = forward(params, X)
    B = X.shape[0]
    w = _weights(w, B)
    r = y[np.arange(B), c] - t
    return 0.5 * float(np.sum(w * r * r) / np.sum(w))


def loss_and_grad(params, X, c, t, w=None):
    """Loss and gradients (same order as ``params``) by backpropagation."""
    W1, b1, W2, b2, W3, b3 = params
    y, (X, z1, a1, z2, a2) = forward(params, X)
    B = X.shape[0]
    w = _weights(w, B)
    r = y[np.arange(B), c] - t
    L = 0.5 * float(np.sum(w * r * r) / np.sum(w))
    dy = np.zeros_like(y)
    dy[np.arange(B), c] = w * r / np.sum(w)
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


# ---------------------------------------------------------------- initialisation

GOLDEN = 0x9E3779B97F4A7C15
_M64 = (1 << 64) - 1


def splitmix64_at(seed: int, index):
    """The (index + 1)-th output of SplitMix64 (Steele, Lea and Flood, 2014)
    started at ``seed``: mix(seed + (index + 1) * golden), in Python integers."""
    out = []
    for i in np.atleast_1d(np.asarray(index, dtype=np.uint64)).tolist():
        z = (seed + (int(i) + 1) * GOLDEN) & _M64
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
        out.append(z ^ (z >> 31))
    return np.array(out, dtype=np.uint64)


def init_he_uniform(K: int, H: int = H_DEFAULT, seed: int = 0):
    """The library's initialisation, in float32: weight at flat index i is
    (2u - 1) * float32(sqrt(6 / fan_in)) with u = (SplitMix64(seed, i) >> 40)
    * 2^-24; biases are zero."""
    flat = np.zeros(sum(int(np.prod(s)) for s in param_shapes(K, H)), dtype=np.float32)
    off = 0
    for shp in param_shapes(K, H):
        sz = int(np.prod(shp))
        if len(shp) == 2:
            idx = np.arange(off, off + sz, dtype=np.uint64)
            u = (splitmix64_at(seed, idx) >> np.uint64(40)).astype(np.float32) * np.float32(2.0 ** -24)
            d = np.float32(2.0) * u - np.float32(1.0)
            flat[off:off + sz] = d * np.float32(np.sqrt(6.0 / shp[1]))
        off += sz
    return flat


# ---------------------------------------------------------------- schedule

N_BUCKETS = 2048
STRAT_WAVE_HASH, STRAT_WG_HASH, STRAT_BSEARCH, STRAT_MERGE = 0, 1, 2, 3


def bucket_features(b):
    """(ob, pb, kind) of bucket b = (kind * 32 + ob) * 32 + pb."""
    b = np.asarray(b, dtype=np.int64)
    return np.stack([(b >> 5) & 31, b & 31, b >> 10], axis=1).astype(np.float64)


def schedule(params, wave_ob_max: int):
    """Per bucket: predicted costs (float64), the cheapest feasible strategy
    (ties to the lower number), and the gap to the runner-up.  The wavefront
    hash is feasible when ob <= wave_ob_max; the workgroup hash (which slices
    long owner lists), binary search and merge always are."""
    b = np.arange(N_BUCKETS)
    X = bucket_features(b)
    y, _ = forward(params, X)
    ob = X[:, 0]
    feas = np.ones((N_BUCKETS, 4), dtype=bool)
    feas[:, STRAT_WAVE_HASH] = ob <= wave_ob_max
    yy = np.where(feas, y[:, :4], np.inf)
    table = np.argmin(yy, axis=1)          # argmin returns the first (lowest) index on ties
    srt = np.sort(yy, axis=1)
    gap = srt[:, 1] - srt[:, 0]
    return table.astype(np.int32), y, gap, feas
