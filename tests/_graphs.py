"""Small graph fixtures for the tests, built with numpy alone (no oracle, no
GPU library), so that they can pin both."""
from __future__ import annotations

import itertools
import math

import numpy as np

import oracle


def csr_from_edges(n, edges) -> oracle.CSR:
    """Simple undirected CSR by numpy: drop loops, symmetrise, unique, sort."""
    e = np.asarray(list(edges), dtype=np.int64).reshape(-1, 2)
    e = e[e[:, 0] != e[:, 1]]
    both = np.concatenate([e, e[:, ::-1]], axis=0)
    keys = np.unique(both[:, 0] * (1 << 32) + both[:, 1]) if len(both) else np.zeros(0, np.int64)
    u = (keys >> 32).astype(np.int64)
    v = (keys & 0xFFFFFFFF).astype(np.int32)
    rp = np.zeros(n + 1, np.int64)
    np.add.at(rp, u + 1, 1)
    rp = np.cumsum(rp)
    return oracle.as_csr(n, rp, v)


def complete(n):
    return csr_from_edges(n, itertools.combinations(range(n), 2))


def wheel(n):
    """Hub 0 joined to a cycle on 1..n-1."""
    rim = [(i, i % (n - 1) + 1) for i in range(1, n)]
    return csr_from_edges(n, [(0, i) for i in range(1, n)] + rim)


def cycle(n):
    return csr_from_edges(n, [(i, (i + 1) % n) for i in range(n)])


def complete_bipartite(a, b):
    return csr_from_edges(a + b, [(i, a + j) for i in range(a) for j in range(b)])


def complete_tripartite(a, b, c):
    parts = [range(0, a), range(a, a + b), range(a + b, a + b + c)]
    e = []
    for p, q in itertools.combinations(parts, 2):
        e += [(i, j) for i in p for j in q]
    return csr_from_edges(a + b + c, e)


def grid(r, c):
    e = []
    for i in range(r):
        for j in range(c):
            v = i * c + j
            if j + 1 < c:
                e.append((v, v + 1))
            if i + 1 < r:
                e.append((v, v + c))
    return csr_from_edges(r * c, e)


def petersen():
    outer = [(i, (i + 1) % 5) for i in range(5)]
    spokes = [(i, i + 5) for i in range(5)]
    inner = [(5 + i, 5 + (i + 2) % 5) for i in range(5)]
    return csr_from_edges(10, outer + spokes + inner)


def friendship(k):
    """k triangles sharing vertex 0."""
    e = []
    for t in range(k):
        a, b = 1 + 2 * t, 2 + 2 * t
        e += [(0, a), (0, b), (a, b)]
    return csr_from_edges(2 * k + 1, e)


def book(k):
    """k triangles sharing the edge (0, 1)."""
    return csr_from_edges(k + 2, [(0, 1)] + [(0, 2 + t) for t in range(k)] + [(1, 2 + t) for t in range(k)])


def random_tree(n, seed):
    rng = np.random.default_rng(seed)
    return csr_from_edges(n, [(i, int(rng.integers(0, i))) for i in range(1, n)])


def gnp(n, p, seed):
    rng = np.random.default_rng(seed)
    iu = np.triu_indices(n, 1)
    keep = rng.random(len(iu[0])) < p
    return csr_from_edges(n, zip(iu[0][keep], iu[1][keep]))


def disjoint_union(*gs):
    e, off = [], 0
    for g in gs:
        for u in range(g.n):
            for v in g.col[g.row_ptr[u]:g.row_ptr[u + 1]]:
                if u < v:
                    e.append((u + off, int(v) + off))
        off += g.n
    return csr_from_edges(off, e)


def relabel(g, perm):
    e = []
    for u in range(g.n):
        for v in g.col[g.row_ptr[u]:g.row_ptr[u + 1]]:
            e.append((int(perm[u]), int(perm[v])))
    return csr_from_edges(g.n, e)


def dense(g):
    A = np.zeros((g.n, g.n), dtype=np.int64)
    for u in range(g.n):
        A[u, g.col[g.row_ptr[u]:g.row_ptr[u + 1]]] = 1
    return A


def brute_force(g):
    """Triple loop over a < b < c on the dense adjacency (tiny n only)."""
    A = dense(g)
    T = 0
    for a in range(g.n):
        for b in range(a + 1, g.n):
            if not A[a, b]:
                continue
            for c in range(b + 1, g.n):
                if A[a, c] and A[b, c]:
                    T += 1
    return T


def choose(n, k):
    return math.comb(n, k) if n >= k else 0
