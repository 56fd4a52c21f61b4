"""The benchmark's byte model B_alg (algorithmic bytes of the intersection
pass), on the CPU: closed forms on small graphs and an edge-by-edge
recomputation in plain Python."""
from __future__ import annotations

import numpy as np
import pytest

import bench
import oracle
from _graphs import complete, csr_from_edges, gnp

torch = pytest.importorskip("torch")


def t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32))


def balg(g, lev):
    return bench.b_alg(t(g.row_ptr), t(g.col), t(lev))


@pytest.mark.parametrize("n", [3, 6, 11])
def test_complete_graph_all_horizontal(n):
    # L = 0: every edge horizontal, no N1 lists; equal degrees, so N0+(v)
    # holds the n - 1 - v larger ids and an edge u < v streams n - 1 - v
    g = complete(n)
    want = 4 * sum(v * (n - 1 - v) for v in range(n)) + 4 * (n * (n - 1) // 2) + 8 * (n * (n - 1) // 2) + 8 * n
    assert balg(g, np.zeros(n, np.int32)) == want


def test_star_has_no_intersections():
    # BFS levels: hub 0, leaves 1; no horizontal edge, so only the N1 lists
    # (read once) and the records count
    n = 9
    g = csr_from_edges(n, [(0, i) for i in range(1, n)])
    lev, _ = oracle.bfs_levels(g)
    assert balg(g, lev) == 4 * g.nnz + 8 * n


@pytest.mark.parametrize("seed", [1, 2])
def test_matches_edge_by_edge_recount(seed):
    g = gnp(60, 0.15, seed)
    lev, _ = oracle.bfs_levels(g)
    deg = np.diff(g.row_ptr)
    rows = [list(g.col[g.row_ptr[u]:g.row_ptr[u + 1]]) for u in range(g.n)]
    rank = lambda x: (deg[x], x)
    d1 = [sum(1 for y in rows[x] if lev[y] != lev[x]) for x in range(g.n)]
    d0p = [sum(1 for y in rows[x] if lev[y] == lev[x] and rank(y) > rank(x)) for x in range(g.n)]
    want = 0
    for x in range(g.n):
        for y in rows[x]:
            if lev[y] == lev[x] and rank(y) > rank(x):
                want += 4 * (min(d1[x], d1[y]) + min(d0p[x], d0p[y])) + 8
    want += 4 * (sum(d1) + sum(d0p)) + 8 * g.n
    assert balg(g, lev) == want


def test_batch_from_union_layout_on_host():
    # the union-to-packed layout conversion is plain torch: check it on CPU
    # tensors against packing the graphs one by one
    import paper_2309_09064_amd as tc
    from _graphs import complete, wheel
    gs = [complete(4), csr_from_edges(0, []), wheel(6), csr_from_edges(3, []), gnp(20, 0.3, 4)]
    voff = np.concatenate([[0], np.cumsum([g.n for g in gs])]).astype(np.int64)
    rp = [0]
    cols = []
    for i, g in enumerate(gs):
        rp.extend((rp[-1] + np.diff(g.row_ptr).cumsum()).tolist())
        cols.append(g.col.astype(np.int64) + voff[i])
    union = tc.Batch.from_union(t(np.array(rp)), t(np.concatenate(cols)), voff)
    ref = tc.pack_csr([(t(g.row_ptr), t(g.col)) for g in gs])
    assert torch.equal(union.row_ptr, ref.row_ptr) and torch.equal(union.col, ref.col)
    assert np.array_equal(union.edge_off, ref.edge_off) and np.array_equal(union.vtx_off, ref.vtx_off)
    assert union.graphs == 5
