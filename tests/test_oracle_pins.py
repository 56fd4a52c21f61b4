"""Pins of the CPU oracle against facts fixed by the paper and by mathematics
(closed forms, brute force, trace(A^3)/6, networkx, printed karate row,
invariants of the method).  No GPU."""
from __future__ import annotations

import os

import networkx as nx
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse import csgraph

import graphgen
import oracle
from _graphs import (book, brute_force, choose, complete, complete_bipartite, complete_tripartite,
                     csr_from_edges, cycle, dense, disjoint_union, friendship, gnp, grid, petersen,
                     random_tree, relabel, wheel)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def all_counts(g, level=None):
    r = oracle.alg4(g, level)
    return r, oracle.count_emd(g), oracle.alg3(g, level)


def assert_T(g, expected):
    r, emd, a3 = all_counts(g)
    assert r.T == expected
    assert emd == expected
    assert a3 == expected


# ------------------------------------------------------------ printed values

def read_golden(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split()
                vals[k] = float(v)
    return vals


def karate():
    G = nx.karate_club_graph()
    return csr_from_edges(G.number_of_nodes(), G.edges())


def test_karate_printed_row():
    """Table I/II, row karate: n=34, m=78, 45 triangles, k=35.9%."""
    gold = read_golden("karate.txt")
    g = karate()
    assert g.n == gold["n"] and g.m == gold["m"]
    r, emd, a3 = all_counts(g)
    assert r.T == emd == a3 == gold["triangles"]
    assert round(r.k, 1) == gold["k_percent"]
    assert r.E0 == 28 and r.T0 == 8 and r.T1 == 37


# ------------------------------------------------------------ closed forms

@pytest.mark.parametrize("n", range(1, 13))
def test_complete_graph(n):
    g = complete(n)
    assert_T(g, choose(n, 3))
    r = oracle.alg4(g)
    # root 0 at level 0, every other vertex at level 1: G0 = K_{n-1}
    assert r.T0 == choose(n - 1, 3)
    assert r.T1 == choose(n - 1, 2)
    assert r.E0 == choose(n - 1, 2)


@pytest.mark.parametrize("n", range(5, 16))
def test_wheel(n):
    g = wheel(n)
    assert_T(g, n - 1)
    r = oracle.alg4(g)
    assert r.T0 == 0 and r.T1 == n - 1 and r.E0 == n - 1


def test_wheel_w4_is_k4():
    assert_T(wheel(4), 4)


@pytest.mark.parametrize("seed", range(6))
def test_trees_have_no_triangles(seed):
    g = random_tree(50 + 17 * seed, seed)
    assert_T(g, 0)
    assert oracle.alg4(g).E0 == 0


@pytest.mark.parametrize("a,b", [(1, 1), (2, 3), (5, 5), (7, 2)])
def test_complete_bipartite(a, b):
    g = complete_bipartite(a, b)
    assert_T(g, 0)
    assert oracle.alg4(g).E0 == 0


@pytest.mark.parametrize("a,b,c", [(1, 1, 1), (2, 3, 4), (5, 1, 3), (4, 4, 4)])
def test_complete_tripartite(a, b, c):
    assert_T(complete_tripartite(a, b, c), a * b * c)


@pytest.mark.parametrize("n", [4, 6, 10, 3, 5, 9])
def test_cycles(n):
    assert_T(cycle(n), 1 if n == 3 else 0)
    assert (oracle.alg4(cycle(n)).E0 == 0) == (n % 2 == 0)


def test_grid_and_petersen():
    assert_T(grid(7, 9), 0)
    assert oracle.alg4(grid(7, 9)).E0 == 0
    p = petersen()
    assert_T(p, 0)
    assert oracle.alg4(p).E0 > 0          # odd cycles: not bipartite


@pytest.mark.parametrize("k", [1, 2, 5, 11])
def test_friendship_and_book(k):
    assert_T(friendship(k), k)
    assert_T(book(k), k)


def test_disjoint_union_is_additive():
    parts = [complete(6), wheel(9), petersen(), friendship(4), gnp(30, 0.3, 3)]
    g = disjoint_union(*parts)
    assert_T(g, sum(oracle.count_emd(p) for p in parts))


def test_empty_and_isolated():
    g = csr_from_edges(5, [])
    assert_T(g, 0)
    lev, roots = oracle.bfs_levels(g)
    assert roots == 5 and (lev == 0).all()
    g0 = csr_from_edges(0, [])
    assert oracle.count_emd(g0) == 0 and oracle.alg4(g0).T == 0


# ------------------------------------------------------------ independent counts

@pytest.mark.parametrize("seed", range(8))
def test_brute_force_small(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(2, 36))
    g = gnp(n, float(rng.uniform(0.05, 0.9)), seed)
    assert_T(g, brute_force(g))


@pytest.mark.parametrize("n,p", [(120, 0.2), (300, 0.05), (400, 0.5), (250, 0.9)])
def test_trace_a_cubed(n, p):
    g = gnp(n, p, n)
    A = dense(g)
    assert_T(g, int(np.trace(A @ A @ A)) // 6)


@pytest.mark.parametrize("scale", [8, 10])
def test_networkx_triangles(scale):
    n, s, d = graphgen.kronecker(scale, seed=scale)
    g = oracle.build_csr(n, s, d)
    G = nx.Graph()
    G.add_nodes_from(range(n))
    for u in range(n):
        G.add_edges_from((u, int(v)) for v in g.col[g.row_ptr[u]:g.row_ptr[u + 1]])
    tri = nx.triangles(G)
    assert_T(g, sum(tri.values()) // 3)
    tv = oracle.vertex_triangles(g)
    assert all(int(tv[v]) == tri[v] for v in range(n))


# ------------------------------------------------------------ levels

def scipy_levels(g):
    """BFS distance from the smallest id of each component (scipy)."""
    A = sp.csr_matrix((np.ones(g.nnz), g.col, g.row_ptr), shape=(g.n, g.n))
    ncomp, lab = csgraph.connected_components(A, directed=False)
    lev = np.full(g.n, -1, np.int64)
    for c in range(ncomp):
        members = np.flatnonzero(lab == c)
        root = members.min()
        dist = csgraph.shortest_path(A, unweighted=True, indices=root, directed=False)
        lev[members] = dist[members].astype(np.int64)
    return lev, ncomp


@pytest.mark.parametrize("gen", ["kron9", "er", "karate", "union"])
def test_levels_match_shortest_paths(gen):
    if gen == "kron9":
        n, s, d = graphgen.kronecker(9, seed=3)
        g = oracle.build_csr(n, s, d)
    elif gen == "er":
        n, s, d = graphgen.erdos_renyi(700, 0.003, 9)
        g = oracle.build_csr(n, s, d)
    elif gen == "karate":
        g = karate()
    else:
        g = disjoint_union(random_tree(20, 1), complete(5), csr_from_edges(3, []), cycle(9))
    lev, roots = oracle.bfs_levels(g)
    ref, ncomp = scipy_levels(g)
    assert roots == ncomp
    assert np.array_equal(lev.astype(np.int64), ref)


def test_levels_are_one_lipschitz():
    n, s, d = graphgen.kronecker(11, seed=5)
    g = oracle.build_csr(n, s, d)
    lev, _ = oracle.bfs_levels(g)
    u = np.repeat(np.arange(g.n), g.degrees())
    assert np.abs(lev[u] - lev[g.col]).max() <= 1


# ------------------------------------------------------------ invariants of the method

@pytest.fixture(scope="module")
def kron12():
    n, s, d = graphgen.kronecker(12, seed=12)
    return oracle.build_csr(n, s, d)


def test_three_counters_agree_kronecker(kron12):
    r, emd, a3 = all_counts(kron12)
    assert r.T == emd == a3
    assert r.T0 + r.T1 == r.T


def test_all_horizontal_levels_give_forward_hashed(kron12):
    """L = 0 everywhere is 1-Lipschitz: all edges horizontal, T1 = 0, T0 = T."""
    z = np.zeros(kron12.n, np.int32)
    r = oracle.alg4(kron12, z)
    assert r.T1 == 0 and r.T0 == oracle.count_emd(kron12)
    assert r.E0 == kron12.m
    assert oracle.alg3(kron12, z) == r.T


def multi_source_levels(g, roots):
    """BFS distance to the nearest of several roots (levels still 1-Lipschitz)."""
    A = sp.csr_matrix((np.ones(g.nnz), g.col, g.row_ptr), shape=(g.n, g.n))
    dist = csgraph.shortest_path(A, unweighted=True, indices=roots, directed=False).min(axis=0)
    lev = np.where(np.isinf(dist), 0, dist).astype(np.int32)
    return lev


@pytest.mark.parametrize("seed", range(3))
def test_count_invariant_under_root_choice(kron12, seed):
    rng = np.random.default_rng(seed)
    roots = rng.choice(kron12.n, size=1 + 5 * seed, replace=False)
    lev = multi_source_levels(kron12, roots)
    r = oracle.alg4(kron12, lev)
    assert r.T == oracle.count_emd(kron12)
    assert oracle.alg3(kron12, lev) == r.T


def test_count_invariant_under_relabelling():
    g = gnp(90, 0.15, 4)
    perm = np.random.default_rng(1).permutation(g.n)
    h = relabel(g, perm)
    assert oracle.alg4(h).T == oracle.alg4(g).T == brute_force(g)


def test_vertex_triangle_sum(kron12):
    assert int(oracle.vertex_triangles(kron12).sum()) == 3 * oracle.count_emd(kron12)


@pytest.mark.parametrize("seed", range(10))
def test_horizontal_edges_iff_not_bipartite(seed):
    rng = np.random.default_rng(seed)
    g = gnp(int(rng.integers(5, 40)), float(rng.uniform(0.02, 0.2)), seed)
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    for u in range(g.n):
        G.add_edges_from((u, int(v)) for v in g.col[g.row_ptr[u]:g.row_ptr[u + 1]])
    assert (oracle.alg4(g).E0 == 0) == nx.is_bipartite(G)


# ------------------------------------------------------------ CSR builder and partition

@pytest.mark.parametrize("scale", [6, 10, 13])
def test_build_csr_matches_numpy(scale):
    n, s, d = graphgen.kronecker(scale, seed=scale + 1)
    g = oracle.build_csr(n, s, d)
    ref = csr_from_edges(n, zip(s.tolist(), d.tolist()))
    assert np.array_equal(g.row_ptr, ref.row_ptr)
    assert np.array_equal(g.col, ref.col)


def test_build_csr_rejects_bad_ids():
    with pytest.raises(ValueError):
        oracle.build_csr(4, np.array([0, 4], np.int32), np.array([1, 2], np.int32))


@pytest.mark.parametrize("by_id", [False, True])
def test_partition_definition(kron12, by_id):
    lev, _ = oracle.bfs_levels(kron12)
    p = oracle.partition(kron12, lev, by_id)
    g = kron12
    deg = g.degrees()
    for x in range(0, g.n, 7):
        nb = g.col[g.row_ptr[x]:g.row_ptr[x + 1]]
        hor = nb[lev[nb] == lev[x]]
        above = (hor > x) if by_id else (deg[hor] > deg[x]) | ((deg[hor] == deg[x]) & (hor > x))
        row0 = p.c0[p.rp0[x]:p.rp0[x + 1]]
        assert np.array_equal(row0, np.concatenate([hor[above], hor[~above]]))
        assert p.up0[x] == above.sum()
        assert np.array_equal(p.c1[p.rp1[x]:p.rp1[x + 1]], nb[lev[nb] != lev[x]])
    assert p.rp0[-1] == 2 * oracle.alg4(g, lev).E0


@pytest.mark.parametrize("by_id", [False, True])
@pytest.mark.parametrize("seed", [1, 2])
def test_partition_orientations_give_forward_t0(by_id, seed):
    """Either orientation makes every horizontal edge the upper-part member
    of exactly one endpoint, and the forward algorithm over the upper parts
    (a triangle x < y < w of the orientation found once, at its two lowest
    vertices) counts the triangles whose three edges are horizontal: brute
    force over all vertex triples, the same for both orientations."""
    n, s, d = graphgen.kronecker(7, seed=seed)
    g = oracle.build_csr(n, s, d)
    lev, _ = oracle.bfs_levels(g)
    p = oracle.partition(g, lev, by_id)
    up = [set(p.c0[p.rp0[x]:p.rp0[x] + p.up0[x]].tolist()) for x in range(g.n)]
    hor = {(x, y) for x in range(g.n) for y in g.col[g.row_ptr[x]:g.row_ptr[x + 1]].tolist() if lev[x] == lev[y]}
    assert sum(len(u) for u in up) * 2 == len(hor)
    assert all((y in up[x]) != (x in up[y]) for x, y in hor)
    forward = sum(len(up[x] & up[y]) for x in range(g.n) for y in up[x])
    adj = [set(g.col[g.row_ptr[x]:g.row_ptr[x + 1]].tolist()) for x in range(g.n)]
    brute = sum(1 for x in range(g.n) for y in adj[x] if y > x for w in adj[x] & adj[y]
                if w > y and lev[x] == lev[y] == lev[w])
    assert forward == brute == oracle.alg4(g, lev).T0


# ------------------------------------------------------------ per-vertex counts

def _both_vertex(g, vs=None):
    """Whole-graph t(v) and the sampled routine's t(v) over every vertex."""
    tv = oracle.vertex_triangles(g)
    at = oracle.vertex_triangles_at(g, np.arange(g.n) if vs is None else vs)
    assert np.array_equal(at, tv if vs is None else tv[vs])
    return tv.astype(np.int64)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 7, 12])
def test_vertex_triangles_complete(n):
    assert np.all(_both_vertex(complete(n)) == choose(n - 1, 2))


@pytest.mark.parametrize("n", [5, 9, 14])
def test_vertex_triangles_wheel(n):
    tv = _both_vertex(wheel(n))
    assert tv[0] == n - 1 and np.all(tv[1:] == 2)


@pytest.mark.parametrize("k", [1, 3, 8])
def test_vertex_triangles_friendship_and_book(k):
    tv = _both_vertex(friendship(k))
    assert tv[0] == k and np.all(tv[1:] == 1)
    tv = _both_vertex(book(k))
    assert tv[0] == tv[1] == k and np.all(tv[2:] == 1)


def test_vertex_triangles_bipartite_and_empty():
    assert np.all(_both_vertex(complete_bipartite(4, 6)) == 0)
    assert _both_vertex(csr_from_edges(3, [])).tolist() == [0, 0, 0]


@pytest.mark.parametrize("n,p,seed", [(80, 0.2, 1), (150, 0.1, 2), (60, 0.6, 3)])
def test_vertex_triangles_diag_a_cubed(n, p, seed):
    # (A^3)[v, v] counts closed walks of length 3 through v: 2 t(v)
    g = gnp(n, p, seed)
    A = dense(g).astype(np.int64)
    tv = _both_vertex(g)
    assert np.array_equal(2 * tv, np.diag(A @ A @ A))


def test_vertex_triangles_sampled_kronecker():
    n, s, d = graphgen.kronecker(12, seed=5)
    g = oracle.build_csr(n, s, d)
    vs = np.random.default_rng(1).choice(n, 300, replace=False)
    tv = _both_vertex(g, vs)
    assert int(oracle.vertex_triangles(g).sum()) == 3 * oracle.count_emd(g)
    with pytest.raises(ValueError):
        oracle.vertex_triangles_at(g, [n])


# ------------------------------------------------------------ per-edge support

def _both_edge(g):
    """Whole-graph support and the one-at-a-time routine over every entry."""
    sup = oracle.edge_support(g)
    assert np.array_equal(oracle.edge_support_at(g, np.arange(g.nnz)), sup)
    return sup.astype(np.int64)


def _entries(g):
    return np.repeat(np.arange(g.n), np.diff(g.row_ptr)), g.col.astype(np.int64)


@pytest.mark.parametrize("n,p,seed", [(70, 0.2, 4), (120, 0.1, 5), (50, 0.7, 6)])
def test_edge_support_a_squared(n, p, seed):
    # (A^2)[u, v] counts the paths u - w - v: the common neighbours
    g = gnp(n, p, seed)
    A = dense(g).astype(np.int64)
    u, v = _entries(g)
    assert np.array_equal(_both_edge(g), (A @ A)[u, v])


@pytest.mark.parametrize("n", [2, 3, 6, 11])
def test_edge_support_complete(n):
    assert np.all(_both_edge(complete(n)) == n - 2)


@pytest.mark.parametrize("n", [5, 8, 13])
def test_edge_support_wheel(n):
    g = wheel(n)
    sup = _both_edge(g)
    u, v = _entries(g)
    spoke = (u == 0) | (v == 0)
    assert np.all(sup[spoke] == 2) and np.all(sup[~spoke] == 1)


@pytest.mark.parametrize("k", [1, 4, 9])
def test_edge_support_book_and_friendship(k):
    g = book(k)
    sup = _both_edge(g)
    u, v = _entries(g)
    spine = ((u == 0) & (v == 1)) | ((u == 1) & (v == 0))
    assert np.all(sup[spine] == k) and np.all(sup[~spine] == 1)
    assert np.all(_both_edge(friendship(k)) == 1)


def test_edge_support_bipartite_is_zero():
    assert np.all(_both_edge(complete_bipartite(3, 5)) == 0)


@pytest.mark.parametrize("seed", [1, 2])
def test_edge_support_sums(seed):
    # each triangle gives 1 to its 3 edges, each stored at 2 entries; the
    # entries of row v see the 2 edges at v of every triangle through v
    n, s, d = graphgen.kronecker(10, seed=seed)
    g = oracle.build_csr(n, s, d)
    sup = _both_edge(g)
    assert int(sup.sum()) == 6 * oracle.count_emd(g)
    u, v = _entries(g)
    assert np.array_equal(np.bincount(u, weights=sup, minlength=g.n).astype(np.int64),
                          2 * oracle.vertex_triangles(g).astype(np.int64))
    # the two entries of an edge agree
    rev = {(int(a), int(b)): int(c) for a, b, c in zip(u, v, sup)}
    assert all(rev[(b, a)] == c for (a, b), c in rev.items())
    with pytest.raises(ValueError):
        oracle.edge_support_at(g, [g.nnz])


# ------------------------------------------------------------ degree relabel

def _check_relabel(g):
    h, perm = oracle.relabel_degree(g)
    deg = g.degrees()
    # the order: numpy's lexsort by (decreasing degree, increasing id)
    assert np.array_equal(perm, np.lexsort((np.arange(g.n), -deg)).astype(np.int32))
    inv = np.empty(g.n, np.int64)
    inv[perm] = np.arange(g.n)
    # the same edge set under the map, rows sorted
    u, v = _entries(g)
    hu, hv = _entries(h)
    assert np.array_equal(np.sort(inv[u] * g.n + inv[v]), hu * g.n + hv)
    assert np.array_equal(h.degrees(), deg[perm])
    return h, perm


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_relabel_degree_kronecker(seed):
    n, s, d = graphgen.kronecker(10, seed=seed)
    g = oracle.build_csr(n, s, d)
    h, _ = _check_relabel(g)
    assert oracle.count_emd(h) == oracle.count_emd(g)
    lev, _ = oracle.bfs_levels(h)
    assert oracle.alg4(h, lev).T == oracle.count_emd(g)


def test_relabel_degree_star_and_ties():
    # star with hub 5: the hub becomes 0; leaves keep their order
    g = csr_from_edges(8, [(5, i) for i in range(8) if i != 5])
    h, perm = _check_relabel(g)
    assert perm.tolist() == [5, 0, 1, 2, 3, 4, 6, 7]
    # all degrees equal: the identity
    h, perm = _check_relabel(cycle(9))
    assert perm.tolist() == list(range(9))
    _check_relabel(csr_from_edges(4, []))


# ---------------------------------------------------------------- edge-sampled edge iterator

@pytest.mark.parametrize("n", [4, 7, 12])
def test_emd_entries_complete_graph(n):
    # in K_n the entry (u, v), u < v, closes a triangle with every w > v
    g = complete(n)
    for e in range(g.nnz):
        u = int(np.searchsorted(g.row_ptr, e, side="right")) - 1
        v = int(g.col[e])
        assert oracle.count_emd_entries(g, [e]) == (n - 1 - v if v > u else 0)
    assert oracle.count_emd_entries(g, np.arange(g.nnz), threads=3) == choose(n, 3)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_emd_entries_partition_sums_to_brute_force(seed):
    g = gnp(30, 0.3, seed)
    want = brute_force(g)
    rng = np.random.default_rng(seed)
    part = rng.integers(0, 3, g.nnz)
    parts = [oracle.count_emd_entries(g, np.nonzero(part == k)[0], threads=k + 1) for k in range(3)]
    assert sum(parts) == want
    assert oracle.count_emd_entries(g, [], threads=2) == 0


def test_emd_entries_threads_agree(kron12):
    g = kron12
    es = np.arange(0, g.nnz, 7)
    one = oracle.count_emd_entries(g, es, threads=1)
    assert oracle.count_emd_entries(g, es, threads=4) == one
    assert oracle.count_emd_entries(g, np.arange(g.nnz), threads=4) == oracle.count_emd(g)


@pytest.mark.parametrize("seed", range(6))
def test_t0_t1_by_brute_force(seed):
    # every triangle classified by its number of horizontal edges: T0 counts
    # those with three, T1 those with one; none has zero or two
    rng = np.random.default_rng(500 + seed)
    g = gnp(int(rng.integers(8, 34)), float(rng.uniform(0.1, 0.7)), 900 + seed)
    lev, _ = oracle.bfs_levels(g)
    A = dense(g).astype(bool)
    hist = [0, 0, 0, 0]
    for a in range(g.n):
        for b in range(a + 1, g.n):
            if not A[a, b]:
                continue
            for c in range(b + 1, g.n):
                if A[a, c] and A[b, c]:
                    hist[int(lev[a] == lev[b]) + int(lev[a] == lev[c]) + int(lev[b] == lev[c])] += 1
    assert hist[0] == 0 and hist[2] == 0
    r = oracle.alg4(g, lev)
    assert (r.T0, r.T1) == (hist[3], hist[1])
