"""GPU parity: every output of the HIP path equals the CPU oracle bit for bit
(integer work), on seeded synthetic graphs that span several tiles and
ragged tails, edge cases, and the full scale-20 Kronecker configuration."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

import graphgen
import oracle
from _graphs import complete, cycle, disjoint_union, friendship, gnp, petersen, random_tree, wheel, csr_from_edges

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2309_09064_amd as tc
    from paper_2309_09064_amd import _capi
    _capi.load()
    return tc


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()


def to_gpu(g):
    col = g.col if g.nnz else np.zeros(0, np.int32)
    return dev(g.row_ptr.astype(np.int32)), dev(col)


def kron(scale, seed=1):
    n, s, d = graphgen.kronecker(scale, seed=seed)
    return oracle.build_csr(n, s, d)


def er(n, p, seed):
    nn, s, d = graphgen.erdos_renyi(n, p, seed)
    return oracle.build_csr(nn, s, d)


def chung_lu_small(seed=3):
    n, s, d = graphgen.chung_lu(1 << 14, 2.1, 16.0, 2048.0, seed=seed)
    return oracle.build_csr(n, s, d)


GRAPHS = {
    "k1": lambda: complete(1),
    "k2": lambda: complete(2),
    "k12": lambda: complete(12),
    "wheel9": lambda: wheel(9),
    "petersen": petersen,
    "tree": lambda: random_tree(300, 4),
    "empty5": lambda: csr_from_edges(5, []),
    "union": lambda: disjoint_union(complete(7), cycle(11), friendship(5), random_tree(40, 2), csr_from_edges(4, [])),
    "gnp": lambda: gnp(400, 0.08, 7),
    "kron8": lambda: kron(8, 2),
    "kron11": lambda: kron(11, 3),
    "kron14": lambda: kron(14, 4),
    "er_sparse": lambda: er(3000, 0.0008, 5),
    "er_dense": lambda: er(1500, 0.03, 6),
    "chunglu14": chung_lu_small,
}

_cache = {}


def graph(name):
    if name not in _cache:
        _cache[name] = GRAPHS[name]()
    return _cache[name]


# ------------------------------------------------------------------ CSR build

@pytest.mark.parametrize("case", ["kron8", "kron13", "er", "loops_dups", "no_edges", "chunglu"])
def test_build_csr_matches_oracle(tc, case):
    if case == "kron8":
        n, s, d = graphgen.kronecker(8, seed=9)
    elif case == "kron13":
        n, s, d = graphgen.kronecker(13, seed=10)
    elif case == "er":
        n, s, d = graphgen.erdos_renyi(5000, 0.002, 11)
    elif case == "loops_dups":
        rng = np.random.default_rng(0)
        n = 300
        s = rng.integers(0, n, 5000).astype(np.int32)
        d = rng.integers(0, n, 5000).astype(np.int32)
        d[:200] = s[:200]                        # self-loops
        s = np.concatenate([s, d[:700]])         # reversed duplicates
        d = np.concatenate([d, s[:700]])
    elif case == "no_edges":
        n, s, d = 17, np.zeros(0, np.int32), np.zeros(0, np.int32)
    else:
        n, s, d = graphgen.chung_lu(1 << 13, 2.1, 8.0, 1024.0, seed=12)
    ref = oracle.build_csr(n, s, d)
    rp, col = tc.build_csr(n, dev(s), dev(d))
    assert np.array_equal(rp.cpu().numpy(), ref.row_ptr.astype(np.int32))
    assert np.array_equal(col.cpu().numpy(), ref.col)


def test_build_csr_range_error(tc):
    with pytest.raises(tc.TCError) as ei:
        tc.build_csr(10, dev([1, 2, 10]), dev([0, 0, 0]))
    assert ei.value.code == -2


def test_build_csr_capacity_error_reports_nnz(tc):
    from paper_2309_09064_amd import _capi
    lib = _capi.load()
    s, d = dev([0, 1, 2, 0]), dev([1, 2, 0, 3])
    need = ctypes.c_size_t()
    assert lib.tc_build_csr_ws(4, 4, ctypes.byref(need)) == 0
    ws = tc.workspace(need.value)
    rp = torch.empty(5, dtype=torch.int32, device="cuda")
    col = torch.empty(8, dtype=torch.int32, device="cuda")
    nnz = ctypes.c_int64()
    rc = lib.tc_build_csr(4, 4, ctypes.c_void_p(s.data_ptr()), ctypes.c_void_p(d.data_ptr()),
                          ctypes.c_void_p(rp.data_ptr()), ctypes.c_void_p(col.data_ptr()), 5, ctypes.byref(nnz),
                          ctypes.c_void_p(ws.data_ptr()), need.value, None)
    assert rc == _capi.TC_ERR_CAPACITY and nnz.value == 8


# ------------------------------------------------------------------ levels

@pytest.mark.parametrize("name", list(GRAPHS))
def test_bfs_levels_match_oracle(tc, name):
    g = graph(name)
    ref, _ = oracle.bfs_levels(g)
    rp, col = to_gpu(g)
    lev, nlev = tc.bfs_levels(rp, col)
    assert np.array_equal(lev.cpu().numpy(), ref)
    assert nlev == (int(ref.max()) + 1 if g.n else 0)


def _bfs_mix(first_small):
    # isolated vertices first (the first BFS starts past vertex 0), a long
    # path (600 top-down levels), a star (its leaves' level goes bottom-up
    # by the edge rule) and a Kronecker graph.  The first BFS covers the
    # smallest-id component, the path or (with first_small) a short cycle;
    # the second pass - linking over every row left, then a multi-source BFS
    # - covers the rest, most of the vertices.
    path = csr_from_edges(600, [(i, i + 1) for i in range(599)])
    star = csr_from_edges(3000, [(0, i) for i in range(1, 3000)])
    parts = [csr_from_edges(5, [])] + ([cycle(40)] if first_small else []) + [path, star, kron(12, 8)]
    return disjoint_union(*parts)


@pytest.mark.parametrize("first_small", [False, True], ids=["path_first", "cycle_first"])
def test_bfs_levels_direction_mix(tc, first_small):
    # both BFS directions and a large second pass, checked level by level
    # against the serial BFS
    g = _bfs_mix(first_small)
    ref, _ = oracle.bfs_levels(g)
    rp, col = to_gpu(g)
    lev, nlev = tc.bfs_levels(rp, col)
    assert np.array_equal(lev.cpu().numpy(), ref)
    assert nlev == int(ref.max()) + 1


# ------------------------------------------------------------------ partition

@pytest.mark.parametrize("orientation", [0, 1])
@pytest.mark.parametrize("name", ["k12", "wheel9", "union", "gnp", "kron11", "kron14", "er_dense", "chunglu14"])
def test_partition_matches_oracle(tc, name, orientation):
    g = graph(name)
    lev, _ = oracle.bfs_levels(g)
    ref = oracle.partition(g, lev, by_id=orientation == tc.TC_ORIENT_ID)
    rp, col = to_gpu(g)
    out = tc.partition(rp, col, dev(lev), orientation=orientation)
    e0 = int(ref.rp0[-1]) // 2
    assert out["e0"] == e0
    assert np.array_equal(out["rp0"].cpu().numpy(), ref.rp0.astype(np.int32))
    assert np.array_equal(out["rp1"].cpu().numpy(), ref.rp1.astype(np.int32))
    assert np.array_equal(out["up0"].cpu().numpy(), ref.up0)
    assert np.array_equal(out["c0"].cpu().numpy()[:2 * e0], ref.c0)
    assert np.array_equal(out["c1"].cpu().numpy()[:len(ref.c1)], ref.c1)


@pytest.mark.parametrize("shift", [1, 2, 3])
def test_partition_and_count_unaligned_col(tc, shift):
    """A column array 4, 8 or 12 bytes past a 16-byte boundary: the row
    passes read each thread's run entry by entry instead of by 16-byte
    loads, with the same partition and counts."""
    g = graph("kron14")
    lev, _ = oracle.bfs_levels(g)
    ref = oracle.partition(g, lev)
    rp, col = to_gpu(g)
    buf = torch.zeros(col.numel() + 4, dtype=torch.int32, device=col.device)
    view = buf[shift:shift + col.numel()]
    view.copy_(col)
    assert view.data_ptr() % 16 == 4 * shift
    out = tc.partition(rp, view, dev(lev))
    e0 = int(ref.rp0[-1]) // 2
    assert out["e0"] == e0
    assert np.array_equal(out["rp0"].cpu().numpy(), ref.rp0.astype(np.int32))
    assert np.array_equal(out["c0"].cpu().numpy()[:2 * e0], ref.c0)
    assert np.array_equal(out["c1"].cpu().numpy()[:len(ref.c1)], ref.c1)
    res = tc.count(rp, view)
    r4 = oracle.alg4(g)
    assert (res.T, res.T0, res.T1, res.e0) == (r4.T, r4.T0, r4.T1, r4.E0)


# ------------------------------------------------------------------ count

def check_count(tc, g, options=None, levels=None):
    ref = oracle.alg4(g, levels)
    rp, col = to_gpu(g)
    res = tc.count(rp, col, None if levels is None else dev(levels), options)
    assert (res.T, res.T0, res.T1, res.e0) == (ref.T, ref.T0, ref.T1, ref.E0), (res, ref)
    return res


@pytest.fixture(scope="module", params=[700, 3000])
def colliding(request):
    """Two owners X, Y (level 1, joined by a horizontal edge, both on the
    root) whose lists hold five ids equal modulo 2^24: the tables hash the
    low 24 bits, so all five share both candidate buckets (four slots) of
    any table and at least one goes on to linear probing; the other
    neighbours also sit above 2^24.  With 700 other neighbours a forced
    wavefront table is loaded above 1/16 (two candidates) and the workgroup
    table below (one); with 3000 the workgroup table takes two candidates.
    The triangles are X-Y-root and X-Y-c for the five c: 6.  The graph, its
    device copy and the oracle's counts are made once per size."""
    c = [7 + (k << 24) for k in range(5)]
    n = (4 << 24) + 16
    fill = request.param
    filler_x = [(1 << 24) + 100 + i for i in range(fill)]
    filler_y = [(1 << 24) + 100 + fill + i for i in range(fill)]
    X, Y = 1, 2
    edges = [(0, X), (0, Y), (X, Y)] + [(X, v) for v in c + filler_x] + [(Y, v) for v in c + filler_y]
    g = csr_from_edges(n, edges)
    return to_gpu(g), oracle.alg4(g)


@pytest.mark.parametrize("opts", [dict(), dict(force_strategy=0), dict(force_strategy=1),
                                  dict(force_strategy=1, wg_slice_max=256)])
def test_count_colliding_ids(tc, colliding, opts):
    (rp, col), ref = colliding
    res = tc.count(rp, col, options=tc.Options(**opts))
    assert (res.T, res.T0, res.T1, res.e0) == (ref.T, ref.T0, ref.T1, ref.E0) == (6, 0, 6, 1)


@pytest.mark.parametrize("strategy", [-1, 0, 1, 3])
@pytest.mark.parametrize("name", ["k12", "union", "kron11", "kron14", "er_dense", "chunglu14"])
def test_count_id_orientation(tc, name, strategy):
    # N0+ lists by id (the u < v of Algorithms 2 and 4): the same T, T0 and T1
    res = check_count(tc, graph(name), tc.Options(orientation=tc.TC_ORIENT_ID, force_strategy=strategy,
                                                   validate=True))
    assert res.T == oracle.count_emd(graph(name))


@pytest.mark.parametrize("name", list(GRAPHS))
def test_count_matches_oracle(tc, name):
    g = graph(name)
    res = check_count(tc, g, tc.Options(validate=True, timing=True))
    assert res.T == oracle.count_emd(g)


STRATS = ["wave_hash", "wg_hash", "bsearch", "merge"]


@pytest.mark.parametrize("strategy", range(4), ids=STRATS)
@pytest.mark.parametrize("name", ["k12", "union", "gnp", "kron11", "kron14", "er_dense", "chunglu14"])
def test_count_strategy_invariance(tc, name, strategy):
    res = check_count(tc, graph(name), tc.Options(force_strategy=strategy))
    if res.items:
        assert sum(res.strategy_items.values()) == res.items


@pytest.mark.parametrize("cfg", [dict(wave_slots=64, wg_slots=1024), dict(wave_slots=128, wg_slots=1024, chunk_work=64),
                                 dict(chunk_work=1), dict(grid_blocks=1), dict(grid_blocks=3, wave_slots=256),
                                 dict(wave_max_owner=8), dict(merge_max_owner=31), dict(merge_max_owner=-1),
                                 dict(merge_max_owner=1, wave_slots=64)])
@pytest.mark.parametrize("name", ["kron14", "chunglu14", "er_dense"])
def test_count_tiles_and_grids(tc, name, cfg):
    check_count(tc, graph(name), tc.Options(**cfg))


@pytest.mark.parametrize("cfg", [dict(wave_slots=64, wg_slots=1024, force_strategy=1),
                                 dict(wave_slots=64, wg_slots=2048), dict(wave_slots=128, wg_slots=1024, chunk_work=256)])
def test_count_sliced_owner_lists(tc, cfg):
    # owner lists longer than half the workgroup table are hashed slice by
    # slice: with every edge horizontal (levels 0) the N0+ lists of a dense
    # graph reach several slices
    for g in (complete(700), gnp(900, 0.5, 7), graph("kron14")):
        res = check_count(tc, g, tc.Options(**cfg), levels=np.zeros(g.n, np.int32))
        assert res.T1 == 0
        check_count(tc, g, tc.Options(**cfg))
    rp, col = to_gpu(complete(700))
    assert tc.count(rp, col, dev(np.zeros(700, np.int32)), tc.Options(**cfg)).T == 700 * 699 * 698 // 6


@pytest.mark.parametrize("slice_max", [64, 128, 512])
def test_count_many_small_slices(tc, slice_max):
    # workgroup slices of 64..512 owner elements: every long owner list is cut
    # into many value ranges, and each partner list is narrowed to each range
    # through the line samples (searches that start and end at every offset
    # within a line); with every edge horizontal both kinds' lists are sliced
    opts = tc.Options(force_strategy=1, wg_slice_max=slice_max)
    for g in (complete(300), gnp(700, 0.3, 11), graph("kron14")):
        check_count(tc, g, opts, levels=np.zeros(g.n, np.int32))
        check_count(tc, g, opts)
    rp, col = to_gpu(complete(300))
    assert tc.count(rp, col, dev(np.zeros(300, np.int32)), opts).T == 300 * 299 * 298 // 6


def test_count_closed_forms(tc):
    from _graphs import book, complete_tripartite, choose
    for n in (3, 5, 9, 20):
        rp, col = to_gpu(complete(n))
        assert tc.count(rp, col).T == choose(n, 3)
    for n in (5, 8, 30):
        rp, col = to_gpu(wheel(n))
        r = tc.count(rp, col)
        assert (r.T, r.T0, r.T1) == (n - 1, 0, n - 1)
    rp, col = to_gpu(complete_tripartite(4, 5, 6))
    assert tc.count(rp, col).T == 120
    rp, col = to_gpu(book(9))
    assert tc.count(rp, col).T == 9


@pytest.mark.parametrize("kind", ["zero", "multi"])
def test_count_with_given_levels(tc, kind):
    g = graph("kron11")
    if kind == "zero":
        lev = np.zeros(g.n, np.int32)
    else:
        import scipy.sparse as sp
        from scipy.sparse import csgraph
        A = sp.csr_matrix((np.ones(g.nnz), g.col, g.row_ptr), shape=(g.n, g.n))
        roots = np.random.default_rng(5).choice(g.n, 9, replace=False)
        dist = csgraph.shortest_path(A, unweighted=True, indices=roots, directed=False).min(axis=0)
        lev = np.where(np.isinf(dist), 0, dist).astype(np.int32)
    res = check_count(tc, g, tc.Options(validate=True), levels=lev)
    assert res.T == oracle.count_emd(g)


def test_validate_rejects_bad_input(tc):
    g = graph("gnp")
    rp, col = to_gpu(g)
    bad = col.clone()
    r0, r1 = int(g.row_ptr[3]), int(g.row_ptr[4])
    assert r1 - r0 >= 2
    bad[r0], bad[r0 + 1] = col[r0 + 1], col[r0]          # unsorted row
    with pytest.raises(tc.TCError) as ei:
        tc.count(rp, bad, options=tc.Options(validate=True))
    assert ei.value.code == -8
    lev = torch.zeros(g.n, dtype=torch.int32, device="cuda")
    lev[int(g.col[r0])] = 5                                # levels 5 apart on an edge
    with pytest.raises(tc.TCError):
        tc.count(rp, col, lev, tc.Options(validate=True))


def test_repeated_calls_reuse_workspace(tc):
    g = graph("kron14")
    rp, col = to_gpu(g)
    c = tc.Counter(g.n, g.nnz)
    ref = oracle.alg4(g)
    for _ in range(3):
        assert c(rp, col).T == ref.T


# ------------------------------------------------------------------ full size

def test_full_size_kronecker_scale20(tc):
    """Kronecker scale 20, edgefactor 16: CSR, levels and counts against the
    oracle, in the configuration the benchmark times."""
    n, s, d = graphgen.kronecker(20, seed=1)
    rp, col = tc.build_csr(n, dev(s), dev(d))
    g = oracle.build_csr(n, s, d)
    assert np.array_equal(rp.cpu().numpy(), g.row_ptr.astype(np.int32))
    assert np.array_equal(col.cpu().numpy(), g.col)
    lev, _ = tc.bfs_levels(rp, col)
    ref_lev, _ = oracle.bfs_levels(g)
    assert np.array_equal(lev.cpu().numpy(), ref_lev)
    ref = oracle.alg4(g, ref_lev)
    res = tc.count(rp, col, options=tc.Options(timing=True))
    assert (res.T, res.T0, res.T1, res.e0) == (ref.T, ref.T0, ref.T1, ref.E0)
