"""GPU parity of the batched count (tc_count_batched, tc_batch_plan_*):
per-graph counts of a packed batch, each graph a CSR with local ids, equal
the oracle's count of each graph on its own.  Small mixed batches check
every graph (empty members included), under every strategy, with given
levels, in several internal groups, and through a captured plan replayed
several times with eager work between the replays; the full 4096-graph batch
of Erdos-Renyi and Kronecker members checks all 4096 counts against the
oracle's stored counts (tests/golden/batch_counts.txt, written by
tests/golden/make_batch_counts.py, which calls the oracle only), both by the
eager call and by plan replays."""
from __future__ import annotations

import concurrent.futures as cf
import os
import time

import numpy as np
import pytest

import graphgen
import oracle
from _graphs import complete, csr_from_edges, cycle, gnp, petersen, random_tree, wheel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "batch_counts.txt")


@pytest.fixture(scope="module")
def tc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2309_09064_amd as tc
    return tc


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()


def to_gpu(g):
    return dev(g.row_ptr.astype(np.int32)), dev(g.col if g.nnz else np.zeros(0, np.int32))


def kron(scale, seed):
    n, s, d = graphgen.kronecker(scale, seed=seed)
    return oracle.build_csr(n, s, d)


def small_batch(seed):
    rng = np.random.default_rng(seed)
    gs = [csr_from_edges(0, []), complete(1), complete(12), wheel(9), petersen(), cycle(7),
          csr_from_edges(5, []), random_tree(80, seed)]
    for i in range(12):
        gs.append(gnp(int(rng.integers(20, 300)), float(rng.uniform(0.02, 0.3)), seed * 100 + i))
    for i in range(6):
        gs.append(kron(int(rng.integers(7, 11)), seed * 100 + i))
    gs.append(csr_from_edges(0, []))
    order = rng.permutation(len(gs))
    return [gs[i] for i in order]


def want_counts(gs):
    return np.array([oracle.alg4(g).T if g.n else 0 for g in gs], dtype=np.int64)


@pytest.mark.parametrize("seed", [1, 2])
def test_small_batch_every_graph(tc, seed):
    gs = small_batch(seed)
    b = tc.pack_csr([to_gpu(g) for g in gs])
    counts, res = tc.count_batched(b, options=tc.Options(validate=True))
    want = want_counts(gs)
    assert np.array_equal(counts.cpu().numpy(), want)
    assert res.T == int(want.sum())
    # T0 and T1 depend on the levels: the per-graph BFS keeps the serial roots
    refs = [oracle.alg4(g) for g in gs if g.n]
    assert (res.T0, res.T1, res.e0) == (sum(r.T0 for r in refs), sum(r.T1 for r in refs), sum(r.E0 for r in refs))


@pytest.mark.parametrize("seed,cap", [(1, 0), (2, 0), (9, 700)])
def test_batched_levels_every_vertex(tc, seed, cap):
    gs = small_batch(seed)
    b = tc.pack_csr([to_gpu(g) for g in gs])
    lev, nl = tc.bfs_levels_batched(b)
    want = np.concatenate([oracle.bfs_levels(g)[0] for g in gs if g.n])
    assert np.array_equal(lev.cpu().numpy(), want)
    assert nl == max(int(oracle.bfs_levels(g)[0].max()) + 1 for g in gs if g.n)


def test_batched_levels_many_components(tc):
    # a graph of many small components and isolated vertices, a long path
    # (one level per vertex) and a star, side by side
    rng = np.random.default_rng(3)
    parts = []
    for i in range(300):
        k = int(rng.integers(1, 6))
        parts.append([(3 * i + a, 3 * i + b) for a in range(k % 3) for b in range(a + 1, 3)])
    comps = csr_from_edges(900 + 50, [e for p in parts for e in p])
    path = csr_from_edges(1500, [(i, i + 1) for i in range(1499)])
    star = csr_from_edges(2000, [(0, i) for i in range(1, 2000)])
    gs = [comps, path, star, gnp(3000, 0.002, 5)]
    b = tc.pack_csr([to_gpu(g) for g in gs])
    lev, nl = tc.bfs_levels_batched(b)
    want = np.concatenate([oracle.bfs_levels(g)[0] for g in gs])
    assert np.array_equal(lev.cpu().numpy(), want)
    assert nl == 1500
    counts, _ = tc.count_batched(b)
    assert np.array_equal(counts.cpu().numpy(), want_counts(gs))


def test_batch_levels_both_bfs_paths(tc):
    # graphs of at most 65536 vertices keep their visited bits in LDS, larger
    # ones claim vertices through the levels: both in one batch, at and
    # around the size limit, with a path (one level per vertex), a star and
    # many components
    big = kron(17, seed=5)   # 131072 vertices
    edge = kron(16, seed=6)  # 65536 vertices
    path = csr_from_edges(70000, [(i, i + 1) for i in range(69999)])
    star = csr_from_edges(65537, [(0, i) for i in range(1, 65537)])
    gs = [big, edge, path, star, gnp(3000, 0.002, 7), complete(9)]
    b = tc.pack_csr([to_gpu(g) for g in gs])
    lev, nl = tc.bfs_levels_batched(b)
    want = np.concatenate([oracle.bfs_levels(g)[0] for g in gs])
    assert np.array_equal(lev.cpu().numpy(), want)
    assert nl == 70000
    counts, _ = tc.count_batched(b, options=tc.Options(validate=True))
    assert np.array_equal(counts.cpu().numpy(), want_counts(gs))


@pytest.mark.parametrize("force", [0, 1, 2, 3])
def test_batch_strategy_invariance(tc, force):
    gs = small_batch(3)
    b = tc.pack_csr([to_gpu(g) for g in gs])
    counts, _ = tc.count_batched(b, options=tc.Options(force_strategy=force))
    assert np.array_equal(counts.cpu().numpy(), want_counts(gs))


def test_batch_id_orientation(tc):
    gs = small_batch(4)
    b = tc.pack_csr([to_gpu(g) for g in gs])
    counts, res = tc.count_batched(b, options=tc.Options(orientation=tc.TC_ORIENT_ID, validate=True))
    want = want_counts(gs)
    assert np.array_equal(counts.cpu().numpy(), want)
    refs = [oracle.alg4(g) for g in gs if g.n]
    assert (res.T0, res.T1) == (sum(r.T0 for r in refs), sum(r.T1 for r in refs))


def test_batch_levels_match_single_graph_levels(tc):
    # given levels: each graph's own BFS levels, packed; same counts, and the
    # batch's own BFS gives the same levels count as the largest graph's
    gs = small_batch(4)
    b = tc.pack_csr([to_gpu(g) for g in gs])
    levs = []
    deepest = 1
    for g in gs:
        if g.n == 0:
            continue
        rp, col = to_gpu(g)
        lev, nl = tc.bfs_levels(rp, col)
        olev, _ = oracle.bfs_levels(g)
        assert np.array_equal(lev.cpu().numpy(), olev)
        levs.append(lev)
        deepest = max(deepest, nl)
    packed = torch.cat(levs)
    a, ra = tc.count_batched(b, levels=packed, options=tc.Options(validate=True))
    c, rc = tc.count_batched(b)
    assert torch.equal(a, c)
    assert np.array_equal(a.cpu().numpy(), want_counts(gs))
    assert rc.levels == deepest and (ra.T0, ra.T1) == (rc.T0, rc.T1)


def test_batch_all_empty_and_single(tc):
    b = tc.pack_csr([to_gpu(csr_from_edges(0, [])), to_gpu(csr_from_edges(3, []))])
    counts, res = tc.count_batched(b)
    assert counts.cpu().tolist() == [0, 0] and res.T == 0
    b = tc.pack_csr([to_gpu(complete(9))])
    counts, res = tc.count_batched(b)
    assert counts.cpu().tolist() == [84] and res.T == 84


def test_batch_validate_rejects_ids_outside_their_graph(tc):
    # a local id beyond its graph's vertices: reported with validation, and
    # clamped into the graph without it (no access outside the buffers)
    b = tc.pack_csr([to_gpu(complete(5)), to_gpu(complete(4))])
    col = b.col.clone()
    col[3] = 7
    bad = tc.Batch(b.row_ptr, col, b.vtx_off, b.edge_off)
    with pytest.raises(tc.TCError) as e:
        tc.count_batched(bad, options=tc.Options(validate=True))
    assert e.value.code == -8
    counts, _ = tc.count_batched(bad)
    assert counts.numel() == 2
    rp = b.row_ptr.clone()
    rp[1] = 9   # row pointers of graph 0 no longer ascending
    with pytest.raises(tc.TCError) as e:
        tc.count_batched(tc.Batch(rp, b.col, b.vtx_off, b.edge_off), options=tc.Options(validate=True))
    assert e.value.code == -8


@pytest.mark.parametrize("cap", [1, 500, 4000])
def test_batch_in_groups(tc, cap):
    # groups of at most `cap` vertices and entries (a larger graph alone in
    # its group) give the same counts as one group
    gs = small_batch(5)
    b = tc.pack_csr([to_gpu(g) for g in gs])
    counts, res = tc.count_batched(b, options=tc.Options(batch_group_entries=cap))
    want = want_counts(gs)
    assert np.array_equal(counts.cpu().numpy(), want)
    assert res.T == int(want.sum())


def test_batch_from_union(tc):
    gs = small_batch(6)
    sizes = [g.n for g in gs]
    voff = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    src = np.concatenate([np.repeat(np.arange(g.n), np.diff(g.row_ptr)) + voff[i] for i, g in enumerate(gs)])
    dst = np.concatenate([g.col.astype(np.int64) + voff[i] for i, g in enumerate(gs)])
    rp, col = tc.build_csr(int(voff[-1]), dev(src), dev(dst))
    b = tc.Batch.from_union(rp, col, voff)
    ref = tc.pack_csr([to_gpu(g) for g in gs])
    assert torch.equal(b.row_ptr, ref.row_ptr) and torch.equal(b.col, ref.col)
    assert np.array_equal(b.edge_off, ref.edge_off)


def test_batch_plan_replays(tc):
    # the captured pipeline replayed three times, eager work (another count,
    # a device copy and a synchronisation) between the replays; every replay
    # equals the oracle's counts; a second plan over new buffer contents
    gs = small_batch(7)
    b = tc.pack_csr([to_gpu(g) for g in gs])
    want = want_counts(gs)
    plan = tc.BatchPlan(b, tc.Options(batch_group_entries=3000))
    other = small_batch(8)
    ob = tc.pack_csr([to_gpu(g) for g in other])
    for i in range(3):
        got = plan.launch().clone()
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy(), want), i
        oc, _ = tc.count_batched(ob)
        assert np.array_equal(oc.cpu().numpy(), want_counts(other))
        junk = torch.arange(1 << 20, device="cuda", dtype=torch.int32) * 3
        torch.cuda.synchronize()
        del junk
    plan.close()


# ---------------------------------------------------------------- full batch

def _golden():
    out = []
    with open(GOLDEN) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                i, kind, n, m, T = line.split()
                out.append((kind, int(n), int(m), int(T)))
    return out


@pytest.fixture(scope="module")
def full_batch(tc):
    t0 = time.time()
    rec = graphgen.batch_recipe(4096, seed=0)
    with cf.ThreadPoolExecutor(16) as ex:
        parts = list(ex.map(graphgen.batch_member_tuples, rec))
    sizes = np.array([p[0] for p in parts], dtype=np.int64)
    voff = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    src = torch.from_numpy(np.concatenate([p[1] + np.int32(voff[i]) for i, p in enumerate(parts)])).cuda()
    dst = torch.from_numpy(np.concatenate([p[2] + np.int32(voff[i]) for i, p in enumerate(parts)])).cuda()
    del parts
    rp, col = tc.build_csr(int(voff[-1]), src, dst)
    del src, dst
    b = tc.Batch.from_union(rp, col, voff)
    del rp, col
    print(f"\nbatch: {len(rec)} graphs, {int(voff[-1])} vertices, {b.col.numel() // 2} edges, "
          f"ready in {time.time() - t0:.1f} s", flush=True)
    yield rec, b
    del b
    torch.cuda.empty_cache()


def test_full_batch_every_graph(tc, full_batch):
    rec, b = full_batch
    gold = _golden()
    assert len(gold) == 4096
    assert [k for k, *_ in gold] == [r.kind for r in rec]
    assert np.array_equal(np.diff(b.vtx_off), [n for _, n, _, _ in gold])
    assert np.array_equal(np.diff(b.edge_off), [2 * m for _, _, m, _ in gold])
    want = np.array([T for *_, T in gold], dtype=np.int64)
    t0 = time.time()
    counts, res = tc.count_batched(b)
    print(f"eager batched count: T={res.T}, {time.time() - t0:.3f} s", flush=True)
    got = counts.cpu().numpy()
    bad = np.nonzero(got != want)[0]
    assert len(bad) == 0, f"{len(bad)} of 4096 graphs differ, first {bad[:5]}"
    assert res.T == int(want.sum())


def test_full_batch_levels_sampled(tc, full_batch):
    # the batched BFS levels of every 64th graph and the largest ones,
    # element by element against the oracle's serial BFS
    rec, b = full_batch
    lev, _ = tc.bfs_levels_batched(b)
    lev = lev.cpu().numpy()
    sizes = np.diff(b.edge_off)
    pick = sorted(set(range(0, 4096, 64)) | set(np.argsort(-sizes)[:8].tolist()))

    def check(i):
        n, s, d = graphgen.batch_member_tuples(rec[i])
        g = oracle.build_csr(n, s, d)
        olev, _ = oracle.bfs_levels(g)
        return i, bool(np.array_equal(lev[b.vtx_off[i]:b.vtx_off[i + 1]], olev))

    with cf.ThreadPoolExecutor(16) as ex:
        for i, ok in ex.map(check, pick):
            assert ok, (i, rec[i])


def test_full_batch_plan_every_graph(tc, full_batch):
    rec, b = full_batch
    want = np.array([T for *_, T in _golden()], dtype=np.int64)
    t0 = time.time()
    plan = tc.BatchPlan(b)
    t1 = time.time()
    for i in range(2):
        counts = plan.launch().clone()
        torch.cuda.synchronize()
        got = counts.cpu().numpy()
        assert np.array_equal(got, want), (i, np.nonzero(got != want)[0][:5])
    print(f"plan: capture {t1 - t0:.3f} s, replays equal the oracle", flush=True)
    plan.close()
