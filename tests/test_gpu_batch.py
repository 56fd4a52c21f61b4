"""GPU parity of the batched count: per-graph counts of a packed batch equal
the oracle's count of each graph on its own, for small mixed batches (every
graph checked, empty members included) and for the full 4096-graph batch of
Erdos-Renyi and Kronecker members (a sample of graphs checked one by one,
the largest among them, plus the total)."""
from __future__ import annotations

import concurrent.futures as cf
import time

import numpy as np
import pytest

import graphgen
import oracle
from _graphs import complete, csr_from_edges, cycle, gnp, petersen, random_tree, wheel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("seed", [1, 2])
def test_small_batch_every_graph(tc, seed):
    gs = small_batch(seed)
    rp, col, off = tc.pack_csr([to_gpu(g) for g in gs])
    counts, res = tc.count_batched(rp, col, off, options=tc.Options(validate=True))
    want = np.array([oracle.alg4(g).T if g.n else 0 for g in gs], dtype=np.int64)
    assert np.array_equal(counts.cpu().numpy(), want)
    assert res.T == int(want.sum())


@pytest.mark.parametrize("force", [0, 1, 2, 3])
def test_batch_strategy_invariance(tc, force):
    gs = small_batch(3)
    rp, col, off = tc.pack_csr([to_gpu(g) for g in gs])
    counts, _ = tc.count_batched(rp, col, off, options=tc.Options(force_strategy=force))
    want = np.array([oracle.alg4(g).T if g.n else 0 for g in gs], dtype=np.int64)
    assert np.array_equal(counts.cpu().numpy(), want)


def test_batch_with_given_levels_and_repeat(tc):
    gs = small_batch(4)
    rp, col, off = tc.pack_csr([to_gpu(g) for g in gs])
    lev, _ = tc.bfs_levels(rp, col)
    a, _ = tc.count_batched(rp, col, off, levels=lev)
    b, _ = tc.count_batched(rp, col, off)
    assert torch.equal(a, b)


def test_batch_all_empty_and_single(tc):
    rp, col, off = tc.pack_csr([to_gpu(csr_from_edges(0, [])), to_gpu(csr_from_edges(3, []))])
    counts, res = tc.count_batched(rp, col, off)
    assert counts.cpu().tolist() == [0, 0] and res.T == 0
    g = complete(9)
    rp, col, off = tc.pack_csr([to_gpu(g)])
    counts, res = tc.count_batched(rp, col, off)
    assert counts.cpu().tolist() == [84] and res.T == 84


def test_batch_validate_rejects_cross_edges(tc):
    g = complete(10)
    rp, col = to_gpu(g)
    with pytest.raises(tc.TCError) as e:
        tc.count_batched(rp, col, np.array([0, 5, 10]), options=tc.Options(validate=True))
    assert e.value.code == -8


# ---------------------------------------------------------------- full batch

def _member(mem):
    n, s, d = graphgen.batch_member_tuples(mem)
    return n, s, d


@pytest.fixture(scope="module")
def full_batch():
    t0 = time.time()
    rec = graphgen.batch_recipe(4096, seed=0)
    with cf.ThreadPoolExecutor(16) as ex:
        parts = list(ex.map(_member, rec))
    sizes = np.array([p[0] for p in parts], dtype=np.int64)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    src = np.concatenate([p[1] + np.int32(off[i]) for i, p in enumerate(parts)])
    dst = np.concatenate([p[2] + np.int32(off[i]) for i, p in enumerate(parts)])
    print(f"\nbatch: {len(rec)} graphs, {int(off[-1])} vertices, {len(src)} tuples, "
          f"generated in {time.time() - t0:.1f} s", flush=True)
    return rec, parts, off, src, dst


def test_full_batch_sampled(tc, full_batch):
    rec, parts, off, src, dst = full_batch
    n = int(off[-1])
    rp, col = tc.build_csr(n, torch.from_numpy(src).cuda(), torch.from_numpy(dst).cuda())
    t0 = time.time()
    counts, res = tc.count_batched(rp, col, off)
    torch.cuda.synchronize()
    print(f"batched count: m={col.numel() // 2}, T={res.T}, {time.time() - t0:.3f} s", flush=True)
    counts = counts.cpu().numpy()
    assert int(counts.sum()) == res.T
    # every 16th graph plus the eight largest of each half, each against the oracle on its own
    sizes = np.diff(off)
    pick = set(range(0, 4096, 16))
    pick |= set(np.argsort(-sizes[:2048])[:8].tolist()) | set((2048 + np.argsort(-sizes[2048:])[:8]).tolist())

    def want(i):
        nn, s, d = parts[i]
        return i, oracle.alg4(oracle.build_csr(nn, s, d)).T

    with cf.ThreadPoolExecutor(16) as ex:
        for i, t in ex.map(want, sorted(pick)):
            assert counts[i] == t, (i, rec[i], counts[i], t)
