"""GPU parity of the per-edge triangle counts (support, tc_edge_support)
against the oracle, entry by entry: every small graph of the parity set,
every forced strategy, tile and slicing configurations, given level
assignments, and the full scale-20 Kronecker graph through checksums of the
oracle's vector (tests/golden/edge_checksums.txt) plus sampled entries
computed one at a time by the oracle."""
from __future__ import annotations

import os

import numpy as np
import pytest

import graphgen
import oracle
from test_gpu_parity import GRAPHS, graph, to_gpu, tc  # noqa: F401  (tc is a fixture)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "edge_checksums.txt")


def check_edge(tc, g, options=None, levels=None):
    rp, col = to_gpu(g)
    lev = None if levels is None else torch.from_numpy(np.ascontiguousarray(levels, dtype=np.int32)).cuda()
    sup, r = tc.edge_support(rp, col, lev, options)
    want = oracle.edge_support(g)
    got = sup.cpu().numpy().view(np.uint32)
    assert got.shape == (g.nnz,)
    assert np.array_equal(got, want), np.nonzero(got != want)[0][:10]
    assert 6 * r.T == int(want.sum(dtype=np.uint64)) and r.T == r.T0 + r.T1
    return r


@pytest.mark.parametrize("name", list(GRAPHS))
def test_edge_support_matches_oracle(tc, name):
    g = graph(name)
    r = check_edge(tc, g)
    assert r.T == oracle.count_emd(g)


@pytest.mark.parametrize("strategy", range(4), ids=["wave", "wg", "search", "merge"])
@pytest.mark.parametrize("name", ["k12", "union", "gnp", "kron11", "kron14", "er_dense", "chunglu14"])
def test_edge_support_every_strategy(tc, name, strategy):
    check_edge(tc, graph(name), tc.Options(force_strategy=strategy))


@pytest.mark.parametrize("cfg", [dict(wave_slots=64, wg_slots=1024), dict(wave_slots=64, wg_slots=1024, force_strategy=1),
                                 dict(merge_max_owner=31), dict(merge_max_owner=-1), dict(chunk_work=64, grid_blocks=3),
                                 dict(validate=True)],
                         ids=["small_tables", "sliced_wg", "lane_merge_wide", "no_merge", "tiny_chunks", "validate"])
@pytest.mark.parametrize("name", ["kron14", "chunglu14"])
def test_edge_support_tiles_and_slices(tc, name, cfg):
    check_edge(tc, graph(name), tc.Options(**cfg))


@pytest.mark.parametrize("kind", ["zero", "half"])
def test_edge_support_given_levels(tc, kind):
    g = graph("kron14")
    lev, _ = oracle.bfs_levels(g)
    levels = np.zeros(g.n, np.int32) if kind == "zero" else (lev // 2).astype(np.int32)
    r = check_edge(tc, g, levels=levels)
    if kind == "zero":
        assert r.T1 == 0


def test_edge_support_no_edges(tc):
    rp = torch.zeros(6, dtype=torch.int32, device="cuda")
    col = torch.zeros(0, dtype=torch.int32, device="cuda")
    sup, r = tc.edge_support(rp, col)
    assert sup.numel() == 0 and r.T == 0


def test_edge_support_repeated_calls_start_from_zero(tc):
    g = graph("kron11")
    rp, col = to_gpu(g)
    a, _ = tc.edge_support(rp, col)
    b, _ = tc.edge_support(rp, col)
    assert torch.equal(a, b)


def golden_checksums():
    out = {}
    with open(GOLDEN) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                name, *vals = line.split()
                out[name] = tuple(int(v) for v in vals)
    return out


def test_edge_support_full_kronecker_scale20(tc):
    from golden.make_vertex_checksums import checksums
    n, s, d = graphgen.kronecker(20, 16, seed=1)
    rp, col = tc.build_csr(n, torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda())
    print(f"\nkronecker20 per-edge: n={n} nnz={col.numel()}", flush=True)
    sup, r = tc.edge_support(rp, col)
    got = sup.cpu().numpy().view(np.uint32)
    gnnz, gsum, gs1, gs2, gmax, garg = golden_checksums()["kronecker20"]
    assert got.shape == (gnnz,)
    assert int(got.sum(dtype=np.uint64)) == gsum == 6 * r.T
    assert checksums(got) == (gs1, gs2, gmax, garg)
    g = oracle.as_csr(n, rp.cpu().numpy().astype(np.int64), col.cpu().numpy())
    rng = np.random.default_rng(21)
    es = rng.choice(g.nnz, 4000, replace=False)
    assert np.array_equal(got[es], oracle.edge_support_at(g, es))
    for opt in (tc.Options(force_strategy=2), tc.Options(force_strategy=3)):
        sup2, _ = tc.edge_support(rp, col, None, opt)
        assert torch.equal(sup2, sup)
    sup3, r3 = tc.edge_support(rp, col, torch.zeros(n, dtype=torch.int32, device="cuda"))
    assert torch.equal(sup3, sup) and r3.T1 == 0
