"""GPU parity of the per-vertex triangle counts t(v) (tc_vertex_triangles)
against the oracle, element by element: every small graph of the parity
set, every forced strategy, the tile and slicing configurations, given
level assignments, and the full scale-20 Kronecker graph through checksums
of the oracle's vector (tests/golden/vertex_checksums.txt) plus sampled
vertices computed one by one by the oracle's second definition."""
from __future__ import annotations

import os

import numpy as np
import pytest

import graphgen
import oracle
from test_gpu_parity import GRAPHS, graph, to_gpu, tc  # noqa: F401  (tc is a fixture)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "vertex_checksums.txt")


def check_vertex(tc, g, options=None, levels=None):
    rp, col = to_gpu(g)
    lev = None if levels is None else torch.from_numpy(np.ascontiguousarray(levels, dtype=np.int32)).cuda()
    tv, r = tc.vertex_triangles(rp, col, lev, options)
    want = oracle.vertex_triangles(g)
    got = tv.cpu().numpy().view(np.uint64)
    assert got.shape == (g.n,)
    assert np.array_equal(got, want), np.nonzero(got != want)[0][:10]
    assert r.T == int(want.sum()) // 3 and r.T == r.T0 + r.T1
    return r


@pytest.mark.parametrize("name", list(GRAPHS))
def test_vertex_triangles_match_oracle(tc, name):
    g = graph(name)
    r = check_vertex(tc, g)
    assert r.T == oracle.count_emd(g)


@pytest.mark.parametrize("strategy", range(4), ids=["wave", "wg", "search", "merge"])
@pytest.mark.parametrize("name", ["k12", "union", "gnp", "kron11", "kron14", "er_dense", "chunglu14"])
def test_vertex_triangles_every_strategy(tc, name, strategy):
    check_vertex(tc, graph(name), tc.Options(force_strategy=strategy))


@pytest.mark.parametrize("cfg", [dict(wave_slots=64, wg_slots=1024), dict(wave_slots=64, wg_slots=1024, force_strategy=1),
                                 dict(merge_max_owner=31), dict(merge_max_owner=-1), dict(chunk_work=64, grid_blocks=3)],
                         ids=["small_tables", "sliced_wg", "lane_merge_wide", "no_merge", "tiny_chunks"])
@pytest.mark.parametrize("name", ["kron14", "chunglu14"])
def test_vertex_triangles_tiles_and_slices(tc, name, cfg):
    check_vertex(tc, graph(name), tc.Options(**cfg))


@pytest.mark.parametrize("kind", ["zero", "half"])
def test_vertex_triangles_given_levels(tc, kind):
    g = graph("kron14")
    lev, _ = oracle.bfs_levels(g)
    levels = np.zeros(g.n, np.int32) if kind == "zero" else (lev // 2).astype(np.int32)
    r = check_vertex(tc, g, levels=levels)
    if kind == "zero":
        assert r.T1 == 0


def test_vertex_triangles_empty_graph(tc):
    rp = torch.zeros(1, dtype=torch.int32, device="cuda")
    col = torch.zeros(0, dtype=torch.int32, device="cuda")
    tv, r = tc.vertex_triangles(rp, col)
    assert tv.numel() == 0 and r.T == 0


def test_vertex_triangles_repeated_calls_start_from_zero(tc):
    g = graph("kron11")
    rp, col = to_gpu(g)
    a, _ = tc.vertex_triangles(rp, col)
    b, _ = tc.vertex_triangles(rp, col)
    assert torch.equal(a, b)


def golden_checksums():
    out = {}
    with open(GOLDEN) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                name, *vals = line.split()
                out[name] = tuple(int(v) for v in vals)
    return out


def test_vertex_triangles_full_kronecker_scale20(tc):
    from golden.make_vertex_checksums import checksums
    n, s, d = graphgen.kronecker(20, 16, seed=1)
    rp, col = tc.build_csr(n, torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda())
    print(f"\nkronecker20 per-vertex: n={n} nnz={col.numel()}", flush=True)
    tv, r = tc.vertex_triangles(rp, col)
    got = tv.cpu().numpy().view(np.uint64)
    gn, gsum, gs1, gs2, gmax, garg = golden_checksums()["kronecker20"]
    assert got.shape == (gn,)
    assert int(got.sum()) == gsum == 3 * r.T
    assert checksums(got) == (gs1, gs2, gmax, garg)
    # sampled vertices, one at a time, by the oracle's second definition
    g = oracle.as_csr(n, rp.cpu().numpy().astype(np.int64), col.cpu().numpy())
    deg = g.degrees()
    rng = np.random.default_rng(20)
    cand = np.nonzero((deg > 0) & (deg <= 2048))[0]
    vs = np.concatenate([rng.choice(cand, 1500, replace=False), cand[np.argsort(deg[cand])[-20:]]])
    assert np.array_equal(got[vs], oracle.vertex_triangles_at(g, vs))
    # the same vector under other schedules and levels
    for opt in (tc.Options(force_strategy=2), tc.Options(force_strategy=3)):
        tv2, _ = tc.vertex_triangles(rp, col, None, opt)
        assert torch.equal(tv2, tv)
    tv3, r3 = tc.vertex_triangles(rp, col, torch.zeros(n, dtype=torch.int32, device="cuda"))
    assert torch.equal(tv3, tv) and r3.T1 == 0
