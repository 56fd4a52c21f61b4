"""GPU parity of the paper's variants on the same kernels: the cover-edge
count (Algorithm 3, CE) over full rows, the degree relabel (BaderD / CED
pre-pass) element by element against the oracle's, and the counts of the
relabelled graphs (BaderD = relabel + Algorithm 4, CED = relabel + CE)."""
from __future__ import annotations

import numpy as np
import pytest

import graphgen
import oracle
from test_gpu_parity import GRAPHS, graph, to_gpu, tc  # noqa: F401  (tc is a fixture)
from test_gpu_full import golden_counts

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", list(GRAPHS))
def test_cover_edge_count_matches_oracle(tc, name):
    g = graph(name)
    rp, col = to_gpu(g)
    r = tc.count_cover_edge(rp, col)
    lev, _ = oracle.bfs_levels(g)
    assert r.T == oracle.alg3(g, lev) == oracle.count_emd(g)
    assert r.T0 == 0 and r.T1 == r.T


@pytest.mark.parametrize("strategy", range(4), ids=["wave", "wg", "search", "merge"])
@pytest.mark.parametrize("name", ["k12", "union", "gnp", "kron11", "kron14", "er_dense", "chunglu14"])
def test_cover_edge_every_strategy(tc, name, strategy):
    g = graph(name)
    rp, col = to_gpu(g)
    assert tc.count_cover_edge(rp, col, None, tc.Options(force_strategy=strategy)).T == oracle.count_emd(g)


@pytest.mark.parametrize("cfg", [dict(wave_slots=64, wg_slots=1024), dict(wave_slots=64, wg_slots=1024, force_strategy=1),
                                 dict(merge_max_owner=31), dict(chunk_work=64, grid_blocks=3), dict(validate=True)],
                         ids=["small_tables", "sliced_wg", "lane_merge_wide", "tiny_chunks", "validate"])
@pytest.mark.parametrize("name", ["kron14", "chunglu14"])
def test_cover_edge_tiles_and_slices(tc, name, cfg):
    g = graph(name)
    rp, col = to_gpu(g)
    assert tc.count_cover_edge(rp, col, None, tc.Options(**cfg)).T == oracle.count_emd(g)


@pytest.mark.parametrize("kind", ["zero", "half"])
def test_cover_edge_given_levels(tc, kind):
    # any levels with |L(u) - L(v)| <= 1 on every edge cover every triangle
    g = graph("kron14")
    lev, _ = oracle.bfs_levels(g)
    levels = np.zeros(g.n, np.int32) if kind == "zero" else (lev // 2).astype(np.int32)
    rp, col = to_gpu(g)
    r = tc.count_cover_edge(rp, col, torch.from_numpy(levels).cuda())
    assert r.T == oracle.alg3(g, levels) == oracle.count_emd(g)


def check_relabel(tc, g):
    rp, col = to_gpu(g)
    rp2, col2, perm = tc.relabel_by_degree(rp, col)
    h, operm = oracle.relabel_degree(g)
    assert np.array_equal(perm.cpu().numpy(), operm)
    assert np.array_equal(rp2.cpu().numpy(), h.row_ptr.astype(np.int32))
    assert np.array_equal(col2.cpu().numpy(), h.col)
    return rp2, col2, h


@pytest.mark.parametrize("name", list(GRAPHS))
def test_relabel_matches_oracle(tc, name):
    g = graph(name)
    rp2, col2, h = check_relabel(tc, g)
    T = oracle.count_emd(g)
    assert tc.count(rp2, col2).T == T                  # BaderD
    assert tc.count_cover_edge(rp2, col2).T == T       # CED


def test_relabel_and_variants_full_kronecker_scale20(tc):
    n, s, d = graphgen.kronecker(20, 16, seed=1)
    rp, col = tc.build_csr(n, torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda())
    print(f"\nkronecker20 variants: n={n} nnz={col.numel()}", flush=True)
    g = oracle.as_csr(n, rp.cpu().numpy().astype(np.int64), col.cpu().numpy())
    rp2, col2, h = check_relabel(tc, g)
    T = golden_counts()["kronecker20"][2]
    assert tc.count_cover_edge(rp, col).T == T
    r = tc.count(rp2, col2)
    assert r.T == T
    lev2, _ = oracle.bfs_levels(h)
    ores = oracle.alg4(h, lev2)
    assert (r.T0, r.T1, r.e0) == (ores.T0, ores.T1, ores.E0)
    assert tc.count_cover_edge(rp2, col2).T == T
