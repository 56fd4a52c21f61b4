"""The autotuner on the GPU: the tuned options are never slower than the
defaults on the tuning graph (the defaults are one of the candidates), the
counts under them stay exact, and the cache returns the same options."""
from __future__ import annotations

import numpy as np
import pytest

import graphgen
import oracle

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


def test_tune_graph_and_cache(tc, tmp_path):
    from paper_2309_09064_amd import autotune
    n, s, d = graphgen.kronecker(16, seed=5)
    g = oracle.build_csr(n, s, d)
    rp, col = dev(g.row_ptr), dev(g.col)
    space = {"chunk_work": [8192, 16384, 65536], "wave_slots": [1024, 2048], "wg_slots": [16384, 32768],
             "grid_blocks": [0, 256]}
    cache = autotune.Cache(str(tmp_path / "tune.json"))
    opts, rep = autotune.tune(rp, col, space=space, repeats=2, cache=cache)
    assert rep["best_ms"] <= rep["default_ms"]
    want = oracle.alg4(g).T
    assert tc.count(rp, col, options=opts).T == want
    again = autotune.tuned_options(rp, col, cache=autotune.Cache(cache.path), tune_if_missing=False)
    assert all(getattr(again, k) == getattr(opts, k) for k in autotune.TUNED_FIELDS)


def test_tuned_batch_counts_exact(tc, tmp_path):
    from paper_2309_09064_amd import autotune
    gs = []
    for i in range(12):
        n, s, d = graphgen.kronecker(8 + i % 5, seed=50 + i)
        gs.append(oracle.build_csr(n, s, d))
    # tuned on the disjoint union (one graph with global ids), applied to the
    # packed batch
    voff = np.concatenate([[0], np.cumsum([g.n for g in gs])]).astype(np.int64)
    urp = np.concatenate([[0], np.cumsum(np.concatenate([np.diff(g.row_ptr) for g in gs]))])
    ucol = np.concatenate([g.col.astype(np.int64) + voff[i] for i, g in enumerate(gs)])
    opts, _ = autotune.tune(dev(urp), dev(ucol), space={"chunk_work": [4096, 16384], "wave_slots": [512, 2048],
                                                        "wg_slots": [32768], "grid_blocks": [0]}, repeats=1)
    counts, _ = tc.count_batched(tc.pack_csr([(dev(g.row_ptr), dev(g.col)) for g in gs]), options=opts)
    assert counts.cpu().tolist() == [oracle.alg4(g).T for g in gs]
