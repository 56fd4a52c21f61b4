"""Full-size parity on the large configurations: Kronecker scale 24 and the
Chung-Lu power-law graph with n = 2^22.  The oracle computes the BFS levels
and the partition of these graphs in seconds, so those are compared element
by element.  The oracle's count of a graph this size takes minutes to most
of an hour, so its T, T0, T1 and |E0| are stored in tests/golden/
large_counts.txt (written by tests/golden/make_large_counts.py, which calls
the oracle only) and compared bit for bit; the count is also checked through
properties that hold at any size: T is the same for every valid level
assignment (the cover-edge argument: any L with |L(u) - L(v)| <= 1 on every
edge), for every forced strategy, T = T0 + T1, |E0| equals the horizontal
edges of the levels, and L = 0 (every edge horizontal) gives T1 = 0."""

from __future__ import annotations

import os

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


def _graph(tc, which):
    if which == "kronecker24":
        n, s, d = graphgen.kronecker(24, 16, seed=1)
    else:
        n, s, d = graphgen.chung_lu(1 << 22, 2.1, 32.0, float(1 << 17), seed=1)
    rp, col = tc.build_csr(n, torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda())
    print(f"\n{which}: n={n} m={col.numel() // 2}", flush=True)
    return n, rp, col


@pytest.fixture(scope="module", params=["kronecker24", "chunglu22"])
def big(tc, request):
    n, rp, col = _graph(tc, request.param)
    host = oracle.as_csr(n, rp.cpu().numpy().astype(np.int64), col.cpu().numpy())
    yield request.param, n, rp, col, host
    del rp, col
    torch.cuda.empty_cache()


def test_levels_and_partition_full(tc, big):
    name, n, rp, col, g = big
    lev, nlev = tc.bfs_levels(rp, col)
    olev, _ = oracle.bfs_levels(g)
    assert np.array_equal(lev.cpu().numpy(), olev)
    assert nlev == int(olev.max()) + 1
    part = tc.partition(rp, col, lev)
    op = oracle.partition(g, olev)
    assert np.array_equal(part["rp0"].cpu().numpy(), op.rp0.astype(np.int32))
    assert np.array_equal(part["up0"].cpu().numpy(), op.up0)
    assert np.array_equal(part["rp1"].cpu().numpy(), op.rp1.astype(np.int32))
    e0x2 = int(op.rp0[-1])
    assert np.array_equal(part["c0"][:e0x2].cpu().numpy(), op.c0)
    assert np.array_equal(part["c1"][:g.nnz - e0x2].cpu().numpy(), op.c1)
    assert part["e0"] * 2 == e0x2


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "large_counts.txt")
GOLDEN_NAME = {"kronecker24": "kronecker24", "chunglu22": "chunglu22"}


def golden_counts():
    out = {}
    with open(GOLDEN) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                name, n, m, T, T0, T1, e0 = line.split()
                out[name] = tuple(int(v) for v in (n, m, T, T0, T1, e0))
    return out


def test_count_properties_full(tc, big):
    name, n, rp, col, g = big
    lev, _ = tc.bfs_levels(rp, col)
    base = tc.count(rp, col)
    gn, gm, gT, gT0, gT1, ge0 = golden_counts()[GOLDEN_NAME[name]]
    assert (n, g.nnz // 2) == (gn, gm)
    assert (base.T, base.T0, base.T1, base.e0) == (gT, gT0, gT1, ge0)
    assert base.T == base.T0 + base.T1 and base.T1 > 0
    # |E0| from the levels, on the host
    deg = np.diff(g.row_ptr)
    u = np.repeat(np.arange(n, dtype=np.int32), deg)
    lh = lev.cpu().numpy()
    assert base.e0 * 2 == int(np.count_nonzero(lh[u] == lh[g.col]))
    del u
    # other valid level assignments: floor(L / 2) and L = 0
    half = torch.div(lev, 2, rounding_mode="floor").contiguous()
    zero = torch.zeros_like(lev)
    r_half = tc.count(rp, col, half)
    r_zero = tc.count(rp, col, zero)
    assert r_half.T == base.T and r_zero.T == base.T
    assert r_zero.T1 == 0 and r_zero.e0 == g.nnz // 2
    for s in (0, 1, 2):
        assert tc.count(rp, col, lev, tc.Options(force_strategy=s)).T == base.T
    print(f"{name}: T={base.T} T0={base.T0} T1={base.T1} |E0|={base.e0}", flush=True)
