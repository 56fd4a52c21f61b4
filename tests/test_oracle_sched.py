"""Pins of the oracle's schedule pieces (not in the paper; the network only
picks among exact kernels): the SplitMix64 generator against its published
outputs, the He-uniform initialisation against its distribution, the
schedule choice against hand-built networks with known costs, and the
per-bucket work split against closed forms and an edge-by-edge recount."""
from __future__ import annotations

import itertools

import numpy as np
import pytest

import oracle
from oracle import mlp

from _graphs import complete, complete_bipartite, csr_from_edges, gnp, wheel


def test_splitmix64_published_outputs():
    # the first three outputs of the reference SplitMix64 seeded with 0
    assert mlp.splitmix64_at(0, [0, 1, 2]).tolist() == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                                        0x06C45D188009454F]


def test_splitmix64_counter_is_stateless():
    # output i of a stream started at seed s is output 0 of a stream started
    # at s + i * golden
    for i in (1, 7, 1000):
        a = mlp.splitmix64_at(12345, [i])[0]
        b = mlp.splitmix64_at((12345 + i * mlp.GOLDEN) % (1 << 64), [0])[0]
        assert a == b


@pytest.mark.parametrize("K,H", [(4, 8), (4, 32), (8, 64)])
def test_he_uniform_init_distribution(K, H):
    flat = mlp.init_he_uniform(K, H, seed=3)
    assert flat.dtype == np.float32
    ps = mlp.unflatten(flat, K, H)
    for p, fan_in in zip(ps[0::2], (3, H, H)):
        bound = np.sqrt(6.0 / fan_in)
        assert np.all(np.abs(p) <= bound * (1 + 1e-7))
        if p.size >= 1000:   # He: variance 2 / fan_in; uniform on [-b, b] has b^2 / 3
            assert abs(p.var() / (2.0 / fan_in) - 1.0) < 0.1
            assert abs(p.mean()) < 0.1 * bound
    for b in ps[1::2]:
        assert np.all(b == 0)
    assert np.array_equal(flat, mlp.init_he_uniform(K, H, seed=3))
    assert not np.array_equal(flat, mlp.init_he_uniform(K, H, seed=4))


def _const_net(costs, H=8):
    K = len(costs)
    ps = [np.zeros(s) for s in mlp.param_shapes(K, H)]
    ps[5] = np.asarray(costs, dtype=np.float64)
    return ps


def _expect(pref, wave_ob_max):
    """Cheapest feasible by a preference order, per bucket."""
    out = np.zeros(2048, np.int32)
    for b in range(2048):
        ob = (b >> 5) & 31
        feas = {0: ob <= wave_ob_max, 1: True, 2: True, 3: True}
        out[b] = next(s for s in pref if feas[s])
    return out


@pytest.mark.parametrize("wave", [9, 4, 0])
def test_schedule_constant_costs(wave):
    t, y, gap, feas = mlp.schedule(_const_net([0.0, 1.0, 2.0, 3.0]), wave)
    assert np.array_equal(t, _expect([0, 1, 2, 3], wave))
    assert np.array_equal(np.nonzero(t == 0)[0], np.nonzero(((np.arange(2048) >> 5) & 31) <= wave)[0])
    t, *_ = mlp.schedule(_const_net([3.0, 2.0, 1.0, 0.0]), wave)
    assert np.all(t == 3)
    t, *_ = mlp.schedule(_const_net([1.0, 1.0, 1.0, 1.0]), wave)   # ties: lowest number
    assert np.array_equal(t, _expect([0, 1, 2, 3], wave))
    t, *_ = mlp.schedule(_const_net([0.5, 5.0, 1.0, 2.0]), wave)
    assert np.array_equal(t, _expect([0, 2, 3, 1], wave))


def test_schedule_cost_growing_with_owner_class():
    # y0 = ob (through both hidden layers), y2 = 5, y1 = y3 = 100: the
    # wavefront hash wins below class 5, ties at 5 (lower number), search above
    H, K = 8, 4
    ps = [np.zeros(s) for s in mlp.param_shapes(K, H)]
    ps[0][0] = [1.0, 0.0, 0.0]
    ps[2][0, 0] = 1.0
    ps[4][0, 0] = 1.0
    ps[5][:] = [0.0, 100.0, 5.0, 100.0]
    t, y, gap, _ = mlp.schedule(ps, 31)
    ob = (np.arange(2048) >> 5) & 31
    assert np.allclose(y[:, 0], ob)
    assert np.array_equal(t, np.where(ob <= 5, 0, 2))
    assert np.all(gap[ob == 5] == 0)


def test_bucket_work_complete_graph():
    # K_n with root 0: level 1 holds K_{n-1} on ids 1..n-1 (equal degrees, so
    # rank = id); |N0+(x)| = n-1-x; |N1(x)| = 1 (the root)
    n = 9
    g = complete(n)
    lev, _ = oracle.bfs_levels(g)
    units, elements = oracle.bucket_work(g, lev)
    eu, ee = np.zeros(2048, np.int64), np.zeros(2048, np.int64)
    for x in range(1, n - 1):          # kind 0: x owns y in (x, n-2] (y = n-1 has an empty list)
        cnt = n - 2 - x
        if cnt == 0:
            continue
        work = sum(n - 1 - y for y in range(x + 1, n - 1))
        sx = n - 1 - x
        b = (0 * 32 + (sx.bit_length() - 1)) * 32 + max(work // cnt, 1).bit_length() - 1
        eu[b] += 1
        ee[b] += work + sx
    for x in range(2, n):              # kind 1: equal sizes, the larger id owns
        eu[(1 * 32 + 0) * 32 + 0] += 1
        ee[(1 * 32 + 0) * 32 + 0] += (x - 1) + 1
    assert np.array_equal(units, eu)
    assert np.array_equal(elements, ee)


@pytest.mark.parametrize("n", [5, 8, 13])
def test_bucket_work_wheel(n):
    # hub 0 at level 0, rim 1..n-1 at level 1, rim degrees all 3 (rank = id)
    g = wheel(n)
    lev, _ = oracle.bfs_levels(g)
    units, elements = oracle.bucket_work(g, lev)
    b000, b010, b100 = 0, 1 * 32, (1 * 32) * 32
    # kind 0: N0+(1) = {2, n-1}, N0+(i) = {i+1} for 2 <= i <= n-2, N0+(n-1) = {}
    # owners: 1 (partner 2), and i+1 for 2 <= i <= n-3 (partner i)
    # kind 1: every rim list is {0}; larger ids own; n-1 owns both 1 and n-2
    assert units[b010] == 1 and elements[b010] == 1 + 2
    assert units[b000] == n - 4 and elements[b000] == 2 * (n - 4)
    assert units[b100] == n - 2 and elements[b100] == 2 * (n - 3) + 3
    assert units.sum() == 1 + (n - 4) + (n - 2)


def test_bucket_work_bipartite_is_empty():
    g = complete_bipartite(5, 7)
    lev, _ = oracle.bfs_levels(g)
    units, elements = oracle.bucket_work(g, lev)
    assert units.sum() == 0 and elements.sum() == 0


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_bucket_work_totals_by_edges(seed):
    # recount edge by edge: every horizontal edge with both lists non-empty
    # streams its smaller list once; every owner hashes its list once
    g = gnp(60, 0.15, seed)
    lev, _ = oracle.bfs_levels(g)
    units, elements = oracle.bucket_work(g, lev)
    deg = g.degrees()
    nb = [set(g.col[g.row_ptr[v]:g.row_ptr[v + 1]].tolist()) for v in range(g.n)]
    rank = lambda v: (deg[v], v)
    s0 = [sum(1 for w in nb[v] if lev[w] == lev[v] and rank(w) > rank(v)) for v in range(g.n)]
    s1 = [sum(1 for w in nb[v] if lev[w] != lev[v]) for v in range(g.n)]
    total, owners = 0, set()
    for u, v in itertools.combinations(range(g.n), 2):
        if v not in nb[u] or lev[u] != lev[v]:
            continue
        for k, s in enumerate((s0, s1)):
            if min(s[u], s[v]) == 0:
                continue
            o = u if (s[u], u) > (s[v], v) else v
            total += min(s[u], s[v])
            owners.add((o, k))
    total += sum((s0, s1)[k][o] for o, k in owners)
    assert elements.sum() == total
    assert units.sum() == len(owners)
