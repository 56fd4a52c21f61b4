"""GPU parity of the learned-schedule pieces against the float64 oracle:
initialisation (bit-exact), forward pass, gradient, Adam and training (to
float32 tolerances derived from the arithmetic), the schedule table (exact
where the oracle's choice is not a near-tie), the per-bucket profile (exact
integer element counts), and exact counts under learned and arbitrary
strategy tables."""
from __future__ import annotations

import numpy as np
import pytest

import graphgen
import oracle
from oracle import mlp
from _graphs import complete, gnp, wheel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2309_09064_amd as tc
    return tc


@pytest.fixture(scope="module")
def sched(tc):
    from paper_2309_09064_amd import sched
    return sched


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()


def to_gpu(g):
    return dev(g.row_ptr.astype(np.int32)), dev(g.col if g.nnz else np.zeros(0, np.int32))


def kron(scale, seed=1):
    n, s, d = graphgen.kronecker(scale, seed=seed)
    return oracle.build_csr(n, s, d)


def features(rows, seed):
    rng = np.random.default_rng(seed)
    return np.column_stack([rng.integers(0, 20, rows), rng.integers(0, 20, rows),
                            rng.integers(0, 2, rows)]).astype(np.float32)


def oracle_params(net):
    return mlp.unflatten(net.params.cpu().numpy().astype(np.float64), net.k, net.hidden)


# float32 forward: each output sums about H products of O(1) terms; 1e-4
# relative to the output scale leaves a wide margin over 2^-24 * H
def close(a, b, scale, rel=1e-4):
    return np.all(np.abs(np.asarray(a, np.float64) - b) <= rel * (1.0 + scale))


@pytest.mark.parametrize("H,K,seed", [(8, 4, 0), (32, 4, 7), (64, 8, 123), (16, 1, 2 ** 63 + 5)])
def test_init_bit_exact(sched, H, K, seed):
    net = sched.CostNet(H, K, seed=seed)
    got = net.params.cpu().numpy()
    want = mlp.init_he_uniform(K, H, seed)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


@pytest.mark.parametrize("H,K,rows", [(8, 4, 1), (32, 4, 257), (64, 8, 3000), (16, 3, 64)])
def test_forward(sched, H, K, rows):
    net = sched.CostNet(H, K, seed=H + K)
    X = features(rows, rows)
    y = net.forward(torch.from_numpy(X)).cpu().numpy()
    want, _ = mlp.forward(oracle_params(net), X.astype(np.float64))
    assert y.shape == (rows, K)
    assert close(y, want, np.abs(want).max())


@pytest.mark.parametrize("H,K,rows", [(8, 4, 40), (32, 4, 700)])
def test_weighted_gradient(sched, H, K, rows):
    net = sched.CostNet(H, K, seed=rows + 1)
    X = features(rows, rows + 3)
    rng = np.random.default_rng(rows + 4)
    c = rng.integers(0, K, rows).astype(np.int32)
    t = rng.normal(0, 3, rows).astype(np.float32)
    w = rng.uniform(0, 5, rows).astype(np.float32)
    w[::5] = 0.0
    loss, g = net.grad(X, c, t, w)
    L, grads = mlp.loss_and_grad(oracle_params(net), X.astype(np.float64), c, t.astype(np.float64),
                                 w.astype(np.float64))
    assert abs(loss - L) <= 1e-5 * (1 + L)
    for a, b in zip(mlp.unflatten(g.cpu().numpy(), K, H), grads):
        assert np.all(np.abs(a - b) <= 1e-4 * np.abs(b).max() + 1e-7)


@pytest.mark.parametrize("H,K,rows", [(8, 4, 17), (32, 4, 1000), (64, 8, 513)])
def test_gradient(sched, H, K, rows):
    net = sched.CostNet(H, K, seed=rows)
    X = features(rows, rows + 1)
    rng = np.random.default_rng(rows + 2)
    c = rng.integers(0, K, rows).astype(np.int32)
    c[::7] = -1          # rows outside [0, K) contribute nothing
    c[3::11] = K
    t = rng.normal(0, 3, rows).astype(np.float32)
    loss, g = net.grad(X, c, t)
    live = (c >= 0) & (c < K)
    L, grads = mlp.loss_and_grad(oracle_params(net), X[live].astype(np.float64), c[live], t[live].astype(np.float64))
    frac = live.sum() / rows   # the library divides by all rows
    assert abs(loss - L * frac) <= 1e-5 * (1 + L)
    got = mlp.unflatten(g.cpu().numpy(), K, H)
    for a, b in zip(got, grads):
        b = b * frac
        assert np.all(np.abs(a - b) <= 1e-4 * np.abs(b).max() + 1e-7)


def test_adam_steps(sched):
    H, K = 32, 4
    net = sched.CostNet(H, K, seed=5)
    ps = oracle_params(net)
    ms = [np.zeros_like(p) for p in ps]
    vs = [np.zeros_like(p) for p in ps]
    rng = np.random.default_rng(9)
    for step in range(1, 6):
        gflat = rng.normal(0, 1, net.count).astype(np.float32)
        gflat[::13] = 0.0
        net.adam(torch.from_numpy(gflat).cuda(), lr=0.01)
        mlp.adam_step(ps, mlp.unflatten(gflat.astype(np.float64), K, H), ms, vs, step, lr=0.01)
    got = mlp.unflatten(net.params.cpu().numpy(), K, H)
    for a, b in zip(got, ps):
        assert np.all(np.abs(a - b) <= 1e-5)


def test_training_matches_oracle_and_manual_steps(sched):
    H, K, rows = 16, 4, 400
    X = features(rows, 11)
    rng = np.random.default_rng(12)
    c = rng.integers(0, K, rows).astype(np.int32)
    t = (0.3 * X[:, 0] - 0.2 * X[:, 1] + c + rng.normal(0, 0.1, rows)).astype(np.float32)
    # one fused step vs the oracle
    net = sched.CostNet(H, K, seed=1)
    ps = oracle_params(net)
    losses = net.train(X, c, t, steps=1, lr=0.01)
    L, grads = mlp.loss_and_grad(ps, X.astype(np.float64), c, t.astype(np.float64))
    mlp.adam_step(ps, grads, [np.zeros_like(p) for p in ps], [np.zeros_like(p) for p in ps], 1, lr=0.01)
    assert abs(losses[0] - L) <= 1e-5 * (1 + L)
    for a, b in zip(mlp.unflatten(net.params.cpu().numpy(), K, H), ps):
        assert np.all(np.abs(a - b) <= 1e-5)
    # tc_mlp_train(20) is 20 gradient + Adam calls, bit for bit
    a = sched.CostNet(H, K, seed=2)
    b = sched.CostNet(H, K, seed=2)
    la = a.train(X, c, t, steps=20, lr=0.01)
    lb = []
    for _ in range(20):
        loss, g = b.grad(X, c, t)
        lb.append(loss)
        b.adam(g, lr=0.01)
    assert np.array_equal(a.params.cpu().numpy().view(np.uint32), b.params.cpu().numpy().view(np.uint32))
    assert np.array_equal(la, np.array(lb, np.float32))
    # loss trajectory vs the float64 oracle, and training reduces the loss
    ps = oracle_params(sched.CostNet(H, K, seed=2))
    ms = [np.zeros_like(p) for p in ps]
    vs = [np.zeros_like(p) for p in ps]
    ol = []
    for step in range(1, 21):
        L, grads = mlp.loss_and_grad(ps, X.astype(np.float64), c, t.astype(np.float64))
        ol.append(L)
        mlp.adam_step(ps, grads, ms, vs, step, lr=0.01)
    assert np.all(np.abs(la - ol) <= 1e-3 * (1 + np.abs(ol)))
    more = a.train(X, c, t, steps=500, lr=0.01)
    assert more[-1] < 0.2 * la[0]


@pytest.mark.parametrize("wave_slots,wg_slots,seed", [(0, 0, 3), (64, 1024, 4), (512, 8192, 5), (2048, 32768, 6)])
def test_schedule_table(tc, sched, wave_slots, wg_slots, seed):
    net = sched.CostNet(32, 4, seed=seed)
    opts = tc.Options(wave_slots=wave_slots, wg_slots=wg_slots)
    table, cost = net.schedule(opts, with_cost=True)
    table, cost = table.cpu().numpy(), cost.cpu().numpy()
    ws, gs = wave_slots or 2048, wg_slots or 32768
    want, y, gap, feas = mlp.schedule(oracle_params(net), int(np.log2(ws)) - 2)
    assert close(cost, y, np.abs(y).max())
    tol = 1e-4 * (1.0 + np.abs(y).max())
    clear = gap > 2 * tol
    assert np.array_equal(table[clear], want[clear])
    # near-ties: any feasible strategy within the tolerance of the best is correct
    for b in np.nonzero(~clear)[0]:
        s = table[b]
        assert feas[b, s] and y[b, s] <= y[b, want[b]] + 2 * tol
    assert clear.mean() > 0.9


@pytest.mark.parametrize("orientation", [0, 1])
def test_profile_elements_and_items(tc, orientation):
    g = kron(12, seed=4)
    lev, _ = oracle.bfs_levels(g)
    units, elements = oracle.bucket_work(g, lev, by_id=orientation == tc.TC_ORIENT_ID)
    rp, col = to_gpu(g)
    want_T = oracle.alg4(g, lev).T
    for s in range(4):
        prof = tc.new_profile()
        r = tc.count_profile(rp, col, prof, options=tc.Options(force_strategy=s, orientation=orientation))
        assert r.T == want_T
        p = prof.cpu().numpy()
        assert np.array_equal(p[:, :, 1].sum(axis=1), elements)
        assert p[:, :, 2].sum() == r.items
        assert np.all(p >= 0) and p[:, :, 0].sum() > 0
        used = p[:, :, 2].sum(axis=0) > 0
        # a forced strategy runs everywhere it is feasible; wavefront-hash
        # buckets too large for its tables go to the (slicing) workgroup hash
        allowed = {0: {0, 1}, 1: {1}, 2: {2}, 3: {3}}[s]
        assert set(np.nonzero(used)[0].tolist()) <= allowed
        assert used[s]


def test_profile_accumulates(tc):
    g = gnp(400, 0.05, 3)
    lev, _ = oracle.bfs_levels(g)
    _, elements = oracle.bucket_work(g, lev)
    rp, col = to_gpu(g)
    prof = tc.new_profile()
    c = tc.Counter(g.n, g.nnz, tc.Options(force_strategy=2))
    for _ in range(3):
        c(rp, col, profile=prof)
    assert np.array_equal(prof.cpu().numpy()[:, :, 1].sum(axis=1), 3 * elements)


def test_learned_schedule_counts_exactly(tc, sched):
    train = [to_gpu(kron(13, seed=s)) for s in (2, 3)]
    # the network's own table (verify=False): any table must count exactly
    table, net, ds, losses = sched.learn_schedule(train, steps=300, min_elements=1024, verify=False)
    assert len(ds.c) > 10 and losses[-1] < losses[0]
    t = table.cpu().numpy()
    assert t.shape == (2048,) and np.all((t >= 0) & (t < 4))
    for g in (kron(12, seed=7), gnp(300, 0.08, 5), complete(30), wheel(17)):
        rp, col = to_gpu(g)
        r = tc.count(rp, col, options=tc.Options(sched_table=table))
        assert r.T == oracle.alg4(g).T


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_arbitrary_tables_count_exactly(tc, seed):
    # any table, including hash choices the tables cannot hold, half-size
    # workgroup slices and out-of-range values, gives T
    rng = np.random.default_rng(seed)
    table = dev(rng.integers(-1, 9, 2048))
    for g in (kron(12, seed=seed), gnp(500, 0.04, seed)):
        rp, col = to_gpu(g)
        for opts in (tc.Options(sched_table=table), tc.Options(sched_table=table, wave_slots=64, wg_slots=1024)):
            r = tc.count(rp, col, options=opts)
            assert r.T == oracle.alg4(g).T
    bad = torch.zeros(2048, dtype=torch.int64, device="cuda")
    with pytest.raises(ValueError):
        tc.Options(sched_table=bad).to_c()


def test_schedule_table_entry_point(tc):
    # the effective table: forced strategies everywhere feasible, the
    # heuristic's three owner-size ranges, and a given table after feasibility
    t = tc.schedule_table(1000, 10000).cpu().numpy()
    ob = (np.arange(2048) >> 5) & 31
    # lane merges up to 31, wavefront tables (2048 slots) up to a quarter of
    # their slots
    assert np.all(t[ob <= 4] == 3) and np.all(t[(ob > 4) & (ob <= 8)] == 0) and np.all(t[ob > 8] == 1)
    t = tc.schedule_table(1000, 10000, tc.Options(merge_max_owner=15)).cpu().numpy()
    assert np.all(t[ob <= 3] == 3) and np.all(t[(ob > 3) & (ob <= 8)] == 0)
    t = tc.schedule_table(1000, 10000, tc.Options(wave_slots=1024)).cpu().numpy()
    assert np.all(t[ob <= 3] == 3) and np.all(t[ob == 4] == 0)
    t = tc.schedule_table(1000, 10000, tc.Options(force_strategy=0, wave_slots=64)).cpu().numpy()
    assert np.all(t[ob <= 4] == 0) and np.all(t[ob > 4] == 1)
    t = tc.schedule_table(1000, 10000, tc.Options(merge_max_owner=-1)).cpu().numpy()
    assert not np.any(t == 3)
    given = dev(np.full(2048, 0))
    t = tc.schedule_table(1000, 10000, tc.Options(sched_table=given, wave_slots=256)).cpu().numpy()
    assert np.all(t[ob <= 6] == 0) and np.all(t[ob > 6] == 1)
    # half-size workgroup slices (bit 2): kept only for the workgroup hash and
    # owners of at least half a slice (slices of 8192: classes 12 and up)
    for v in (5, 4, 7):
        t = tc.schedule_table(1 << 20, 1 << 24, tc.Options(sched_table=dev(np.full(2048, v)))).cpu().numpy()
        want = np.where(ob >= 12, 5, 1) if v == 5 else np.full(2048, v & 3)
        if v == 4:   # wavefront hash where it fits, else the workgroup hash
            want = np.where(ob <= 9, 0, np.where(ob >= 12, 5, 1))
        assert np.array_equal(t, want), v
    assert np.all(tc.schedule_table(1000, 10000, tc.Options(sched_table=dev(np.full(2048, 9)))).cpu().numpy() == 2)


def test_marginal_rows_and_counts(tc, sched):
    # the whole-pass measurement on a small graph: one row per (bucket,
    # alternative) plus one for the heuristic's own choice, targets consistent
    # with the measured changes, and exact counts under every trained table
    g = kron(14, seed=2)
    rp, col = to_gpu(g)
    lev, _ = tc.bfs_levels(rp, col)
    net, ms, losses, hull = sched.learn_marginal([(rp, col, lev)], steps=200, min_share=0.05, pairs=1)
    assert len(ms.c) >= 2 and losses[-1] < losses[0]
    heur = tc.schedule_table(g.n, g.nnz).cpu().numpy()
    own = ms.delta_ms == 0
    assert np.all(ms.c[own] == heur[ms.bucket[own]]) and np.all(ms.t[own] == 0)
    assert np.all(np.sign(ms.t[~own]) == np.sign(ms.delta_ms[~own]))
    assert np.all(ms.w >= 0.05 - 1e-6)
    table = sched.learned_table(net, g.n, g.nnz, hull, margin=0.0)
    outside = ~sched.inside_hull(hull)
    assert np.array_equal(table.cpu().numpy()[outside], heur[outside])
    T = oracle.alg4(g).T
    for t in (table, sched.learned_table(net, g.n, g.nnz, hull, margin=-100.0)):
        assert tc.Counter(g.n, g.nnz, tc.Options(sched_table=t))(rp, col, lev).T == T


def test_stored_network_on_a_held_out_graph(tc, sched):
    # the committed network (trained on Kronecker scale 22, seeds 2 and 3,
    # and Chung-Lu 2^20) on a graph it never saw: it changes the heuristic
    # only inside its training ranges, counts exactly, and its table is not
    # slower than the heuristic's beyond timing noise (alternating runs,
    # intersection pass by HIP events)
    import os
    path = os.path.join(os.path.dirname(sched.__file__), "sched_net.json")
    net, hull, margin, doc = sched.load_net(path)
    assert doc["rows"] > 0 and set(hull) <= {0, 1}
    g = kron(18, seed=11)
    rp, col = to_gpu(g)
    lev, _ = tc.bfs_levels(rp, col)
    veto = [tuple(c) for c in doc.get("veto", [])]
    table = sched.learned_table(net, g.n, g.nnz, hull, margin, veto=veto)
    heur = tc.schedule_table(g.n, g.nnz).cpu().numpy()
    t = table.cpu().numpy()
    assert not set(sched.changed_classes(heur, t)) & set(veto)
    assert np.all((t == heur) | sched.inside_hull(hull))
    assert tc.Counter(g.n, g.nnz, tc.Options(sched_table=table))(rp, col, lev).T == oracle.alg4(g).T
    if np.array_equal(t, heur):
        return
    ch = tc.Counter(g.n, g.nnz, tc.Options(timing=True))
    cl = tc.Counter(g.n, g.nnz, tc.Options(timing=True, sched_table=table))
    th, tl = [], []
    for _ in range(9):
        th.append(ch(rp, col, lev).ms["isect"])
        tl.append(cl(rp, col, lev).ms["isect"])
    print(f"\nlearned / heuristic {np.median(tl) / np.median(th):.3f} ({int((t != heur).sum())} buckets changed)")
    assert np.median(tl) < 1.05 * np.median(th)
