"""Learned schedule: measurements, cost network, per-bucket strategy table.

Not part of the paper's method.  Every strategy counts exactly, so the
schedule only decides speed.  Two ways to train the network are here:

Whole-pass marginal costs (the one the stored network uses):

1. ``collect_marginal``: per bucket with enough work and per alternative
   action (a strategy, or the workgroup hash with half-size slices), the
   change in the bucketing + intersection time when only that bucket
   switches, measured in paired runs.
2. ``learn_marginal``: training rows (features (ob, pb, kind), action,
   sign(t) log2(1 + |t|) of the change per element), full-batch Adam on the
   device (``tc_mlp_train``).
3. ``learned_table``: per bucket the cheapest feasible action by the
   network's prediction (``tc_mlp_forward``), kept only inside the training
   ranges, beyond a margin and outside vetoed classes of change.
4. ``verify_schedule``: the classes of change (heuristic strategy ->
   proposed action) are tried one at a time on the training graphs and
   vetoed where they do not pay; ``save_net`` / ``load_net`` store the
   network with its ranges, margin and vetoes.

Per-bucket wave-tick profiles (the earlier signal, kept and tested):
``collect_profile`` runs the instrumented kernels (``tc_count_profile``),
``dataset`` turns the ticks per element into rows, ``learn_schedule`` trains
and schedules with ``tc_mlp_schedule``.  Ticks say which kernel spends less
time on a bucket, not which one shortens the pass.

Every numeric step of the network runs in the library's HIP kernels; this
module marshals arguments, turns measurements into training rows and
applies the decision rule.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import Counter, Options, TCError, _capi, _check, _ptr, _stream, new_profile, schedule_table, workspace
from ._capi import TC_MLP_IN, TC_NUM_BUCKETS, TC_NUM_STRATEGIES

HIDDEN = 32


def bucket_features(b: np.ndarray) -> np.ndarray:
    """(ob, pb, kind) of bucket ids b = (kind * 32 + ob) * 32 + pb."""
    b = np.asarray(b, dtype=np.int64)
    return np.stack([(b >> 5) & 31, b & 31, b >> 10], axis=1).astype(np.float32)


class CostNet:
    """Device parameters and Adam state of the cost network."""

    def __init__(self, hidden: int = HIDDEN, k: int = TC_NUM_STRATEGIES, seed: int = 0, device=None):
        self.hidden, self.k = hidden, k
        self.device = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        lib = _capi.load()
        cnt = ctypes.c_int64()
        _check(lib.tc_mlp_param_count(hidden, k, ctypes.byref(cnt)), "tc_mlp_param_count")
        self.count = cnt.value
        self.params = torch.empty(self.count, dtype=torch.float32, device=self.device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0
        _check(lib.tc_mlp_init(_ptr(self.params), hidden, k, seed, _stream()), "tc_mlp_init")

    def forward(self, X: torch.Tensor) -> torch.Tensor:
        X = X.to(self.device, torch.float32).contiguous()
        rows = X.shape[0]
        Y = torch.empty(rows, self.k, dtype=torch.float32, device=self.device)
        _check(_capi.load().tc_mlp_forward(_ptr(self.params), self.hidden, self.k, _ptr(X), rows, _ptr(Y),
                                           _stream()), "tc_mlp_forward")
        return Y

    def grad(self, X, c, t, w=None):
        """(loss, gradient) on the batch, without an update."""
        lib = _capi.load()
        X, c, t, w = self._batch(X, c, t, w)
        rows = X.shape[0]
        need = ctypes.c_size_t()
        _check(lib.tc_mlp_grad_ws(self.hidden, self.k, rows, ctypes.byref(need)), "tc_mlp_grad_ws")
        ws = workspace(need.value, self.device)
        g = torch.empty_like(self.params)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        _check(lib.tc_mlp_grad(_ptr(self.params), self.hidden, self.k, _ptr(X), _ptr(c), _ptr(t), _ptr(w), rows,
                               _ptr(g), _ptr(loss), _ptr(ws), need.value, _stream()), "tc_mlp_grad")
        return float(loss.item()), g

    def adam(self, grad: torch.Tensor, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step += 1
        _check(_capi.load().tc_mlp_adam(_ptr(self.params), _ptr(grad), _ptr(self.m), _ptr(self.v), self.count,
                                        self.step, lr, beta1, beta2, eps, _stream()), "tc_mlp_adam")

    def train(self, X, c, t, steps: int, lr=1e-2, beta1=0.9, beta2=0.999, eps=1e-8, w=None) -> np.ndarray:
        """``steps`` full-batch Adam steps; returns each step's loss."""
        lib = _capi.load()
        X, c, t, w = self._batch(X, c, t, w)
        rows = X.shape[0]
        need = ctypes.c_size_t()
        _check(lib.tc_mlp_train_ws(self.hidden, self.k, rows, ctypes.byref(need)), "tc_mlp_train_ws")
        ws = workspace(need.value, self.device)
        losses = torch.empty(max(steps, 1), dtype=torch.float32, device=self.device)
        _check(lib.tc_mlp_train(_ptr(self.params), _ptr(self.m), _ptr(self.v), self.hidden, self.k, _ptr(X),
                                _ptr(c), _ptr(t), _ptr(w), rows, self.step + 1, steps, lr, beta1, beta2, eps,
                                _ptr(losses),
                                _ptr(ws), need.value, _stream()), "tc_mlp_train")
        self.step += steps
        return losses[:steps].cpu().numpy()

    def schedule(self, options: Options | None = None, with_cost: bool = False):
        """Strategy table (int32[TC_NUM_BUCKETS], device) for ``options``'
        table sizes; with ``with_cost`` also the predicted costs."""
        opt = (options or Options()).to_c()
        table = torch.empty(TC_NUM_BUCKETS, dtype=torch.int32, device=self.device)
        cost = torch.empty(TC_NUM_BUCKETS, self.k, dtype=torch.float32, device=self.device) if with_cost else None
        _check(_capi.load().tc_mlp_schedule(_ptr(self.params), self.hidden, self.k, ctypes.byref(opt), _ptr(table),
                                            _ptr(cost), _stream()), "tc_mlp_schedule")
        return (table, cost) if with_cost else table

    def _batch(self, X, c, t, w=None):
        X = torch.as_tensor(X, dtype=torch.float32).to(self.device).contiguous()
        c = torch.as_tensor(c, dtype=torch.int32).to(self.device).contiguous()
        t = torch.as_tensor(t, dtype=torch.float32).to(self.device).contiguous()
        if w is not None:
            w = torch.as_tensor(w, dtype=torch.float32).to(self.device).contiguous()
        if X.ndim != 2 or X.shape[1] != TC_MLP_IN or c.shape != (X.shape[0],) or t.shape != (X.shape[0],):
            raise ValueError("batch shapes: X [R, 3], c [R], t [R]")
        if w is not None and (w.shape != (X.shape[0],) or bool((w < 0).any()) or float(w.sum()) <= 0):
            raise ValueError("weights: [R], non-negative, positive sum")
        if X.shape[0] < 1:
            raise ValueError("empty batch")
        return X, c, t, w


def collect_profile(graphs, options: Options | None = None, strategies=range(TC_NUM_STRATEGIES), repeats: int = 1,
                    profile: torch.Tensor | None = None, mode: str = "context", groups: int = 4,
                    seed: int = 0) -> torch.Tensor:
    """Profile every (row_ptr, col[, levels]) graph; returns the accumulated
    profile [TC_NUM_BUCKETS, 4, 3].  ``mode`` "context": per group of
    buckets and strategy, one run with that group switched to the strategy
    and the rest on the heuristic's choice; "forced": one run per strategy
    forced on every bucket."""
    if mode not in ("context", "forced"):
        raise ValueError("mode is 'context' or 'forced'")
    base = options or Options()
    prof = profile if profile is not None else new_profile()
    rng = np.random.default_rng(seed)
    for g in graphs:
        rp, col = g[0], g[1]
        lev = g[2] if len(g) > 2 else None
        n, nnz = rp.numel() - 1, col.numel()
        runs = []
        if mode == "forced":
            runs = [Options(**{**base.__dict__, "force_strategy": int(s), "sched_table": None}) for s in strategies]
        else:
            heur = schedule_table(n, nnz, Options(**{**base.__dict__, "sched_table": None}), rp.device).cpu().numpy()
            grp = rng.permutation(TC_NUM_BUCKETS) % groups
            for r in range(groups):
                for s in strategies:
                    t = heur.copy()
                    t[grp == r] = int(s)
                    runs.append(Options(**{**base.__dict__, "force_strategy": -1,
                                           "sched_table": torch.from_numpy(t).to(rp.device)}))
        for o in runs:
            cnt = Counter(n, nnz, o, rp.device)
            cnt(rp, col, lev)          # warm (not profiled)
            for _ in range(repeats):
                cnt(rp, col, lev, profile=prof)
    return prof


@dataclass
class Dataset:
    X: np.ndarray        # [R, 3] float32 features (ob, pb, kind)
    c: np.ndarray        # [R] int32 strategy
    t: np.ndarray        # [R] float32 log2(wavefront-ticks per element)
    bucket: np.ndarray   # [R] bucket id
    elements: np.ndarray  # [R] elements behind the row
    w: np.ndarray        # [R] float32 training weight


def dataset(profile: torch.Tensor, min_elements: int = 1 << 14, weight_power: float = 1.0) -> Dataset:
    """Training rows from a profile: every (bucket, strategy) that ran at
    least one item over at least ``min_elements`` elements.  A row weighs
    (elements / max elements) ** weight_power: the time a schedule costs is
    the elements-weighted sum of its per-element costs, so errors on large
    buckets matter in proportion."""
    p = profile.cpu().numpy().astype(np.float64)
    ticks, elems, items = p[..., 0], p[..., 1], p[..., 2]
    b, s = np.nonzero((items > 0) & (elems >= min_elements) & (ticks > 0))
    t = np.log2(ticks[b, s] / elems[b, s])
    e = elems[b, s]
    w = (e / e.max()) ** weight_power if len(e) else e
    return Dataset(X=bucket_features(b), c=s.astype(np.int32), t=t.astype(np.float32), bucket=b,
                   elements=e, w=w.astype(np.float32))


def isect_ms(graphs, table: np.ndarray | None, options: Options | None = None, runs: int = 7) -> float:
    """Intersection-pass time (HIP events, median of ``runs`` after one
    warm-up) summed over the graphs, under ``table`` (None: the heuristic)."""
    base = options or Options()
    total = 0.0
    for g in graphs:
        rp, col = g[0], g[1]
        lev = g[2] if len(g) > 2 else None
        t = None if table is None else torch.from_numpy(np.ascontiguousarray(table, dtype=np.int32)).to(rp.device)
        o = Options(**{**base.__dict__, "timing": True, "force_strategy": -1, "sched_table": t})
        cnt = Counter(rp.numel() - 1, col.numel(), o, rp.device)
        cnt(rp, col, lev)
        total += float(np.median([cnt(rp, col, lev).ms["isect"] for _ in range(runs)]))
    return total


def verify_schedule(graphs, table, options: Options | None = None, runs: int = 7, margin: float = 0.01):
    """Measured check of a proposed table on the graphs it was learned from.

    Per-bucket costs measured one bucket group at a time do not add up to
    the pass's wall time (a bucket's items can end up on the critical path),
    so each class of change, (heuristic strategy a -> proposed strategy b),
    is tried on its own: a class is reverted to the heuristic's choice when
    the pass runs faster without it (by more than ``margin``).  If the
    result is not faster than the heuristic by more than ``margin`` as
    well, the heuristic's table is returned (the heuristic is the fallback
    and the judge of the learned table's gain).  Returns (table as an int32 device tensor, {"heuristic_ms",
    "proposed_ms", "ms", "reverted": [(a, b), ...]})."""
    rp0, col0 = graphs[0][0], graphs[0][1]
    heur = schedule_table(rp0.numel() - 1, col0.numel(), Options(**{**(options or Options()).__dict__,
                                                                   "sched_table": None}), rp0.device).cpu().numpy()
    cur = (table.cpu().numpy() if isinstance(table, torch.Tensor) else np.asarray(table)).astype(np.int32)
    t_heur = isect_ms(graphs, None, options, runs)
    t_prop = t_cur = isect_ms(graphs, cur, options, runs)
    reverted = []
    for a, b in sorted({(int(x), int(y)) for x, y in zip(heur, cur) if x != y}):
        trial = cur.copy()
        trial[(heur == a) & (cur == b)] = a
        t = isect_ms(graphs, trial, options, runs)
        if t < t_cur * (1.0 - margin):
            cur, t_cur = trial, t
            reverted.append((a, b))
    if t_cur >= t_heur * (1.0 - margin):
        cur, t_cur = heur.astype(np.int32), t_heur
    info = {"heuristic_ms": t_heur, "proposed_ms": t_prop, "ms": t_cur, "reverted": reverted}
    return torch.from_numpy(np.ascontiguousarray(cur)).to(rp0.device), info


def learn_schedule(graphs, options: Options | None = None, seed: int = 0, steps: int = 3000, lr: float = 1e-2,
                   repeats: int = 1, min_elements: int = 1 << 14, weight_power: float = 1.0, verify: bool = True):
    """Profile, train, schedule and (with ``verify``) check the table by
    measurement on the same graphs (``verify_schedule``).  Returns (table,
    net, dataset, losses); the network's own table is ``net.schedule()``."""
    prof = collect_profile(graphs, options, repeats=repeats)
    ds = dataset(prof, min_elements, weight_power)
    if len(ds.c) == 0:
        raise ValueError("the profile holds no bucket with enough work to learn from")
    net = CostNet(seed=seed)
    losses = net.train(ds.X, ds.c, ds.t, steps, lr=lr, w=ds.w)
    table = net.schedule(options)
    if verify:
        table, _ = verify_schedule(graphs, table, options)
    return table, net, ds, losses


# Actions of the marginal-cost schedule, as strategy-table values: the four
# strategies, and the workgroup hash with half-size slices (table bit 2).
TILE_HALF = 4
ACTIONS = np.array([0, 1, 2, 3, 1 | TILE_HALF], dtype=np.int32)
ACTION_NAMES = ["wave_hash", "wg_hash", "bsearch", "merge", "wg_hash_half_slices"]


def feasible(n: int, nnz: int, options: Options | None = None, device=None) -> np.ndarray:
    """[TC_NUM_BUCKETS, len(ACTIONS)] bool: action a can run bucket b under
    ``options`` (the library maps an infeasible request to another strategy,
    or drops the tile choice where it changes nothing, so an action is
    feasible where asking for it leaves it in place)."""
    base = {**(options or Options()).__dict__, "sched_table": None, "force_strategy": -1}
    dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
    out = np.zeros((TC_NUM_BUCKETS, len(ACTIONS)), dtype=bool)
    for a, v in enumerate(ACTIONS):
        want = torch.full((TC_NUM_BUCKETS,), int(v), dtype=torch.int32, device=dev)
        t = schedule_table(n, nnz, Options(**{**base, "sched_table": want}), dev).cpu().numpy()
        out[:, a] = t == v
    return out


def bucket_elements(row_ptr, col, levels=None, options: Options | None = None) -> np.ndarray:
    """Probe elements per bucket under the heuristic (float64[TC_NUM_BUCKETS])."""
    base = {**(options or Options()).__dict__, "sched_table": None, "force_strategy": -1}
    prof = new_profile(row_ptr.device)
    Counter(row_ptr.numel() - 1, col.numel(), Options(**base), row_ptr.device)(row_ptr, col, levels, profile=prof)
    return prof.cpu().numpy().astype(np.float64)[..., 1].sum(axis=1)


@dataclass
class MarginalSet:
    X: np.ndarray         # [R, 3] float32 features (ob, pb, kind)
    c: np.ndarray         # [R] int32 action (index into ACTIONS)
    t: np.ndarray         # [R] float32 pass-time change per element (ps), 0 for the heuristic's choice
    w: np.ndarray         # [R] float32 weight: the bucket's share of its graph's elements
    bucket: np.ndarray    # [R] bucket id
    graph: np.ndarray     # [R] index of the graph
    delta_ms: np.ndarray  # [R] measured pass-time change (ms)
    spread_ms: np.ndarray  # [R] half the inter-quartile range of the paired differences (ms)
    base_ms: list         # per graph: median pass time under the heuristic (ms)


def collect_marginal(graphs, options: Options | None = None, min_share: float = 0.002, pairs: int = 5,
                     log=None) -> MarginalSet:
    """Whole-pass cost of each strategy change, one bucket at a time.

    Per graph and per bucket holding at least ``min_share`` of the probe
    elements, every other feasible action (a strategy, or the workgroup hash
    with half-size slices) replaces the heuristic's choice for that bucket
    alone, and the bucketing plus intersection time (HIP
    events) is measured in ``pairs`` (heuristic, changed) pairs run back to
    back; the change's cost is the median paired difference.  A bucket's
    items share the pass with every other bucket, so only the pass time says
    what a change is worth: a strategy that spends fewer wave-ticks on a
    bucket can still lengthen the pass (its items finish last, or it takes
    memory bandwidth from the rest).  Training rows: the change per element
    in picoseconds, and 0 for the heuristic's own choice."""
    base = {**(options or Options()).__dict__, "timing": True, "force_strategy": -1}
    rows = {k: [] for k in ("b", "c", "t", "w", "g", "d", "sp")}
    base_ms = []
    for gi, g in enumerate(graphs):
        rp, col = g[0], g[1]
        lev = g[2] if len(g) > 2 else None
        n, nnz = rp.numel() - 1, col.numel()
        heur = schedule_table(n, nnz, Options(**{**base, "sched_table": None}), rp.device)
        heur_np = heur.cpu().numpy()
        feas = feasible(n, nnz, Options(**{**base, "timing": False}), rp.device)
        elems = bucket_elements(rp, col, lev, options)
        share = elems / max(elems.sum(), 1.0)
        table = heur.clone()
        cnt = Counter(n, nnz, Options(**{**base, "sched_table": table}), rp.device)

        def run(t_np):
            table.copy_(torch.from_numpy(t_np))
            r = cnt(rp, col, lev)
            return r.ms["bucket"] + r.ms["isect"]

        for _ in range(2):
            run(heur_np)
        hs = []
        for b in np.nonzero(share >= min_share)[0]:
            for s in np.nonzero(feas[b])[0]:
                if ACTIONS[s] == heur_np[b]:
                    continue
                alt = heur_np.copy()
                alt[b] = ACTIONS[s]
                run(alt)                       # warm the changed shape
                d = []
                for _ in range(pairs):
                    h = run(heur_np)
                    a = run(alt)
                    hs.append(h)
                    d.append(a - h)
                q1, med, q3 = np.percentile(d, [25, 50, 75])
                for k, v in (("b", b), ("c", s), ("t", med * 1e9 / elems[b]), ("w", share[b]), ("g", gi),
                             ("d", med), ("sp", 0.5 * (q3 - q1))):
                    rows[k].append(v)
            for k, v in (("b", b), ("c", heur_np[b]), ("t", 0.0), ("w", share[b]), ("g", gi), ("d", 0.0),
                         ("sp", 0.0)):
                rows[k].append(v)
            if log:
                log(f"graph {gi} bucket {b} share {share[b]:.3f} heur {heur_np[b]}: "
                    + " ".join(f"{c}:{d:+.3f}" for c, d, bb in zip(rows['c'], rows['d'], rows['b'])
                               if bb == b and c != heur_np[b]))
        base_ms.append(float(np.median(hs)) if hs else float("nan"))
    b = np.asarray(rows["b"], dtype=np.int64)
    return MarginalSet(X=bucket_features(b), c=np.asarray(rows["c"], np.int32), t=np.asarray(rows["t"], np.float32),
                       w=np.asarray(rows["w"], np.float32), bucket=b, graph=np.asarray(rows["g"], np.int32),
                       delta_ms=np.asarray(rows["d"]), spread_ms=np.asarray(rows["sp"]), base_ms=base_ms)


def sgnlog(t) -> np.ndarray:
    """The marginal training target: sign(t) * log2(1 + |t|) of the pass-time
    change t in picoseconds per element (changes span four decades; the
    small ones near zero decide the schedule)."""
    t = np.asarray(t, dtype=np.float64)
    return (np.sign(t) * np.log2(1.0 + np.abs(t))).astype(np.float32)


def feature_hull(X: np.ndarray) -> dict:
    """Per kind, the owner- and partner-class ranges seen in training:
    {kind: [ob_min, ob_max, pb_min, pb_max]}."""
    X = np.asarray(X)
    out = {}
    for k in np.unique(X[:, 2]).astype(int):
        m = X[:, 2] == k
        out[int(k)] = [int(X[m, 0].min()), int(X[m, 0].max()), int(X[m, 1].min()), int(X[m, 1].max())]
    return out


def inside_hull(hull: dict) -> np.ndarray:
    """bool[TC_NUM_BUCKETS]: the bucket's features lie in the training ranges."""
    X = bucket_features(np.arange(TC_NUM_BUCKETS))
    ins = np.zeros(TC_NUM_BUCKETS, dtype=bool)
    for k, (o0, o1, p0, p1) in hull.items():
        ins |= (X[:, 2] == int(k)) & (X[:, 0] >= o0) & (X[:, 0] <= o1) & (X[:, 1] >= p0) & (X[:, 1] <= p1)
    return ins


def select_table(cost: np.ndarray, feas: np.ndarray, heur: np.ndarray, inside: np.ndarray,
                 margin: float) -> np.ndarray:
    """Per bucket: the cheapest feasible strategy by the predicted cost when
    the bucket lies inside the training ranges and the prediction beats the
    heuristic's choice by more than ``margin``; else the heuristic's choice.
    Ties go to the lower strategy number."""
    c = np.where(feas, np.asarray(cost, dtype=np.float64), np.inf)
    best = np.argmin(c, axis=1)
    b = np.arange(c.shape[0])
    gain = c[b, heur] - c[b, best]
    return np.where(inside & (gain > margin), best, heur).astype(np.int32)


def changed_classes(heur, table) -> list:
    """The classes of change (heuristic strategy a -> table strategy b) of a table."""
    h, t = np.asarray(heur), np.asarray(table)
    return sorted({(int(a), int(b)) for a, b in zip(h, t) if a != b})


def learned_table(net: "CostNet", n: int, nnz: int, hull: dict, margin: float, options: Options | None = None,
                  device=None, veto=()) -> torch.Tensor:
    """The table a trained marginal-cost network gives a graph of n vertices
    and nnz entries under ``options`` (int32 device tensor).  Changes of a
    class in ``veto`` ((heuristic strategy, proposed strategy) pairs, those
    that measured slower on the training graphs) keep the heuristic's choice."""
    base = {**(options or Options()).__dict__, "sched_table": None, "force_strategy": -1}
    dev = device if device is not None else net.device
    heur = schedule_table(n, nnz, Options(**base), dev).cpu().numpy()   # heuristic values are actions 0..3
    feas = feasible(n, nnz, Options(**base), dev)[:, :net.k]
    cost = net.forward(torch.from_numpy(bucket_features(np.arange(TC_NUM_BUCKETS)))).cpu().numpy()
    t = ACTIONS[select_table(cost, feas, heur, inside_hull(hull), margin)]
    for a, b in veto:
        t[(heur == a) & (t == b)] = a
    return torch.from_numpy(np.ascontiguousarray(t, dtype=np.int32)).to(dev)


def learn_marginal(graphs, options: Options | None = None, seed: int = 0, steps: int = 3000, lr: float = 1e-2,
                   min_share: float = 0.002, pairs: int = 5, log=None):
    """Measure (``collect_marginal``), then train the network on sgnlog of
    the per-element pass-time changes, each row weighed by its bucket's
    share of the elements.  Returns (net, marginal set, losses, hull)."""
    ms = collect_marginal(graphs, options, min_share, pairs, log)
    if len(ms.c) == 0:
        raise ValueError("no bucket holds min_share of the elements")
    net = CostNet(k=len(ACTIONS), seed=seed)
    losses = net.train(ms.X, ms.c, sgnlog(ms.t), steps, lr=lr, w=ms.w)
    return net, ms, losses, feature_hull(ms.X)


def save_net(path: str, net: "CostNet", hull: dict, margin: float, meta: dict, veto=()):
    """The trained network as JSON: parameters (float32 values, in the
    library's order), training ranges, decision margin, vetoed classes of
    change, and ``meta``."""
    import json
    doc = {"hidden": net.hidden, "k": net.k, "params": [float(x) for x in net.params.cpu().numpy()],
           "hull": {str(k): v for k, v in hull.items()}, "margin": margin,
           "veto": [list(map(int, c)) for c in veto], **meta}
    with open(path, "w") as f:
        json.dump(doc, f, indent=1)


def load_net(path: str, device=None):
    """(net, hull, margin, document) from a file written by ``save_net``;
    the vetoed classes are ``document["veto"]``."""
    import json
    with open(path) as f:
        doc = json.load(f)
    net = CostNet(hidden=doc["hidden"], k=doc["k"], device=device)
    p = torch.tensor(doc["params"], dtype=torch.float32)
    if p.numel() != net.count:
        raise ValueError(f"{path}: {p.numel()} parameters, the network has {net.count}")
    net.params.copy_(p.to(net.device))
    return net, {int(k): v for k, v in doc["hull"].items()}, float(doc["margin"]), doc


__all__ = ["CostNet", "Dataset", "bucket_features", "collect_profile", "dataset", "isect_ms", "learn_schedule",
           "verify_schedule", "TCError", "MarginalSet", "collect_marginal", "feasible", "bucket_elements", "sgnlog", "feature_hull", "inside_hull",
           "select_table", "learned_table", "learn_marginal", "save_net", "load_net", "changed_classes", "ACTIONS",
           "ACTION_NAMES", "TILE_HALF"]
