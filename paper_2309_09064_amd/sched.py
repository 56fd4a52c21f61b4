"""Learned schedule: profile, cost network, per-bucket strategy table.

Not part of the paper's method.  Every strategy counts exactly, so the
schedule only decides speed.  The cycle:

1. ``collect_profile``: count graphs with the instrumented kernels
   (``tc_count_profile``), which accumulate per (bucket, strategy) the
   wavefront-ticks spent and the elements handled.  In the default
   "context" mode the buckets are split into four random groups and each
   group in turn runs each strategy while the other buckets keep the
   heuristic's choice, so every (bucket, strategy) cost is measured once
   inside a realistic mix (costs measured with one strategy forced
   everywhere do not carry over: e.g. binary search then competes only with
   itself for memory).
2. ``dataset``: one training row per (bucket, strategy) with enough work:
   features (ob, pb, kind) of the bucket, the strategy, and the target
   log2(wavefront-ticks per element).
3. ``CostNet.train``: full-batch Adam on the device (``tc_mlp_train``).
4. ``CostNet.schedule``: per bucket the cheapest feasible strategy by the
   network's prediction (``tc_mlp_schedule``), a table that
   ``Options(sched_table=...)`` hands to ``tc_count``.
5. ``verify_schedule``: the table's changes against the heuristic, one class
   (heuristic strategy -> proposed strategy) at a time, are kept only where
   the measured pass is faster with them.

Every numeric step of the network runs in the library's HIP kernels; this
module marshals arguments and turns profile counters into training rows.
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
    result is still not faster than the heuristic, the heuristic's table is
    returned.  Returns (table as an int32 device tensor, {"heuristic_ms",
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
    if t_cur >= t_heur:
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


__all__ = ["CostNet", "Dataset", "bucket_features", "collect_profile", "dataset", "isect_ms", "learn_schedule",
           "verify_schedule", "TCError"]
