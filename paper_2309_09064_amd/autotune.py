"""Autotuner for the intersection pass's tile and launch parameters.

The tunable options never change a count; they set the work-item size
(``chunk_work``), the LDS hash-table sizes (``wave_slots``, ``wg_slots``,
which also move the wavefront / workgroup / search thresholds), and the
persistent grid (``grid_blocks``).  The search is a coordinate descent from
the defaults: each pass tries every value of one parameter with the others
fixed and keeps the fastest, until a pass changes nothing.  A candidate's
cost is the median over ``repeats`` runs of the bucketing + intersection
time, from the HIP events the library records on its stream (levels are
computed once and passed in, since they do not depend on these options).

Results are cached in a JSON file keyed by the device name and a graph
signature (rounded log2 of n, nnz and the largest degree), so graphs of the
same shape reuse a tuning.
"""
from __future__ import annotations

import json
import math
import os
from dataclasses import fields

import numpy as np

from . import Counter, Options

SPACE = {
    "chunk_work": [4096, 8192, 16384, 32768, 65536],
    "wave_slots": [512, 1024, 2048],
    "wg_slots": [8192, 16384, 32768],
    "grid_blocks": [0, 128, 512],
}
TUNED_FIELDS = tuple(SPACE)


def default_cache_path() -> str:
    return os.environ.get("TC_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "paper_2309_09064_amd", "autotune.json"))


def signature(n: int, nnz: int, max_degree: int) -> str:
    r = lambda v: int(round(math.log2(max(int(v), 1))))
    return f"n{r(n)}-nnz{r(nnz)}-dmax{r(max_degree)}"


def graph_signature(row_ptr, col) -> str:
    import torch
    n = row_ptr.numel() - 1
    dmax = int(torch.diff(row_ptr).max().item()) if n > 0 else 0
    return signature(n, col.numel(), dmax)


def device_key() -> str:
    import torch
    return torch.cuda.get_device_properties(torch.cuda.current_device()).name


def coordinate_descent(cost, start: dict, space: dict = SPACE, max_passes: int = 3):
    """Minimise ``cost(point) -> float`` over the grid ``space`` from
    ``start``; returns (best point, best cost, every evaluation)."""
    seen = {}

    def ev(p):
        key = tuple(sorted(p.items()))
        if key not in seen:
            seen[key] = float(cost(dict(p)))
        return seen[key]

    best = dict(start)
    best_c = ev(best)
    for _ in range(max_passes):
        changed = False
        for name, values in space.items():
            for v in values:
                if v == best[name]:
                    continue
                cand = {**best, name: v}
                c = ev(cand)
                if c < best_c:
                    best, best_c, changed = cand, c, True
        if not changed:
            break
    return best, best_c, [(dict(k), c) for k, c in seen.items()]


def _valid(p: dict) -> bool:
    # sixteen wavefront tables share one workgroup's LDS
    return p["wave_slots"] * 16 <= 32768


class Cache:
    def __init__(self, path: str | None = None):
        self.path = path or default_cache_path()
        self.data = {}
        if os.path.exists(self.path):
            try:
                with open(self.path) as f:
                    self.data = json.load(f)
            except (OSError, ValueError):
                self.data = {}

    def get(self, device: str, sig: str):
        e = self.data.get(device, {}).get(sig)
        if not isinstance(e, dict) or not all(k in e.get("options", {}) for k in TUNED_FIELDS):
            return None
        return e

    def put(self, device: str, sig: str, options: dict, ms: float, default_ms: float):
        self.data.setdefault(device, {})[sig] = {"options": {k: int(options[k]) for k in TUNED_FIELDS},
                                                 "ms": ms, "default_ms": default_ms}
        os.makedirs(os.path.dirname(os.path.abspath(self.path)), exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.data, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


def _options(p: dict, base: Options | None) -> Options:
    b = {f.name: getattr(base, f.name) for f in fields(base)} if base is not None else {}
    b.update({k: int(p[k]) for k in TUNED_FIELDS})
    b["timing"] = True
    return Options(**b)


def tune(row_ptr, col, levels=None, space: dict = SPACE, repeats: int = 3, base: Options | None = None,
         cache: Cache | None = None, timer=None):
    """Tune for this graph.  Returns (Options, report dict).  ``timer``
    (for tests) replaces the measured cost: ``timer(point) -> ms``."""
    from . import bfs_levels
    n, nnz = row_ptr.numel() - 1, col.numel()
    if timer is None:
        lev = levels if levels is not None else bfs_levels(row_ptr, col)[0]

        def timer(p):
            if not _valid(p):
                return math.inf
            c = Counter(n, nnz, _options(p, base), row_ptr.device)
            ms = []
            for _ in range(repeats + 1):
                r = c(row_ptr, col, lev)
                ms.append(r.ms["bucket"] + r.ms["isect"])
            return float(np.median(ms[1:]))

    start = {"chunk_work": 16384, "wave_slots": 2048, "wg_slots": 32768, "grid_blocks": 0}
    best, best_ms, evals = coordinate_descent(timer, start, space)
    default_ms = next(c for p, c in evals if p == start)   # the search's own timing of the defaults
    report = {"signature": graph_signature(row_ptr, col), "default_ms": default_ms, "best_ms": best_ms,
              "best": best, "evaluations": len(evals)}
    if cache is not None:
        cache.put(device_key(), report["signature"], best, best_ms, default_ms)
    opts = _options(best, base)
    opts.timing = base.timing if base is not None else False
    return opts, report


def tuned_options(row_ptr, col, levels=None, cache: Cache | None = None, base: Options | None = None,
                  tune_if_missing: bool = True, **kw) -> Options:
    """Options from the cache for this graph's signature, tuning (and
    caching) on a miss when ``tune_if_missing``; else the defaults."""
    cache = cache or Cache()
    e = cache.get(device_key(), graph_signature(row_ptr, col))
    if e is not None:
        opts = _options(e["options"], base)
        opts.timing = base.timing if base is not None else False
        return opts
    if not tune_if_missing:
        return base or Options()
    return tune(row_ptr, col, levels, base=base, cache=cache, **kw)[0]


__all__ = ["SPACE", "Cache", "coordinate_descent", "signature", "graph_signature", "tune", "tuned_options"]
