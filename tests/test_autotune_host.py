"""Host logic of the autotuner: the coordinate descent, the cache and the
signature, with a synthetic cost in place of GPU timings."""
from __future__ import annotations

import json

import pytest

torch = pytest.importorskip("torch")

from paper_2309_09064_amd import autotune  # noqa: E402


def test_descent_finds_separable_minimum():
    space = {"a": [1, 2, 3, 4], "b": [10, 20, 30], "c": [0, 5]}
    target = {"a": 3, "b": 10, "c": 5}
    cost = lambda p: sum((p[k] - target[k]) ** 2 for k in p)
    best, c, evals = autotune.coordinate_descent(cost, {"a": 1, "b": 30, "c": 0}, space)
    assert best == target and c == 0
    assert len(evals) <= 1 + 2 * sum(len(v) - 1 for v in space.values())


def test_descent_stops_at_coordinate_minimum():
    # a coupled cost: the result is a point no single-coordinate move improves
    space = {"x": list(range(5)), "y": list(range(5))}
    cost = lambda p: (p["x"] - p["y"]) ** 2 + 0.1 * (p["x"] - 3) ** 2
    best, c, _ = autotune.coordinate_descent(cost, {"x": 0, "y": 4}, space)
    for k in space:
        for v in space[k]:
            assert cost({**best, k: v}) >= c


def test_tune_with_injected_timer():
    rp = torch.tensor([0, 2, 4, 6], dtype=torch.int32)
    col = torch.tensor([1, 2, 0, 2, 0, 1], dtype=torch.int32)
    ms = lambda p: abs(p["chunk_work"] - 8192) / 1e4 + (0 if p["wave_slots"] == 1024 else 1) + p["grid_blocks"] / 1e3
    opts, rep = autotune.tune(rp, col, timer=ms)
    assert (opts.chunk_work, opts.wave_slots, opts.grid_blocks) == (8192, 1024, 0)
    assert rep["best_ms"] < rep["default_ms"] and opts.timing is False


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "cache.json")
    c = autotune.Cache(path)
    assert c.get("dev", "sig") is None
    best = {"chunk_work": 4096, "wave_slots": 512, "wg_slots": 8192, "grid_blocks": 128}
    c.put("dev", "sig", best, 1.5, 2.0)
    again = autotune.Cache(path)
    assert again.get("dev", "sig")["options"] == best
    with open(path, "w") as f:
        json.dump({"dev": {"sig": {"options": {"chunk_work": 1}}}}, f)   # incomplete entry
    assert autotune.Cache(path).get("dev", "sig") is None
    with open(path, "w") as f:
        f.write("{not json")
    assert autotune.Cache(path).data == {}


def test_signature_rounds_log2():
    assert autotune.signature(1 << 20, 31_402_138, 65_000) == "n20-nnz25-dmax16"
    assert autotune.signature(0, 0, 0) == "n0-nnz0-dmax0"
