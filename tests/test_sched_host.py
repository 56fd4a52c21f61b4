"""Host logic of the learned schedule: the target transform, the training
ranges, and the trusted-table rule (no GPU)."""
from __future__ import annotations

import numpy as np
import pytest

pytest.importorskip("torch")
from paper_2309_09064_amd import sched  # noqa: E402


def test_sgnlog_is_odd_monotone_and_fixes_zero():
    t = np.array([-1000.0, -3.0, -1.0, 0.0, 1.0, 3.0, 1000.0])
    y = sched.sgnlog(t)
    assert y.dtype == np.float32
    assert np.allclose(y, -y[::-1]) and np.all(np.diff(y) > 0)
    assert y[3] == 0 and y[4] == 1.0 and y[5] == 2.0   # log2(1 + 1), log2(1 + 3)


def bucket(kind, ob, pb):
    return (kind * 32 + ob) * 32 + pb


def test_hull_and_inside():
    b = np.array([bucket(0, 5, 3), bucket(0, 9, 7), bucket(1, 12, 10)])
    hull = sched.feature_hull(sched.bucket_features(b))
    assert hull == {0: [5, 9, 3, 7], 1: [12, 12, 10, 10]}
    ins = sched.inside_hull(hull)
    assert ins.sum() == 5 * 5 + 1
    assert ins[bucket(0, 7, 5)] and ins[bucket(1, 12, 10)]
    assert not ins[bucket(0, 10, 5)] and not ins[bucket(1, 12, 9)] and not ins[bucket(1, 5, 3)]


def test_select_table_rule():
    B = 2048
    heur = np.full(B, 1, dtype=np.int64)
    feas = np.ones((B, 4), dtype=bool)
    feas[:, 0] = False            # wavefront hash infeasible everywhere
    cost = np.zeros((B, 4))
    cost[:, 0] = -50.0            # cheapest but infeasible: never chosen
    cost[:, 1] = 2.0              # the heuristic's choice
    cost[:, 2] = 0.5              # gain 1.5
    cost[:, 3] = 1.5              # gain 0.5
    inside = np.zeros(B, dtype=bool)
    inside[:100] = True
    t = sched.select_table(cost, feas, heur, inside, margin=1.0)
    assert np.all(t[:100] == 2) and np.all(t[100:] == 1)
    t = sched.select_table(cost, feas, heur, inside, margin=2.0)   # gain below the margin
    assert np.all(t == 1)
    cost[:, 3] = 0.5              # tie between 2 and 3: the lower number
    t = sched.select_table(cost, feas, heur, np.ones(B, dtype=bool), margin=0.0)
    assert np.all(t == 2)


def test_changed_classes():
    heur = np.array([0, 0, 1, 1, 3, 3])
    table = np.array([0, 1, 1, 2, 0, 0])
    assert sched.changed_classes(heur, table) == [(0, 1), (1, 2), (3, 0)]
    assert sched.changed_classes(heur, heur) == []


def test_actions_are_table_values():
    # the four strategies as themselves, then the workgroup hash (1) with the
    # half-slice bit
    assert sched.ACTIONS.tolist() == [0, 1, 2, 3, 1 | sched.TILE_HALF]
    assert sched.TILE_HALF == 4 and len(sched.ACTION_NAMES) == len(sched.ACTIONS)
