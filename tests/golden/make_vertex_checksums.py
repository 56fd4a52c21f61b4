"""Writes tests/golden/vertex_checksums.txt: checksums of the oracle's
per-vertex triangle counts t(v) of the scale-20 Kronecker graph, computed on
the CPU with the oracle only (the whole-graph sorted-merge definition).  The
8 MB vector itself is not stored; the GPU test compares the same three
functions of its own vector:

    s1 = sum_v (v + 1) * t(v)  mod 2^64
    s2 = sum_v t(v)^2          mod 2^64
    mx = max_v t(v), and the smallest v where it is reached

Run once from the repository root (a few minutes):

    python tests/golden/make_vertex_checksums.py
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import graphgen  # noqa: E402
import oracle  # noqa: E402

GRAPHS = {
    "kronecker20": lambda: graphgen.kronecker(20, 16, seed=1),
}


def checksums(tv: np.ndarray):
    t = tv.astype(np.uint64)
    idx = np.arange(1, len(t) + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        s1 = int(np.sum(idx * t, dtype=np.uint64))
        s2 = int(np.sum(t * t, dtype=np.uint64))
    return s1, s2, int(t.max()), int(np.argmax(t))


def main():
    out = os.path.join(HERE, "vertex_checksums.txt")
    lines = ["# checksums of the oracle's per-vertex triangle counts (whole-graph sorted merge, gcc -O2)",
             "# written by tests/golden/make_vertex_checksums.py; columns: name n sum_t s1 s2 max argmax"]
    for name, gen in GRAPHS.items():
        t0 = time.time()
        n, s, d = gen()
        g = oracle.build_csr(n, s, d)
        del s, d
        tv = oracle.vertex_triangles(g)
        s1, s2, mx, am = checksums(tv)
        lines.append(f"{name} {g.n} {int(tv.sum())} {s1} {s2} {mx} {am}")
        print(lines[-1], f"({time.time() - t0:.0f} s)", flush=True)
        with open(out, "w") as f:
            f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
