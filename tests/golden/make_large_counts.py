"""Writes tests/golden/large_counts.txt: the oracle's T, T0, T1 and |E0| of
the large seeded graphs, computed on the CPU with the oracle only (serial
BFS levels + Algorithm 4).  Run once from the repository root:

    python tests/golden/make_large_counts.py

It takes tens of minutes and about 20 GB of host memory at scale 24.
"""
from __future__ import annotations

import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import graphgen  # noqa: E402
import oracle  # noqa: E402

GRAPHS = {
    "kronecker20": lambda: graphgen.kronecker(20, 16, seed=1),
    "chunglu22": lambda: graphgen.chung_lu(1 << 22, 2.1, 32.0, float(1 << 17), seed=1),
    "kronecker24": lambda: graphgen.kronecker(24, 16, seed=1),
}


def main():
    out = os.path.join(HERE, "large_counts.txt")
    lines = ["# oracle counts (serial BFS levels + Algorithm 4, gcc -O2) of the large seeded graphs",
             "# written by tests/golden/make_large_counts.py; columns: name n m T T0 T1 e0"]
    for name, gen in GRAPHS.items():
        t0 = time.time()
        n, s, d = gen()
        g = oracle.build_csr(n, s, d)
        del s, d
        lev, _ = oracle.bfs_levels(g)
        r = oracle.alg4(g, lev)
        lines.append(f"{name} {g.n} {g.m} {r.T} {r.T0} {r.T1} {r.E0}")
        print(lines[-1], f"({time.time() - t0:.0f} s)", flush=True)
        with open(out, "w") as f:
            f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
