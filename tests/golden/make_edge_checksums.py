"""Writes tests/golden/edge_checksums.txt: checksums of the oracle's
per-edge triangle counts (support, one per CSR entry) of the scale-20
Kronecker graph, computed on the CPU with the oracle only (a sorted merge of
the two rows of every entry).  The 126 MB vector is not stored; the GPU test
compares the same functions of its own vector (see make_vertex_checksums.py:
s1 = sum (e + 1) * sup[e], s2 = sum sup[e]^2, both mod 2^64, the maximum and
its first entry).

Run once from the repository root (several minutes):

    python tests/golden/make_edge_checksums.py
"""
from __future__ import annotations

import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, HERE)

import graphgen  # noqa: E402
import oracle  # noqa: E402
from make_vertex_checksums import checksums  # noqa: E402

GRAPHS = {
    "kronecker20": lambda: graphgen.kronecker(20, 16, seed=1),
}


def main():
    out = os.path.join(HERE, "edge_checksums.txt")
    lines = ["# checksums of the oracle's per-edge triangle counts (sorted merge per CSR entry, gcc -O2)",
             "# written by tests/golden/make_edge_checksums.py; columns: name nnz sum_sup s1 s2 max argmax"]
    for name, gen in GRAPHS.items():
        t0 = time.time()
        n, s, d = gen()
        g = oracle.build_csr(n, s, d)
        del s, d
        sup = oracle.edge_support(g)
        s1, s2, mx, am = checksums(sup)
        lines.append(f"{name} {g.nnz} {int(sup.sum(dtype='uint64'))} {s1} {s2} {mx} {am}")
        print(lines[-1], f"({time.time() - t0:.0f} s)", flush=True)
        with open(out, "w") as f:
            f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
