"""Writes tests/golden/batch_counts.txt: the oracle's triangle count of every
graph of the 4096-graph batch (half Erdos-Renyi G(n, p) with n log-uniform in
[64, 65536] and mean degree uniform in [8, 64], half Kronecker with scale
uniform in {8..16}, edgefactor 16; member i seeded 1000 + i, size draws seeded
0), each graph cleaned and counted on its own on the CPU by the oracle only
(serial BFS levels + Algorithm 4's T0 and T1).  Run once from the repository
root:

    python tests/golden/make_batch_counts.py

It takes a few minutes on 8 cores.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import graphgen  # noqa: E402
import oracle  # noqa: E402


def member(mem):
    n, s, d = graphgen.batch_member_tuples(mem)
    g = oracle.build_csr(n, s, d)
    r = oracle.alg4(g)
    return g.n, g.m, r.T


def main():
    t0 = time.time()
    rec = graphgen.batch_recipe(4096, seed=0)
    with cf.ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
        rows = list(ex.map(member, rec))
    lines = ["# oracle triangle counts of the 4096-graph batch (graphgen.batch_recipe(4096, seed=0)),",
             "# each graph cleaned and counted alone (serial BFS levels + Algorithm 4's T0 and T1);",
             "# written by tests/golden/make_batch_counts.py; columns: index kind n m T"]
    for i, (mem, (n, m, T)) in enumerate(zip(rec, rows)):
        lines.append(f"{i} {mem.kind} {n} {m} {T}")
    with open(os.path.join(HERE, "batch_counts.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"{len(rows)} graphs, {sum(r[1] for r in rows)} edges, {sum(r[2] for r in rows)} triangles, "
          f"{time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
