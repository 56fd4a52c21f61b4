"""CPU oracle for the triangle count -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never does, and the
oracle imports nothing from it: the two share no code.  Both take their
inputs from ``graphgen``.

``tc_oracle.c`` (plain serial C, built with gcc) follows Bader, "Fast Triangle
Counting" (arXiv 2309.09064):

* :func:`build_csr`          simple undirected CSR from tuples (Introduction)
* :func:`bfs_levels`         BFS from each unvisited vertex in id order (Alg. 4)
* :func:`partition`          E0/E1 split, N0 rows split by rank or by id (Alg. 4)
* :func:`alg4`               T0 = triangles inside G0, T1 = triangles with one
                             horizontal edge (the two sums of Alg. 4), by merges
* :func:`count_emd`          direction-oriented sorted-merge edge iterator
* :func:`count_emd_entries`  the same over a sample of edges, on host threads
* :func:`alg3`               cover-edge count (Alg. 3)
* :func:`vertex_triangles`   per-vertex triangle counts
* :func:`vertex_triangles_at`  the same for sampled vertices, by another definition
* :func:`edge_support`       per-edge triangle counts (k-truss support)
* :func:`edge_support_at`    the same for sampled entries
* :func:`relabel_degree`     degree ordering of the vertices (BaderD / CED)

:mod:`oracle.mlp` holds the float64 reference of the scheduler network.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tc_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_i32 = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_i64 = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_u64 = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
_u32 = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")


def build(force: bool = True, opt: str = "-O2") -> str:
    """Compile the oracle with gcc (``-O2``, as the paper compiled its C)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", opt, "-fopenmp", "-fPIC", "-shared", "-std=c11", "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        lib.orc_build_csr.argtypes = [ctypes.c_int64, ctypes.c_int64, _i32, _i32, _i64, _i32, ctypes.c_int64]
        lib.orc_build_csr.restype = ctypes.c_int64
        lib.orc_bfs_levels.argtypes = [ctypes.c_int64, _i64, _i32, _i32]
        lib.orc_bfs_levels.restype = ctypes.c_int64
        lib.orc_partition.argtypes = [ctypes.c_int64, _i64, _i32, _i32, ctypes.c_int32, _i64, _i32, _i32, _i64, _i32]
        lib.orc_partition.restype = None
        lib.orc_alg4.argtypes = [ctypes.c_int64, _i64, _i32, _i32, ctypes.POINTER(ctypes.c_uint64),
                                 ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_int64)]
        lib.orc_alg4.restype = ctypes.c_int
        lib.orc_count_emd.argtypes = [ctypes.c_int64, _i64, _i32]
        lib.orc_count_emd.restype = ctypes.c_uint64
        lib.orc_count_emd_entries.argtypes = [ctypes.c_int64, _i64, _i32, ctypes.c_int64, _i64, ctypes.c_int]
        lib.orc_count_emd_entries.restype = ctypes.c_uint64
        lib.orc_alg3.argtypes = [ctypes.c_int64, _i64, _i32, _i32]
        lib.orc_alg3.restype = ctypes.c_uint64
        lib.orc_vertex_triangles.argtypes = [ctypes.c_int64, _i64, _i32, _u64]
        lib.orc_vertex_triangles.restype = None
        lib.orc_vertex_triangles_at.argtypes = [ctypes.c_int64, _i64, _i32, ctypes.c_int64, _i64, _u64]
        lib.orc_vertex_triangles_at.restype = None
        lib.orc_edge_support.argtypes = [ctypes.c_int64, _i64, _i32, _u32]
        lib.orc_edge_support.restype = None
        lib.orc_edge_support_at.argtypes = [ctypes.c_int64, _i64, _i32, ctypes.c_int64, _i64, _u32]
        lib.orc_edge_support_at.restype = None
        lib.orc_relabel_degree.argtypes = [ctypes.c_int64, _i64, _i32, _i64, _i32, _i32]
        lib.orc_relabel_degree.restype = ctypes.c_int
        _lib = lib
    return _lib


@dataclass
class CSR:
    """Host CSR: ``row_ptr`` int64[n+1], ``col`` int32[nnz], rows sorted."""
    n: int
    row_ptr: np.ndarray
    col: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def m(self) -> int:
        """Undirected edge count."""
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)


def as_csr(n, row_ptr, col) -> CSR:
    return CSR(int(n), np.ascontiguousarray(row_ptr, dtype=np.int64),
               np.ascontiguousarray(col, dtype=np.int32))


def build_csr(n: int, src: np.ndarray, dst: np.ndarray) -> CSR:
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    m = len(src)
    rp = np.zeros(n + 1, dtype=np.int64)
    col = np.empty(max(2 * m, 1), dtype=np.int32)
    nnz = _load().orc_build_csr(n, m, src, dst, rp, col, len(col))
    if nnz == -1:
        raise ValueError("vertex id out of range")
    if nnz < 0:
        raise RuntimeError(f"orc_build_csr failed ({nnz})")
    return CSR(n, rp, col[:nnz].copy())


def bfs_levels(g: CSR):
    """Levels (int32[n]) and the number of components."""
    lev = np.empty(max(g.n, 1), dtype=np.int32)
    roots = _load().orc_bfs_levels(g.n, g.row_ptr, g.col if g.nnz else np.zeros(1, np.int32), lev)
    if roots < 0:
        raise RuntimeError("orc_bfs_levels failed")
    return lev[:g.n], int(roots)


@dataclass
class Partition:
    rp0: np.ndarray   # int64[n+1]
    c0: np.ndarray    # int32[2|E0|]: per row, rank-upper part then rank-lower part
    up0: np.ndarray   # int32[n]: size of the rank-upper part of each row
    rp1: np.ndarray   # int64[n+1]
    c1: np.ndarray    # int32[2|E1|]


def _col_or_dummy(g: CSR):
    return g.col if g.nnz else np.zeros(1, np.int32)


def partition(g: CSR, level: np.ndarray, by_id: bool = False) -> Partition:
    """E0/E1 split of Alg. 4; each N0 row holds its upper part first: the
    neighbours of higher (degree, id) rank, or of higher id with ``by_id``."""
    lev = np.ascontiguousarray(level, dtype=np.int32)
    rp0 = np.zeros(g.n + 1, np.int64)
    rp1 = np.zeros(g.n + 1, np.int64)
    c0 = np.empty(max(g.nnz, 1), np.int32)
    c1 = np.empty(max(g.nnz, 1), np.int32)
    up0 = np.zeros(max(g.n, 1), np.int32)
    _load().orc_partition(g.n, g.row_ptr, _col_or_dummy(g), lev if g.n else np.zeros(1, np.int32),
                          1 if by_id else 0, rp0, c0, up0, rp1, c1)
    return Partition(rp0, c0[:rp0[-1]].copy(), up0[:g.n].copy(), rp1, c1[:rp1[-1]].copy())


@dataclass
class Alg4Result:
    T: int
    T0: int
    T1: int
    E0: int           # undirected horizontal edges
    k: float          # percentage of edges that are horizontal


def alg4(g: CSR, level: np.ndarray | None = None) -> Alg4Result:
    """The counts of Algorithm 4 for levels ``level`` (serial BFS levels when
    None): T0 = triangles whose three edges are horizontal, T1 = triangles
    with exactly one horizontal edge, T = T0 + T1, |E0| and k."""
    if level is None:
        level, _ = bfs_levels(g)
    lev = np.ascontiguousarray(level, dtype=np.int32)
    t0 = ctypes.c_uint64()
    t1 = ctypes.c_uint64()
    e0 = ctypes.c_int64()
    rc = _load().orc_alg4(g.n, g.row_ptr, _col_or_dummy(g), lev if g.n else np.zeros(1, np.int32),
                          ctypes.byref(t0), ctypes.byref(t1), ctypes.byref(e0))
    if rc != 0:
        raise RuntimeError("orc_alg4 failed")
    m = g.m
    return Alg4Result(t0.value + t1.value, t0.value, t1.value, e0.value,
                      100.0 * e0.value / m if m else 0.0)


def count_emd(g: CSR) -> int:
    return int(_load().orc_count_emd(g.n, g.row_ptr, _col_or_dummy(g)))


def count_emd_entries(g: CSR, entries, threads: int = 1) -> int:
    """Triangles u < v < w whose edge uv has its entry (u, v) in ``entries``
    (CSR entry indices), by the same sorted-merge edge iterator, the entries
    shared among ``threads`` host threads.  All entries give T."""
    es = np.ascontiguousarray(entries, dtype=np.int64)
    if es.size and (es.min() < 0 or es.max() >= g.nnz):
        raise ValueError("entry out of range")
    return int(_load().orc_count_emd_entries(g.n, g.row_ptr, _col_or_dummy(g), es.size,
                                             es if es.size else np.zeros(1, np.int64), int(threads)))


def alg3(g: CSR, level: np.ndarray | None = None) -> int:
    if level is None:
        level, _ = bfs_levels(g)
    lev = np.ascontiguousarray(level, dtype=np.int32)
    return int(_load().orc_alg3(g.n, g.row_ptr, _col_or_dummy(g), lev if g.n else np.zeros(1, np.int32)))


def vertex_triangles(g: CSR) -> np.ndarray:
    tv = np.zeros(max(g.n, 1), np.uint64)
    _load().orc_vertex_triangles(g.n, g.row_ptr, _col_or_dummy(g), tv)
    return tv[:g.n]


def vertex_triangles_at(g: CSR, vertices) -> np.ndarray:
    """t(v) for the given vertices only, from the edges among each one's
    neighbours (cost about deg(v)^2 log d_max per vertex)."""
    vs = np.ascontiguousarray(vertices, dtype=np.int64)
    if vs.size and (vs.min() < 0 or vs.max() >= g.n):
        raise ValueError("vertex out of range")
    out = np.zeros(max(vs.size, 1), np.uint64)
    _load().orc_vertex_triangles_at(g.n, g.row_ptr, _col_or_dummy(g), vs.size, vs if vs.size else np.zeros(1, np.int64),
                                    out)
    return out[:vs.size]


def edge_support(g: CSR) -> np.ndarray:
    """Triangles through the edge of every CSR entry (uint32, nnz entries)."""
    sup = np.zeros(max(g.nnz, 1), np.uint32)
    _load().orc_edge_support(g.n, g.row_ptr, _col_or_dummy(g), sup)
    return sup[:g.nnz]


def edge_support_at(g: CSR, entries) -> np.ndarray:
    """edge_support for the given CSR entries only, one at a time."""
    es = np.ascontiguousarray(entries, dtype=np.int64)
    if es.size and (es.min() < 0 or es.max() >= g.nnz):
        raise ValueError("entry out of range")
    out = np.zeros(max(es.size, 1), np.uint32)
    _load().orc_edge_support_at(g.n, g.row_ptr, _col_or_dummy(g), es.size, es if es.size else np.zeros(1, np.int64),
                                out)
    return out[:es.size]


def relabel_degree(g: CSR):
    """Degree ordering: returns (relabelled CSR, perm) with perm[new] = old,
    new ids by decreasing degree, ties by increasing old id."""
    rp = np.zeros(g.n + 1, np.int64)
    col = np.zeros(max(g.nnz, 1), np.int32)
    perm = np.zeros(max(g.n, 1), np.int32)
    rc = _load().orc_relabel_degree(g.n, g.row_ptr, _col_or_dummy(g), rp, col, perm)
    if rc != 0:
        raise MemoryError("oracle relabel")
    return as_csr(g.n, rp, col[:g.nnz]), perm[:g.n]


def _floor_log2(v) -> np.ndarray:
    """floor(log2 v) for integers v >= 1, and 0 for v <= 1."""
    return np.array([max(int(x), 1).bit_length() - 1 for x in np.atleast_1d(v)], dtype=np.int64)


def bucket_work(g: CSR, level: np.ndarray, by_id: bool = False):
    """Units and elements per schedule bucket (the library's work split, not
    the paper's): for kind 0 the lists are N0+ (sizes |N0+|), for kind 1 the
    N1 lists.  Each horizontal edge {x, y} belongs, per kind, to the endpoint
    with the larger list (ties: larger id) unless the other list is empty.
    Owner x of kind k forms one unit with cnt owned partners and work = the
    sum of their list sizes; its bucket is (k * 32 + ob) * 32 + pb with
    ob = floor(log2 |list(x)|), pb = floor(log2 (work // cnt)), both capped at
    31; the unit adds work + |list(x)| elements.  ``by_id``: N0+ lists of the
    id orientation.  Returns int64 arrays units[2048], elements[2048]."""
    p = partition(g, level, by_id)
    n = g.n
    sizes = [p.up0.astype(np.int64), np.diff(p.rp1).astype(np.int64)]
    x = np.repeat(np.arange(n, dtype=np.int64), np.diff(p.rp0))   # every directed horizontal edge (x, y)
    y = p.c0.astype(np.int64)
    units = np.zeros(2048, dtype=np.int64)
    elements = np.zeros(2048, dtype=np.int64)
    for kind in (0, 1):
        s = sizes[kind]
        sx, sy = s[x], s[y]
        own = (sy > 0) & ((sx > sy) | ((sx == sy) & (x > y)))
        cnt = np.zeros(n, dtype=np.int64)
        work = np.zeros(n, dtype=np.int64)
        np.add.at(cnt, x[own], 1)
        np.add.at(work, x[own], sy[own])
        owners = np.nonzero(cnt)[0]
        if len(owners) == 0:
            continue
        ob = np.minimum(_floor_log2(s[owners]), 31)
        pb = np.minimum(_floor_log2(work[owners] // cnt[owners]), 31)
        b = (kind * 32 + ob) * 32 + pb
        np.add.at(units, b, 1)
        np.add.at(elements, b, work[owners] + s[owners])
    return units, elements
