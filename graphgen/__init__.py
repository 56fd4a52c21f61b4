"""Seeded synthetic graph generators (raw edge tuples, before cleanup).

Both the GPU library's tests/benchmarks and the CPU oracle draw their inputs
from here; the module holds none of the triangle-counting arithmetic.  The
native part (``graphgen.c``) is built with gcc by :func:`build`.

Generators
----------
* :func:`kronecker` -- Graph500-style R-MAT tuples, ``edgefactor * 2**scale``
  of them, initiator (A, B, C, D) = (0.57, 0.19, 0.19, 0.05) by default,
  vertex ids permuted by a seeded Fisher-Yates shuffle.
* :func:`erdos_renyi` -- G(n, p) by geometric skipping.
* :func:`chung_lu` -- expected-degree power-law graph.
* :func:`batch_recipe` -- the mixed batch of many small ER/Kronecker graphs.

All outputs are ``(n, src, dst)`` with int32 numpy arrays; self-loops and
duplicates are still present.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB_PATH = os.path.join(_HERE, "libgraphgen.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``graphgen.c`` into ``libgraphgen.so`` (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        lib.gg_kronecker.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_uint64, i32p, i32p]
        lib.gg_kronecker.restype = ctypes.c_int
        lib.gg_erdos_renyi.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_uint64,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
        lib.gg_erdos_renyi.restype = ctypes.c_int64
        lib.gg_chung_lu_weights.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_double,
                                            np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")]
        lib.gg_chung_lu_weights.restype = ctypes.c_double
        lib.gg_chung_lu.argtypes = [ctypes.c_int64,
                                    np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS"),
                                    ctypes.c_int64, ctypes.c_uint64, i32p, i32p]
        lib.gg_chung_lu.restype = ctypes.c_int
        lib.gg_permutation.argtypes = [ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint64, i32p]
        lib.gg_permutation.restype = None
        lib.gg_draws.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64,
                                 np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")]
        lib.gg_draws.restype = None
        _lib = lib
    return _lib


def draws(seed: int, stream: int, count: int) -> np.ndarray:
    """``count`` raw 64-bit counter-based draws for (seed, stream)."""
    out = np.empty(count, dtype=np.uint64)
    _load().gg_draws(seed, stream, count, out)
    return out


def uniforms(seed: int, stream: int, count: int) -> np.ndarray:
    """``count`` doubles in [0, 1) from the counter-based generator."""
    return (draws(seed, stream, count) >> np.uint64(11)).astype(np.float64) * (1.0 / 2.0 ** 53)


def permutation(n: int, seed: int, stream: int = 7) -> np.ndarray:
    """Seeded Fisher-Yates permutation of ``range(n)`` (int32)."""
    out = np.empty(n, dtype=np.int32)
    _load().gg_permutation(n, seed, stream, out)
    return out


def kronecker(scale: int, edgefactor: int = 16, A: float = 0.57, B: float = 0.19, C: float = 0.19,
              seed: int = 1):
    """Graph500-style Kronecker tuples: returns ``(n, src, dst)``."""
    n = 1 << scale
    m = edgefactor * n
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    rc = _load().gg_kronecker(scale, edgefactor, A, B, C, seed, src, dst)
    if rc != 0:
        raise RuntimeError(f"gg_kronecker failed ({rc})")
    return n, src, dst


def erdos_renyi(n: int, p: float, seed: int):
    """G(n, p) tuples (each undirected edge once, w < v): ``(n, src, dst)``."""
    lib = _load()
    cnt = lib.gg_erdos_renyi(n, p, seed, None, None, 0)
    if cnt < 0:
        raise RuntimeError(f"gg_erdos_renyi failed ({cnt})")
    src = np.empty(max(cnt, 1), dtype=np.int32)
    dst = np.empty(max(cnt, 1), dtype=np.int32)
    got = lib.gg_erdos_renyi(n, p, seed, src.ctypes.data, dst.ctypes.data, cnt)
    if got != cnt:
        raise RuntimeError("gg_erdos_renyi: count and fill passes disagree")
    return n, src[:cnt], dst[:cnt]


def chung_lu_weights(n: int, gamma: float = 2.1, mean_deg: float = 32.0, max_deg: float = 2.0 ** 17):
    """Expected-degree weights and the fitted offset i0."""
    w = np.empty(n, dtype=np.float64)
    i0 = _load().gg_chung_lu_weights(n, gamma, mean_deg, max_deg, w)
    if i0 < 0:
        raise RuntimeError("gg_chung_lu_weights failed")
    return w, i0


def chung_lu(n: int, gamma: float = 2.1, mean_deg: float = 32.0, max_deg: float = 2.0 ** 17,
             seed: int = 1):
    """Chung-Lu tuples with ``round(sum(w)/2)`` draws: ``(n, src, dst)``."""
    w, _ = chung_lu_weights(n, gamma, mean_deg, max_deg)
    m = int(round(w.sum() / 2.0))
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    rc = _load().gg_chung_lu(n, w, m, seed, src, dst)
    if rc != 0:
        raise RuntimeError(f"gg_chung_lu failed ({rc})")
    return n, src, dst


@dataclass(frozen=True)
class BatchMember:
    kind: str          # "er" or "kron"
    n: int
    seed: int
    p: float = 0.0     # ER edge probability
    scale: int = 0     # Kronecker scale


def batch_recipe(count: int = 4096, seed: int = 0, n_min: int = 64, n_max: int = 65536,
                 deg_lo: float = 8.0, deg_hi: float = 64.0, scale_lo: int = 8, scale_hi: int = 16):
    """The mixed batch: first half ER with n log-uniform in [n_min, n_max] and
    mean degree uniform in [deg_lo, deg_hi]; second half Kronecker with scale
    uniform in {scale_lo..scale_hi}, edgefactor 16.  Member i uses graph seed
    1000 + i; the size draws use ``seed``."""
    half = count // 2
    u = uniforms(seed, 11, 3 * count)
    out = []
    for i in range(count):
        gseed = 1000 + i
        if i < half:
            n = int(round(math.exp(math.log(n_min) + u[3 * i] * (math.log(n_max) - math.log(n_min)))))
            n = max(n_min, min(n_max, n))
            d = deg_lo + u[3 * i + 1] * (deg_hi - deg_lo)
            p = min(1.0, d / (n - 1))
            out.append(BatchMember("er", n, gseed, p=p))
        else:
            s = scale_lo + int(u[3 * i + 2] * (scale_hi - scale_lo + 1))
            s = min(s, scale_hi)
            out.append(BatchMember("kron", 1 << s, gseed, scale=s))
    return out


def batch_member_tuples(mem: BatchMember):
    """Raw tuples of one batch member."""
    if mem.kind == "er":
        return erdos_renyi(mem.n, mem.p, mem.seed)
    return kronecker(mem.scale, 16, seed=mem.seed)
