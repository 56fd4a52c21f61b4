"""ctypes declarations of ``include/tc.h`` (argument marshalling only).

Every function keeps its C name.  Loading fails loudly when ``libtc.so`` has
not been built: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtc.so")

TC_OK = 0
TC_ERR_ARG = -1
TC_ERR_RANGE = -2
TC_ERR_OVERFLOW = -3
TC_ERR_CAPACITY = -4
TC_ERR_WORKSPACE = -5
TC_ERR_HIP = -6
TC_ERR_NO_DEVICE = -7
TC_ERR_INVALID_CSR = -8
TC_ERR_TOO_LARGE = -9
TC_COUNT_ERROR = (1 << 64) - 1

TC_STRAT_AUTO = -1
TC_STRAT_WAVE_HASH = 0
TC_STRAT_WG_HASH = 1
TC_STRAT_BSEARCH = 2
TC_STRAT_MERGE = 3
TC_NUM_STRATEGIES = 4
STRATEGY_NAMES = ["wave_hash", "wg_hash", "bsearch", "merge"]

TC_SCHED_HEURISTIC = 0
TC_SCHED_TABLE = 1
TC_ORIENT_RANK = 0
TC_ORIENT_ID = 1
TC_NUM_BUCKETS = 2048
TC_MLP_IN = 3

TC_VALIDATE = 1
TC_TIMING = 2


class tc_options(ctypes.Structure):
    _fields_ = [
        ("schedule", ctypes.c_int32),
        ("force_strategy", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("wave_slots", ctypes.c_int32),
        ("wg_slots", ctypes.c_int32),
        ("chunk_work", ctypes.c_int32),
        ("grid_blocks", ctypes.c_int32),
        ("wave_max_owner", ctypes.c_int32),
        ("merge_max_owner", ctypes.c_int32),
        ("sched_table", ctypes.c_void_p),
        ("batch_group_entries", ctypes.c_int64),
        ("wg_slice_max", ctypes.c_int32),
        ("orientation", ctypes.c_int32),
    ]


class tc_stats(ctypes.Structure):
    _fields_ = [
        ("T0", ctypes.c_uint64),
        ("T1", ctypes.c_uint64),
        ("e0", ctypes.c_int64),
        ("units", ctypes.c_int64),
        ("items", ctypes.c_int64),
        ("probes", ctypes.c_int64),
        ("hashed", ctypes.c_int64),
        ("levels", ctypes.c_int32),
        ("bfs_rounds", ctypes.c_int32),
        ("ms_bfs", ctypes.c_float),
        ("ms_partition", ctypes.c_float),
        ("ms_bucket", ctypes.c_float),
        ("ms_isect", ctypes.c_float),
        ("strategy_items", ctypes.c_int32 * TC_NUM_STRATEGIES),
    ]


_lib = None

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_u64 = ctypes.c_uint64
_f32 = ctypes.c_float
_sz = ctypes.c_size_t
_P = ctypes.POINTER

_SIGNATURES = {
    "tc_last_error": (ctypes.c_int, []),
    "tc_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "tc_version": (ctypes.c_int, []),
    "tc_thread_release": (ctypes.c_int, []),
    "tc_build_csr_ws": (ctypes.c_int, [_i32, _i64, _P(_sz)]),
    "tc_build_csr": (ctypes.c_int, [_i32, _i64, _vp, _vp, _vp, _vp, _i64, _P(_i64), _vp, _sz, _vp]),
    "tc_bfs_levels_ws": (ctypes.c_int, [_i32, _i64, _P(_sz)]),
    "tc_bfs_levels": (ctypes.c_int, [_i32, _i64, _vp, _vp, _vp, _P(_i32), _vp, _sz, _vp]),
    "tc_count_ws": (ctypes.c_int, [_i32, _i64, _P(tc_options), _P(_sz)]),
    "tc_count": (ctypes.c_uint64, [_i32, _i64, _vp, _vp, _vp, _P(tc_options), _P(tc_stats), _vp, _sz, _vp]),
    "tc_count_profile": (ctypes.c_uint64, [_i32, _i64, _vp, _vp, _vp, _P(tc_options), _P(tc_stats), _vp, _vp, _sz,
                                           _vp]),
    "tc_vertex_triangles": (ctypes.c_uint64, [_i32, _i64, _vp, _vp, _vp, _P(tc_options), _vp, _P(tc_stats), _vp,
                                              _sz, _vp]),
    "tc_edge_support_ws": (ctypes.c_int, [_i32, _i64, _P(tc_options), _P(_sz)]),
    "tc_edge_support": (ctypes.c_uint64, [_i32, _i64, _vp, _vp, _vp, _P(tc_options), _vp, _P(tc_stats), _vp, _sz,
                                          _vp]),
    "tc_relabel_degree_ws": (ctypes.c_int, [_i32, _i64, _P(_sz)]),
    "tc_relabel_degree": (ctypes.c_int, [_i32, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "tc_count_cover_edge": (ctypes.c_uint64, [_i32, _i64, _vp, _vp, _vp, _P(tc_options), _P(tc_stats), _vp, _sz,
                                              _vp]),
    "tc_count_batched_ws": (ctypes.c_int, [_i32, _vp, _vp, _P(tc_options), _P(_sz)]),
    "tc_count_batched": (ctypes.c_uint64, [_i32, _vp, _vp, _vp, _vp, _vp, _P(tc_options), _vp, _P(tc_stats), _vp,
                                           _sz, _vp]),
    "tc_batch_plan_create": (ctypes.c_int, [_i32, _vp, _vp, _vp, _vp, _P(tc_options), _vp, _vp, _sz, _vp,
                                            _P(_vp)]),
    "tc_batch_plan_launch": (ctypes.c_int, [_vp, _vp]),
    "tc_bfs_levels_batched": (ctypes.c_int, [_i32, _vp, _vp, _vp, _vp, _vp, _P(_i32), _vp, _sz, _vp]),
    "tc_batch_plan_destroy": (ctypes.c_int, [_vp]),
    "tc_schedule_table": (ctypes.c_int, [_i32, _i64, _P(tc_options), _vp, _vp]),
    "tc_count_noalloc": (ctypes.c_int, [_i32, _i64, _vp, _vp, _vp, _P(tc_options), _vp, _vp]),
    "tc_mlp_param_count": (ctypes.c_int, [_i32, _i32, _P(_i64)]),
    "tc_mlp_init": (ctypes.c_int, [_vp, _i32, _i32, _u64, _vp]),
    "tc_mlp_forward": (ctypes.c_int, [_vp, _i32, _i32, _vp, _i32, _vp, _vp]),
    "tc_mlp_grad_ws": (ctypes.c_int, [_i32, _i32, _i32, _P(_sz)]),
    "tc_mlp_grad": (ctypes.c_int, [_vp, _i32, _i32, _vp, _vp, _vp, _vp, _i32, _vp, _vp, _vp, _sz, _vp]),
    "tc_mlp_adam": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i64, _i32, _f32, _f32, _f32, _f32, _vp]),
    "tc_mlp_train_ws": (ctypes.c_int, [_i32, _i32, _i32, _P(_sz)]),
    "tc_mlp_train": (ctypes.c_int, [_vp, _vp, _vp, _i32, _i32, _vp, _vp, _vp, _vp, _i32, _i32, _i32, _f32, _f32,
                                    _f32, _f32, _vp, _vp, _sz, _vp]),
    "tc_mlp_schedule": (ctypes.c_int, [_vp, _i32, _i32, _P(tc_options), _vp, _vp, _vp]),
    "tc_partition_ws": (ctypes.c_int, [_i32, _i64, _P(_sz)]),
    "tc_partition": (ctypes.c_int, [_i32, _i64, _vp, _vp, _vp, _i32, _vp, _vp, _vp, _vp, _vp, _P(_i64), _vp,
                                    _sz, _vp]),
}


def load():
    """Load ``libtc.so`` (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2309_09064_amd.build.build()")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def declared_functions():
    return sorted(_SIGNATURES)


def __getattr__(name):
    if name in _SIGNATURES:
        return getattr(load(), name)
    raise AttributeError(name)
