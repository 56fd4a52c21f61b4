"""Host-side checks of the C ABI (no GPU): the library loads, exports every
function include/tc.h declares, and rejects bad arguments before any device
work.  No compute call is made."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

from paper_2309_09064_amd import _capi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(tc_[a-z0-9_]+)\s*\(", text))
    return names


@pytest.fixture(scope="module")
def lib():
    return _capi.load()


def test_library_exports_every_declared_function(lib):
    declared = header_functions()
    assert declared, "no declarations found"
    for name in declared:
        assert hasattr(lib, name), name
    assert declared == set(_capi.declared_functions())


def test_version_and_strerror(lib):
    assert lib.tc_version() >= 10000
    for code in range(0, -9, -1):
        assert lib.tc_strerror(code)
    assert lib.tc_strerror(-99) == b"unknown error"


def size_q(fn, *args):
    out = ctypes.c_size_t()
    rc = fn(*args, ctypes.byref(out))
    return rc, out.value


def test_workspace_queries(lib):
    rc, a = size_q(lib.tc_bfs_levels_ws, 1000, 20000)
    assert rc == 0 and a > 0
    rc, b = size_q(lib.tc_bfs_levels_ws, 100000, 2000000)
    assert rc == 0 and b > a
    rc, c = size_q(lib.tc_build_csr_ws, 1024, 16384)
    assert rc == 0 and c >= 2 * 2 * 16384 * 8
    rc, d = size_q(lib.tc_partition_ws, 1024, 20000)
    assert rc == 0 and d > 20000
    out = ctypes.c_size_t()
    assert lib.tc_count_ws(1024, 20000, None, ctypes.byref(out)) == 0 and out.value > 0
    rc, e = size_q(lib.tc_bfs_levels_ws, 0, 0)
    assert rc == 0


def test_bad_sizes_rejected(lib):
    out = ctypes.c_size_t()
    assert lib.tc_bfs_levels_ws(-1, 0, ctypes.byref(out)) == _capi.TC_ERR_ARG
    assert lib.tc_bfs_levels_ws(10, -5, ctypes.byref(out)) == _capi.TC_ERR_ARG
    assert lib.tc_bfs_levels_ws(10, 1 << 31, ctypes.byref(out)) == _capi.TC_ERR_OVERFLOW
    assert lib.tc_build_csr_ws(10, 1 << 30, ctypes.byref(out)) == _capi.TC_ERR_OVERFLOW
    assert lib.tc_bfs_levels_ws(0, 4, ctypes.byref(out)) == _capi.TC_ERR_ARG
    assert lib.tc_count_ws(10, 10, None, None) == _capi.TC_ERR_ARG
    assert lib.tc_last_error() == _capi.TC_ERR_ARG


@pytest.mark.parametrize("field,value", [("schedule", 7), ("force_strategy", 9), ("force_strategy", -2),
                                         ("wave_slots", 100), ("wave_slots", 8192), ("wg_slots", 512),
                                         ("wg_slots", 65536), ("chunk_work", -1), ("flags", 4)])
def test_bad_options_rejected(lib, field, value):
    opt = _capi.tc_options()
    setattr(opt, field, value)
    out = ctypes.c_size_t()
    assert lib.tc_count_ws(100, 100, ctypes.byref(opt), ctypes.byref(out)) == _capi.TC_ERR_ARG


def test_count_rejects_null_and_small_workspace_before_device(lib):
    fake = ctypes.c_void_p(0x1000)
    # NULL row_ptr
    T = lib.tc_count(10, 20, None, fake, None, None, None, fake, 1 << 20, None)
    assert T == _capi.TC_COUNT_ERROR and lib.tc_last_error() == _capi.TC_ERR_ARG
    # too-small workspace
    T = lib.tc_count(10, 20, fake, fake, None, None, None, fake, 16, None)
    assert T == _capi.TC_COUNT_ERROR and lib.tc_last_error() == _capi.TC_ERR_WORKSPACE
    # misaligned workspace
    T = lib.tc_count(10, 20, fake, fake, None, None, None, ctypes.c_void_p(0x1001), 1 << 30, None)
    assert T == _capi.TC_COUNT_ERROR and lib.tc_last_error() == _capi.TC_ERR_WORKSPACE
    # nnz that does not fit int32 CSR
    T = lib.tc_count(10, 1 << 31, fake, fake, None, None, None, fake, 1 << 30, None)
    assert T == _capi.TC_COUNT_ERROR and lib.tc_last_error() == _capi.TC_ERR_OVERFLOW


def test_build_csr_rejects_before_device(lib):
    fake = ctypes.c_void_p(0x1000)
    nnz = ctypes.c_int64()
    assert lib.tc_build_csr(10, 5, None, fake, fake, fake, 10, ctypes.byref(nnz), fake, 1 << 20,
                            None) == _capi.TC_ERR_ARG
    assert lib.tc_build_csr(10, 1 << 30, fake, fake, fake, fake, 10, ctypes.byref(nnz), fake, 1 << 20,
                            None) == _capi.TC_ERR_OVERFLOW
    assert lib.tc_build_csr(10, 5, fake, fake, fake, fake, 10, ctypes.byref(nnz), fake, 8,
                            None) == _capi.TC_ERR_WORKSPACE
