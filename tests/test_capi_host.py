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
                                         ("wg_slots", 65536), ("chunk_work", -1), ("flags", 4),
                                         ("merge_max_owner", -2), ("merge_max_owner", 32), ("wg_slice_max", 100),
                                         ("wg_slice_max", 32), ("wg_slice_max", 32768), ("orientation", 2),
                                         ("orientation", -1)])
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


def test_table_schedule_needs_a_table_before_device(lib):
    fake = ctypes.c_void_p(0x1000)
    opt = _capi.tc_options()
    opt.schedule = _capi.TC_SCHED_TABLE
    out = ctypes.c_size_t()
    assert lib.tc_count_ws(10, 20, ctypes.byref(opt), ctypes.byref(out)) == _capi.TC_OK   # size needs no table
    T = lib.tc_count(10, 20, fake, fake, None, ctypes.byref(opt), None, fake, 1 << 30, None)
    assert T == _capi.TC_COUNT_ERROR and lib.tc_last_error() == _capi.TC_ERR_ARG


def test_count_profile_needs_a_buffer_before_device(lib):
    fake = ctypes.c_void_p(0x1000)
    T = lib.tc_count_profile(10, 20, fake, fake, None, None, None, None, fake, 1 << 30, None)
    assert T == _capi.TC_COUNT_ERROR and lib.tc_last_error() == _capi.TC_ERR_ARG


@pytest.mark.parametrize("H,K,ok", [(8, 4, True), (32, 4, True), (64, 8, True), (16, 1, True), (12, 4, False),
                                    (32, 0, False), (32, 9, False), (128, 4, False)])
def test_mlp_sizes(lib, H, K, ok):
    cnt = ctypes.c_int64()
    rc = lib.tc_mlp_param_count(H, K, ctypes.byref(cnt))
    if ok:
        assert rc == _capi.TC_OK and cnt.value == 3 * H + H + H * H + H + K * H + K
    else:
        assert rc == _capi.TC_ERR_ARG


def test_mlp_args_rejected_before_device(lib):
    fake = ctypes.c_void_p(0x1000)
    sz = ctypes.c_size_t()
    assert lib.tc_mlp_grad_ws(32, 4, 0, ctypes.byref(sz)) == _capi.TC_ERR_ARG
    assert lib.tc_mlp_grad_ws(32, 4, 10, ctypes.byref(sz)) == _capi.TC_OK and sz.value >= 10 * (4 * 32 + 2) * 4
    assert lib.tc_mlp_train_ws(32, 4, 10, ctypes.byref(sz)) == _capi.TC_OK
    # missing workspace / too small / misaligned
    assert lib.tc_mlp_grad(fake, 32, 4, fake, fake, fake, None, 10, fake, None, None, 0, None) == _capi.TC_ERR_WORKSPACE
    assert lib.tc_mlp_grad(fake, 32, 4, fake, fake, fake, None, 10, fake, None, fake, 64, None) == _capi.TC_ERR_WORKSPACE
    # Adam: step 0, beta outside [0, 1), negative lr
    assert lib.tc_mlp_adam(fake, fake, fake, fake, 10, 0, 0.01, 0.9, 0.999, 1e-8, None) == _capi.TC_ERR_ARG
    assert lib.tc_mlp_adam(fake, fake, fake, fake, 10, 1, 0.01, 1.0, 0.999, 1e-8, None) == _capi.TC_ERR_ARG
    assert lib.tc_mlp_adam(fake, fake, fake, fake, 10, 1, -0.01, 0.9, 0.999, 1e-8, None) == _capi.TC_ERR_ARG
    assert lib.tc_mlp_adam(fake, fake, fake, fake, 0, 1, 0.01, 0.9, 0.999, 1e-8, None) == _capi.TC_OK   # no-op
    # the schedule needs K = 4 strategies and valid options
    opt = _capi.tc_options()
    assert lib.tc_mlp_schedule(fake, 32, 3, ctypes.byref(opt), fake, None, None) == _capi.TC_ERR_ARG
    opt.wave_slots = 100
    assert lib.tc_mlp_schedule(fake, 32, 4, ctypes.byref(opt), fake, None, None) == _capi.TC_ERR_ARG
    assert lib.tc_mlp_forward(fake, 32, 4, fake, 0, fake, None) == _capi.TC_OK   # zero rows: no-op
    assert lib.tc_mlp_forward(fake, 32, 4, fake, -1, fake, None) == _capi.TC_ERR_ARG


def _i64s(v):
    return (ctypes.c_int64 * len(v))(*v)


# bad offsets: not starting at 0, decreasing, edges on an empty graph, a
# graph beyond int32 (overflow)
@pytest.mark.parametrize("voff,eoff,code", [
    ([1, 5, 10], [0, 8, 20], _capi.TC_ERR_ARG),
    ([0, 5, 10], [2, 8, 20], _capi.TC_ERR_ARG),
    ([0, 6, 5], [0, 8, 20], _capi.TC_ERR_ARG),
    ([0, 5, 10], [0, 9, 7], _capi.TC_ERR_ARG),
    ([0, 0, 10], [0, 4, 20], _capi.TC_ERR_ARG),
    ([0, 5, 5 + (1 << 31)], [0, 8, 20], _capi.TC_ERR_OVERFLOW),
    ([0, 5, 10], [0, 8, 8 + (1 << 31)], _capi.TC_ERR_OVERFLOW),
])
def test_batch_offsets_rejected_before_device(lib, voff, eoff, code):
    fake = ctypes.c_void_p(0x1000)
    T = lib.tc_count_batched(len(voff) - 1, _i64s(voff), _i64s(eoff), fake, fake, None, None, fake, None, fake,
                             1 << 40, None)
    assert T == _capi.TC_COUNT_ERROR and lib.tc_last_error() == code
    sz = ctypes.c_size_t()
    assert lib.tc_count_batched_ws(len(voff) - 1, _i64s(voff), _i64s(eoff), None, ctypes.byref(sz)) == code
    plan = ctypes.c_void_p()
    assert lib.tc_batch_plan_create(len(voff) - 1, _i64s(voff), _i64s(eoff), fake, fake, None, fake, fake, 1 << 40,
                                    None, ctypes.byref(plan)) == code
    assert not plan.value


def test_batch_needs_counts_buffer_and_workspace(lib):
    fake = ctypes.c_void_p(0x1000)
    voff, eoff = _i64s([0, 4, 10]), _i64s([0, 8, 20])
    T = lib.tc_count_batched(2, voff, eoff, fake, fake, None, None, None, None, fake, 1 << 30, None)
    assert T == _capi.TC_COUNT_ERROR and lib.tc_last_error() == _capi.TC_ERR_ARG
    sz, sz1 = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.tc_count_batched_ws(2, voff, eoff, None, ctypes.byref(sz)) == _capi.TC_OK
    assert lib.tc_count_ws(10, 20, None, ctypes.byref(sz1)) == _capi.TC_OK
    assert sz.value > sz1.value   # the rebased copy of the group CSR and the BFS scratch
    T = lib.tc_count_batched(2, voff, eoff, fake, fake, None, None, fake, None, fake, 256, None)
    assert T == _capi.TC_COUNT_ERROR and lib.tc_last_error() == _capi.TC_ERR_WORKSPACE


def test_batch_groups_shrink_the_workspace(lib):
    # cutting the batch into groups sizes the workspace for the largest group
    voff = _i64s([0] + [1000 * (i + 1) for i in range(64)])
    eoff = _i64s([0] + [20000 * (i + 1) for i in range(64)])
    whole, grouped = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.tc_count_batched_ws(64, voff, eoff, None, ctypes.byref(whole)) == _capi.TC_OK
    opt = _capi.tc_options()
    opt.batch_group_entries = 40000
    assert lib.tc_count_batched_ws(64, voff, eoff, ctypes.byref(opt), ctypes.byref(grouped)) == _capi.TC_OK
    assert grouped.value * 8 < whole.value
    opt.batch_group_entries = -1
    assert lib.tc_count_batched_ws(64, voff, eoff, ctypes.byref(opt), ctypes.byref(grouped)) == _capi.TC_ERR_ARG


def test_batch_plan_arguments(lib):
    fake = ctypes.c_void_p(0x1000)
    voff, eoff = _i64s([0, 4, 10]), _i64s([0, 8, 20])
    plan = ctypes.c_void_p()
    for flags in (_capi.TC_TIMING, _capi.TC_VALIDATE):   # both read results on the host
        opt = _capi.tc_options()
        opt.flags = flags
        assert lib.tc_batch_plan_create(2, voff, eoff, fake, fake, ctypes.byref(opt), fake, fake, 1 << 30, None,
                                        ctypes.byref(plan)) == _capi.TC_ERR_ARG
    assert lib.tc_batch_plan_create(2, voff, eoff, fake, fake, None, fake, fake, 1 << 30, None, None) == \
        _capi.TC_ERR_ARG
    assert lib.tc_batch_plan_create(2, voff, eoff, fake, fake, None, None, fake, 1 << 30, None,
                                    ctypes.byref(plan)) == _capi.TC_ERR_ARG
    assert lib.tc_batch_plan_create(2, voff, eoff, fake, fake, None, fake, fake, 64, None,
                                    ctypes.byref(plan)) == _capi.TC_ERR_WORKSPACE
    assert lib.tc_batch_plan_launch(None, None) == _capi.TC_ERR_ARG
    assert lib.tc_batch_plan_destroy(None) == _capi.TC_OK


def test_vertex_triangles_needs_an_output_before_device(lib):
    fake = ctypes.c_void_p(0x1000)
    T = lib.tc_vertex_triangles(10, 20, fake, fake, None, None, None, None, fake, 1 << 30, None)
    assert T == _capi.TC_COUNT_ERROR and lib.tc_last_error() == _capi.TC_ERR_ARG
    T = lib.tc_vertex_triangles(10, 20, fake, fake, None, None, fake, None, fake, 16, None)
    assert T == _capi.TC_COUNT_ERROR and lib.tc_last_error() == _capi.TC_ERR_WORKSPACE


def test_edge_support_needs_an_output_and_its_workspace(lib):
    fake = ctypes.c_void_p(0x1000)
    T = lib.tc_edge_support(10, 20, fake, fake, None, None, None, None, fake, 1 << 30, None)
    assert T == _capi.TC_COUNT_ERROR and lib.tc_last_error() == _capi.TC_ERR_ARG
    rc, plain = size_q(lib.tc_count_ws, 1000, 20000, None)
    rc2, edge = size_q(lib.tc_edge_support_ws, 1000, 20000, None)
    assert rc == 0 and rc2 == 0 and edge >= plain + 2 * 4 * 20000
    T = lib.tc_edge_support(1000, 20000, fake, fake, None, None, fake, None, fake, plain, None)
    assert T == _capi.TC_COUNT_ERROR and lib.tc_last_error() == _capi.TC_ERR_WORKSPACE


def test_partition_rejects_bad_orientation_before_device(lib):
    fake = ctypes.c_void_p(0x1000)
    e0 = ctypes.c_int64()
    for orient in (2, -1):
        assert lib.tc_partition(10, 20, fake, fake, fake, orient, fake, fake, fake, fake, fake, ctypes.byref(e0), fake,
                                1 << 30, None) == _capi.TC_ERR_ARG


@pytest.mark.parametrize("struct", ["tc_options", "tc_stats"])
def test_struct_layout_matches_header(tmp_path, struct):
    """The ctypes mirrors of the option and statistics structs have the C
    layout: every field's offset and the struct's size, as gcc lays out
    include/tc.h."""
    cls = getattr(_capi, struct)
    lines = [f'printf("size %zu\\n", sizeof({struct}));']
    for name, _ in cls._fields_:
        lines.append(f'printf("{name} %zu\\n", offsetof({struct}, {name}));')
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "tc.h"\nint main(void) {\n' +
                   "\n".join(lines) + "\nreturn 0;\n}\n")
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(l.split() for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                 text=True).stdout.splitlines())
    assert int(out["size"]) == ctypes.sizeof(cls)
    for name, _ in cls._fields_:
        assert int(out[name]) == getattr(cls, name).offset, name
