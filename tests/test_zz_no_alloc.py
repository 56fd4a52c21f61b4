"""tc_count_noalloc (the count that allocates nothing) against tc_count,
through the C ABI: {T, T0, T1, |E0|} bit-exact on two calls in a row, the
second on a smaller graph (the shared scratch keeps the first call's
contents), with computed and with given levels, under a forced strategy,
and graphs beyond the fixed scratch rejected before any device work."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

import graphgen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2309_09064_amd as tc
    return tc


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()


def graph(scale, seed):
    n, s, d = graphgen.kronecker(scale, seed=seed)
    g = oracle.build_csr(n, s, d)
    return g, dev(g.row_ptr.astype(np.int32)), dev(g.col)


def noalloc(tc, g, rp, col, levels=None, options=None):
    lib = tc._capi.load()
    out = torch.full((4,), -1, dtype=torch.int64, device="cuda")
    opt = ctypes.byref(options.to_c()) if options is not None else None
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.tc_count_noalloc(g.n, g.nnz, ctypes.c_void_p(rp.data_ptr()), ctypes.c_void_p(col.data_ptr()),
                              ctypes.c_void_p(levels.data_ptr()) if levels is not None else None, opt,
                              ctypes.c_void_p(out.data_ptr()), stream)
    assert rc == 0, tc._capi.load().tc_strerror(rc)
    torch.cuda.synchronize()
    return tuple(int(x) for x in out.cpu().tolist())


def reference(tc, rp, col, levels=None, options=None):
    r = tc.count(rp, col, levels, options)
    return (r.T, r.T0, r.T1, r.e0)


def test_two_calls_second_smaller(tc):
    big, rp1, col1 = graph(17, 3)
    small, rp2, col2 = graph(11, 4)
    a = noalloc(tc, big, rp1, col1)
    b = noalloc(tc, small, rp2, col2)
    assert a == reference(tc, rp1, col1)
    assert b == reference(tc, rp2, col2)
    assert a[0] == oracle.alg4(big).T and b[0] == oracle.alg4(small).T


def test_given_levels_and_forced_strategy(tc):
    g, rp, col = graph(14, 5)
    half = torch.div(tc.bfs_levels(rp, col)[0], 2, rounding_mode="floor").contiguous()
    assert noalloc(tc, g, rp, col, half) == reference(tc, rp, col, half)
    for s in (0, 1, 3):
        opts = tc.Options(force_strategy=s)
        assert noalloc(tc, g, rp, col, options=opts) == reference(tc, rp, col, options=opts)
    opts = tc.Options(orientation=tc.TC_ORIENT_ID)
    assert noalloc(tc, g, rp, col, options=opts) == reference(tc, rp, col)
    g2, rp2, col2 = graph(9, 6)
    assert noalloc(tc, g2, rp2, col2) == reference(tc, rp2, col2)


SCRATCH = 256 << 20


def count_ws(tc, g):
    b = ctypes.c_size_t()
    assert tc._capi.load().tc_count_ws(g.n, g.nnz, None, ctypes.byref(b)) == 0
    return b.value


def test_largest_that_fits(tc):
    g, rp, col = graph(18, 3)
    assert count_ws(tc, g) <= SCRATCH
    assert noalloc(tc, g, rp, col) == reference(tc, rp, col)


def test_rejects_before_device_work(tc):
    lib = tc._capi.load()
    g, rp, col = graph(19, 3)
    assert count_ws(tc, g) > SCRATCH
    out = torch.zeros(4, dtype=torch.int64, device="cuda")
    assert lib.tc_count_noalloc(g.n, g.nnz, ctypes.c_void_p(rp.data_ptr()), ctypes.c_void_p(col.data_ptr()), None,
                                None, ctypes.c_void_p(out.data_ptr()), None) == -9
    assert int(out.abs().sum()) == 0
    fake = ctypes.c_void_p(0x1000)
    assert lib.tc_count_noalloc(1 << 20, 1 << 24, fake, fake, None, None, fake, None) == -9
    opt = tc._capi.tc_options()
    opt.flags = tc.TC_TIMING
    assert lib.tc_count_noalloc(100, 200, fake, fake, None, ctypes.byref(opt), fake, None) == -1
    assert lib.tc_count_noalloc(100, 200, fake, fake, None, None, None, None) == -1
