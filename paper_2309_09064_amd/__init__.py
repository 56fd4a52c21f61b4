"""MI355X triangle counting (cover-edge + forward + hashing, Bader 2023).

A thin torch-facing layer over the C ABI in ``include/tc.h``: it allocates
device tensors (outputs and workspaces) with PyTorch, passes raw pointers and
the current HIP stream, and converts status codes into exceptions.  Every
step of the computation runs in ``libtc.so``'s HIP kernels.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import torch

from . import _capi
from ._capi import (STRATEGY_NAMES, TC_COUNT_ERROR, TC_NUM_BUCKETS, TC_NUM_STRATEGIES, TC_ORIENT_ID,
                    TC_ORIENT_RANK, TC_SCHED_HEURISTIC, TC_SCHED_TABLE, TC_STRAT_AUTO, TC_STRAT_BSEARCH,
                    TC_STRAT_MERGE, TC_STRAT_WAVE_HASH, TC_STRAT_WG_HASH, TC_TIMING, TC_VALIDATE)

__all__ = ["TCError", "Options", "build_csr", "bfs_levels", "partition", "count", "count_profile", "workspace",
           "count_batched", "pack_csr", "Batch", "BatchPlan", "batch_workspace_bytes", "bfs_levels_batched", "schedule_table", "vertex_triangles", "edge_support",
           "relabel_by_degree", "count_cover_edge",
           "Counter", "CountResult", "new_profile",
           "STRATEGY_NAMES", "TC_STRAT_AUTO", "TC_STRAT_WAVE_HASH", "TC_STRAT_WG_HASH", "TC_STRAT_BSEARCH",
           "TC_STRAT_MERGE", "TC_SCHED_HEURISTIC", "TC_SCHED_TABLE", "TC_NUM_BUCKETS", "TC_NUM_STRATEGIES",
           "TC_VALIDATE", "TC_TIMING", "TC_ORIENT_RANK", "TC_ORIENT_ID"]


class TCError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = _capi.load().tc_strerror(code).decode()
        super().__init__(f"{where}: {msg} ({code})")


def _check(rc: int, where: str):
    if rc != 0:
        raise TCError(rc, where)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _require_i32_cuda(t, name):
    if t.dtype != torch.int32 or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous int32 CUDA tensor")


def workspace(nbytes: int, device=None):
    """A 256-byte aligned device workspace (a uint8 tensor view)."""
    dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
    raw = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=dev)
    off = (-raw.data_ptr()) % 256
    return raw[off:off + int(nbytes)] if nbytes else raw[off:off + 1]


@dataclass
class Options:
    schedule: int = TC_SCHED_HEURISTIC
    force_strategy: int = TC_STRAT_AUTO
    validate: bool = False
    timing: bool = False
    wave_slots: int = 0
    wg_slots: int = 0
    chunk_work: int = 0
    grid_blocks: int = 0
    wave_max_owner: int = 0
    merge_max_owner: int = 0            # 0 = default (31 for counts, 15 per vertex / edge), -1 = never
    sched_table: torch.Tensor | None = None   # int32[TC_NUM_BUCKETS] on the device: selects TC_SCHED_TABLE
    batch_group_entries: int = 0        # batched counts: vertices / entries per internal group; 0 = int32 limit
    wg_slice_max: int = 0               # longest owner slice of a workgroup table; 0 = wg_slots / 4
    orientation: int = TC_ORIENT_RANK   # N0+ lists by (degree, id) rank, or by id (TC_ORIENT_ID)

    def to_c(self):
        o = _capi.tc_options()
        if self.sched_table is not None:
            t = self.sched_table
            if t.dtype != torch.int32 or not t.is_cuda or not t.is_contiguous() or t.numel() != TC_NUM_BUCKETS:
                raise ValueError("sched_table must be a contiguous int32 CUDA tensor of TC_NUM_BUCKETS entries")
            o.schedule = TC_SCHED_TABLE
            o.sched_table = t.data_ptr()
        else:
            o.schedule = self.schedule
        o.force_strategy = self.force_strategy
        o.flags = (TC_VALIDATE if self.validate else 0) | (TC_TIMING if self.timing else 0)
        o.wave_slots = self.wave_slots
        o.wg_slots = self.wg_slots
        o.chunk_work = self.chunk_work
        o.grid_blocks = self.grid_blocks
        o.wave_max_owner = self.wave_max_owner
        o.merge_max_owner = self.merge_max_owner
        o.batch_group_entries = self.batch_group_entries
        o.wg_slice_max = self.wg_slice_max
        o.orientation = self.orientation
        return o


@dataclass
class CountResult:
    T: int
    T0: int
    T1: int
    e0: int
    units: int
    items: int
    probes: int
    hashed: int
    levels: int
    bfs_rounds: int
    ms: dict = field(default_factory=dict)
    strategy_items: dict = field(default_factory=dict)


def build_csr(n: int, src: torch.Tensor, dst: torch.Tensor, stream=None):
    """Simple undirected CSR (row_ptr, col_idx) from device tuples."""
    _require_i32_cuda(src, "src")
    _require_i32_cuda(dst, "dst")
    lib = _capi.load()
    m = src.numel()
    if dst.numel() != m:
        raise ValueError("src and dst differ in length")
    need = ctypes.c_size_t()
    _check(lib.tc_build_csr_ws(n, m, ctypes.byref(need)), "tc_build_csr_ws")
    ws = workspace(need.value, src.device)
    row_ptr = torch.empty(n + 1, dtype=torch.int32, device=src.device)
    col = torch.empty(max(2 * m, 1), dtype=torch.int32, device=src.device)
    nnz = ctypes.c_int64()
    _check(lib.tc_build_csr(n, m, _ptr(src), _ptr(dst), _ptr(row_ptr), _ptr(col), col.numel(),
                            ctypes.byref(nnz), _ptr(ws), need.value, _stream(stream)), "tc_build_csr")
    return row_ptr, col[:nnz.value]


def bfs_levels(row_ptr: torch.Tensor, col: torch.Tensor, stream=None):
    """Levels (int32 CUDA tensor) and the number of levels."""
    _require_i32_cuda(row_ptr, "row_ptr")
    _require_i32_cuda(col, "col")
    lib = _capi.load()
    n = row_ptr.numel() - 1
    nnz = col.numel()
    need = ctypes.c_size_t()
    _check(lib.tc_bfs_levels_ws(n, nnz, ctypes.byref(need)), "tc_bfs_levels_ws")
    ws = workspace(need.value, row_ptr.device)
    lev = torch.empty(max(n, 1), dtype=torch.int32, device=row_ptr.device)
    nlev = ctypes.c_int32()
    _check(lib.tc_bfs_levels(n, nnz, _ptr(row_ptr), _ptr(col), _ptr(lev), ctypes.byref(nlev), _ptr(ws),
                             need.value, _stream(stream)), "tc_bfs_levels")
    return lev[:n], nlev.value


def partition(row_ptr: torch.Tensor, col: torch.Tensor, levels: torch.Tensor, stream=None,
              orientation: int = TC_ORIENT_RANK):
    """The E0/E1 partition CSRs as a dict of device tensors (N0+ lists in the
    given orientation)."""
    for t, nm in ((row_ptr, "row_ptr"), (col, "col"), (levels, "levels")):
        _require_i32_cuda(t, nm)
    lib = _capi.load()
    n = row_ptr.numel() - 1
    nnz = col.numel()
    need = ctypes.c_size_t()
    _check(lib.tc_partition_ws(n, nnz, ctypes.byref(need)), "tc_partition_ws")
    ws = workspace(need.value, row_ptr.device)
    dev = row_ptr.device
    out = {
        "rp0": torch.empty(n + 1, dtype=torch.int32, device=dev),
        "c0": torch.empty(max(nnz, 1), dtype=torch.int32, device=dev),
        "up0": torch.empty(max(n, 1), dtype=torch.int32, device=dev),
        "rp1": torch.empty(n + 1, dtype=torch.int32, device=dev),
        "c1": torch.empty(max(nnz, 1), dtype=torch.int32, device=dev),
    }
    e0 = ctypes.c_int64()
    _check(lib.tc_partition(n, nnz, _ptr(row_ptr), _ptr(col), _ptr(levels), orientation, _ptr(out["rp0"]),
                            _ptr(out["c0"]), _ptr(out["up0"]), _ptr(out["rp1"]), _ptr(out["c1"]), ctypes.byref(e0),
                            _ptr(ws), need.value, _stream(stream)), "tc_partition")
    out["e0"] = e0.value
    out["up0"] = out["up0"][:n]
    return out


class Counter:
    """Reusable counting context: one workspace for repeated calls."""

    def __init__(self, n: int, nnz: int, options: Options | None = None, device=None):
        self.n, self.nnz = n, nnz
        self.options = options or Options()
        self._opt = self.options.to_c()
        lib = _capi.load()
        need = ctypes.c_size_t()
        _check(lib.tc_count_ws(n, nnz, ctypes.byref(self._opt), ctypes.byref(need)), "tc_count_ws")
        self.ws_bytes = need.value
        self.ws = workspace(need.value, device)

    def __call__(self, row_ptr, col, levels=None, stream=None, profile=None) -> CountResult:
        """Count; with ``profile`` (see :func:`new_profile`) the instrumented
        kernels also add the per-bucket costs into it."""
        lib = _capi.load()
        st = _capi.tc_stats()
        if profile is None:
            T = lib.tc_count(self.n, self.nnz, _ptr(row_ptr), _ptr(col), _ptr(levels), ctypes.byref(self._opt),
                             ctypes.byref(st), _ptr(self.ws), self.ws_bytes, _stream(stream))
        else:
            _check_profile(profile)
            T = lib.tc_count_profile(self.n, self.nnz, _ptr(row_ptr), _ptr(col), _ptr(levels),
                                     ctypes.byref(self._opt), ctypes.byref(st), _ptr(profile), _ptr(self.ws),
                                     self.ws_bytes, _stream(stream))
        if T == TC_COUNT_ERROR:
            raise TCError(lib.tc_last_error(), "tc_count_profile" if profile is not None else "tc_count")
        return CountResult(
            T=int(T), T0=int(st.T0), T1=int(st.T1), e0=int(st.e0), units=int(st.units), items=int(st.items),
            probes=int(st.probes), hashed=int(st.hashed), levels=int(st.levels), bfs_rounds=int(st.bfs_rounds),
            ms={"bfs": st.ms_bfs, "partition": st.ms_partition, "bucket": st.ms_bucket, "isect": st.ms_isect},
            strategy_items={STRATEGY_NAMES[k]: int(st.strategy_items[k]) for k in range(TC_NUM_STRATEGIES)})


def schedule_table(n: int, nnz: int, options: Options | None = None, device=None, stream=None) -> torch.Tensor:
    """The strategy tc_count gives every bucket under ``options`` for a graph
    of n vertices and nnz entries (int32 device tensor of TC_NUM_BUCKETS)."""
    dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
    opt = (options or Options()).to_c()
    t = torch.empty(TC_NUM_BUCKETS, dtype=torch.int32, device=dev)
    _check(_capi.load().tc_schedule_table(n, nnz, ctypes.byref(opt), _ptr(t), _stream(stream)), "tc_schedule_table")
    return t


PROFILE_LEN = TC_NUM_BUCKETS * TC_NUM_STRATEGIES * 3


def new_profile(device=None) -> torch.Tensor:
    """A zeroed per-(bucket, strategy) profile: int64 view of the C uint64
    array, shape [TC_NUM_BUCKETS, TC_NUM_STRATEGIES, 3] = (wavefront-ticks,
    elements, items)."""
    dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
    return torch.zeros(TC_NUM_BUCKETS, TC_NUM_STRATEGIES, 3, dtype=torch.int64, device=dev)


def _check_profile(p):
    if p.dtype != torch.int64 or not p.is_cuda or not p.is_contiguous() or p.numel() != PROFILE_LEN:
        raise ValueError("profile must come from new_profile()")


def count_profile(row_ptr: torch.Tensor, col: torch.Tensor, profile: torch.Tensor, levels: torch.Tensor | None = None,
                  options: Options | None = None, stream=None) -> CountResult:
    """tc_count_profile: count and add the per-bucket costs into ``profile``."""
    _require_i32_cuda(row_ptr, "row_ptr")
    _require_i32_cuda(col, "col")
    c = Counter(row_ptr.numel() - 1, col.numel(), options, row_ptr.device)
    return c(row_ptr, col, levels, stream, profile=profile)


def _result(T, st) -> CountResult:
    return CountResult(
        T=int(T), T0=int(st.T0), T1=int(st.T1), e0=int(st.e0), units=int(st.units), items=int(st.items),
        probes=int(st.probes), hashed=int(st.hashed), levels=int(st.levels), bfs_rounds=int(st.bfs_rounds),
        ms={"bfs": st.ms_bfs, "partition": st.ms_partition, "bucket": st.ms_bucket, "isect": st.ms_isect},
        strategy_items={STRATEGY_NAMES[k]: int(st.strategy_items[k]) for k in range(TC_NUM_STRATEGIES)})


@dataclass
class Batch:
    """A packed batch of graphs, each a CSR with local ids (see
    ``tc_count_batched`` in include/tc.h): graph g's n_g + 1 row pointers
    start at ``row_ptr[vtx_off[g] + g]``, its entries at
    ``col[edge_off[g]]``."""
    row_ptr: torch.Tensor     # int32 device, vtx_off[-1] + graphs entries
    col: torch.Tensor         # int32 device, edge_off[-1] entries (local ids)
    vtx_off: "object"         # numpy int64[graphs + 1]
    edge_off: "object"        # numpy int64[graphs + 1]

    @property
    def graphs(self) -> int:
        return len(self.vtx_off) - 1

    @classmethod
    def from_union(cls, row_ptr: torch.Tensor, col: torch.Tensor, vtx_off) -> "Batch":
        """Layout conversion (torch ops on the device, no counting): a CSR
        over the disjoint union with global ids, graph g owning the vertices
        [vtx_off[g], vtx_off[g+1]), becomes the packed per-graph CSRs with
        local ids.  Rows must hold only their own graph's vertices."""
        import numpy as np
        voff = np.ascontiguousarray(vtx_off, dtype=np.int64)
        G = len(voff) - 1
        dev = row_ptr.device
        voff_t = torch.from_numpy(voff).to(dev)
        rp64 = row_ptr.to(torch.int64)
        eoff_t = rp64[voff_t]
        n_g = voff_t[1:] - voff_t[:-1]
        slot_g = torch.repeat_interleave(torch.arange(G, device=dev), n_g + 1)
        slot_v = torch.arange(slot_g.numel(), device=dev) - slot_g      # vertex of each row-pointer slot
        rp_packed = (rp64[slot_v] - eoff_t[slot_g]).to(torch.int32)
        ent_g = torch.repeat_interleave(torch.arange(G, device=dev), eoff_t[1:] - eoff_t[:-1])
        col_local = (col.to(torch.int64) - voff_t[ent_g]).to(torch.int32)
        return cls(rp_packed.contiguous(), col_local.contiguous(), voff, eoff_t.cpu().numpy().astype(np.int64))


def pack_csr(graphs) -> Batch:
    """Packs device CSRs [(row_ptr, col), ...] (local ids kept) into a Batch."""
    import numpy as np
    sizes = [int(rp.numel()) - 1 for rp, _ in graphs]
    nnzs = [int(c.numel()) for _, c in graphs]
    voff = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    eoff = np.concatenate([[0], np.cumsum(nnzs)]).astype(np.int64)
    dev = graphs[0][0].device if graphs else torch.device("cuda", torch.cuda.current_device())
    row_ptr = torch.cat([rp.to(torch.int32) for rp, _ in graphs]) if graphs else torch.zeros(0, dtype=torch.int32,
                                                                                               device=dev)
    col = torch.cat([c.to(torch.int32) for _, c in graphs]) if graphs else torch.zeros(0, dtype=torch.int32,
                                                                                       device=dev)
    return Batch(row_ptr.contiguous(), col.contiguous(), voff, eoff)


def _offsets(batch: Batch):
    import numpy as np
    voff = np.ascontiguousarray(batch.vtx_off, dtype=np.int64)
    eoff = np.ascontiguousarray(batch.edge_off, dtype=np.int64)
    if voff.shape != eoff.shape or voff.ndim != 1 or len(voff) < 1:
        raise ValueError("vtx_off and edge_off: int64 arrays of graphs + 1 entries")
    return voff, eoff


def batch_workspace_bytes(batch: Batch, options: Options | None = None) -> int:
    voff, eoff = _offsets(batch)
    opt = (options or Options()).to_c()
    need = ctypes.c_size_t()
    _check(_capi.load().tc_count_batched_ws(len(voff) - 1, voff.ctypes.data_as(ctypes.c_void_p),
                                            eoff.ctypes.data_as(ctypes.c_void_p), ctypes.byref(opt),
                                            ctypes.byref(need)), "tc_count_batched_ws")
    return need.value


def count_batched(batch: Batch, levels: torch.Tensor | None = None, options: Options | None = None, stream=None,
                  ws: torch.Tensor | None = None):
    """Per-graph triangle counts of a packed batch (tc_count_batched).
    Returns (counts: int64 tensor viewing the uint64 counts, CountResult of
    the whole batch)."""
    _require_i32_cuda(batch.row_ptr, "row_ptr")
    _require_i32_cuda(batch.col, "col")
    if levels is not None:
        _require_i32_cuda(levels, "levels")
    voff, eoff = _offsets(batch)
    graphs = len(voff) - 1
    lib = _capi.load()
    opt = (options or Options()).to_c()
    need = batch_workspace_bytes(batch, options)
    if ws is None or ws.numel() < need:
        ws = workspace(need, batch.row_ptr.device)
    counts = torch.empty(max(graphs, 1), dtype=torch.int64, device=batch.row_ptr.device)
    st = _capi.tc_stats()
    T = lib.tc_count_batched(graphs, voff.ctypes.data_as(ctypes.c_void_p), eoff.ctypes.data_as(ctypes.c_void_p),
                             _ptr(batch.row_ptr), _ptr(batch.col), _ptr(levels), ctypes.byref(opt), _ptr(counts),
                             ctypes.byref(st), _ptr(ws), need, _stream(stream))
    if T == TC_COUNT_ERROR:
        raise TCError(lib.tc_last_error(), "tc_count_batched")
    return counts[:graphs], _result(T, st)


def bfs_levels_batched(batch: Batch, stream=None):
    """BFS levels of every graph of the batch, packed like its vertices
    (tc_bfs_levels_batched); returns (levels, largest level count)."""
    _require_i32_cuda(batch.row_ptr, "row_ptr")
    _require_i32_cuda(batch.col, "col")
    voff, eoff = _offsets(batch)
    need = batch_workspace_bytes(batch)
    ws = workspace(need, batch.row_ptr.device)
    lev = torch.empty(max(int(voff[-1]), 1), dtype=torch.int32, device=batch.row_ptr.device)
    nl = ctypes.c_int32()
    _check(_capi.load().tc_bfs_levels_batched(len(voff) - 1, voff.ctypes.data_as(ctypes.c_void_p),
                                              eoff.ctypes.data_as(ctypes.c_void_p), _ptr(batch.row_ptr),
                                              _ptr(batch.col), _ptr(lev), ctypes.byref(nl), _ptr(ws), need,
                                              _stream(stream)), "tc_bfs_levels_batched")
    return lev[:int(voff[-1])], nl.value


class BatchPlan:
    """The batch's whole pipeline captured once into a HIP graph
    (tc_batch_plan_create) and replayed by :meth:`launch`
    (tc_batch_plan_launch).  Holds the workspace and the counts buffer."""

    def __init__(self, batch: Batch, options: Options | None = None, stream=None):
        _require_i32_cuda(batch.row_ptr, "row_ptr")
        _require_i32_cuda(batch.col, "col")
        self.batch = batch
        voff, eoff = _offsets(batch)
        self.graphs = len(voff) - 1
        self._opt = (options or Options()).to_c()
        need = batch_workspace_bytes(batch, options)
        self.ws = workspace(need, batch.row_ptr.device)
        self.counts = torch.zeros(max(self.graphs, 1), dtype=torch.int64, device=batch.row_ptr.device)
        self._plan = ctypes.c_void_p()
        lib = _capi.load()
        _check(lib.tc_batch_plan_create(self.graphs, voff.ctypes.data_as(ctypes.c_void_p),
                                        eoff.ctypes.data_as(ctypes.c_void_p), _ptr(batch.row_ptr), _ptr(batch.col),
                                        ctypes.byref(self._opt), _ptr(self.counts), _ptr(self.ws), need,
                                        _stream(stream), ctypes.byref(self._plan)), "tc_batch_plan_create")

    def launch(self, stream=None):
        """Replays the pipeline on ``stream`` (asynchronous); the counts are
        in ``self.counts[:graphs]`` once the stream reaches this point."""
        _check(_capi.load().tc_batch_plan_launch(self._plan, _stream(stream)), "tc_batch_plan_launch")
        return self.counts[:self.graphs]

    def close(self):
        if self._plan:
            _check(_capi.load().tc_batch_plan_destroy(self._plan), "tc_batch_plan_destroy")
            self._plan = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def vertex_triangles(row_ptr: torch.Tensor, col: torch.Tensor, levels: torch.Tensor | None = None,
                     options: Options | None = None, stream=None):
    """Triangles through every vertex (tc_vertex_triangles).  Returns
    (tv: int64 tensor of n entries viewing the uint64 counts, CountResult)."""
    _require_i32_cuda(row_ptr, "row_ptr")
    _require_i32_cuda(col, "col")
    if levels is not None:
        _require_i32_cuda(levels, "levels")
    n, nnz = row_ptr.numel() - 1, col.numel()
    lib = _capi.load()
    opt = (options or Options()).to_c()
    need = ctypes.c_size_t()
    _check(lib.tc_count_ws(n, nnz, ctypes.byref(opt), ctypes.byref(need)), "tc_count_ws")
    ws = workspace(need.value, row_ptr.device)
    tv = torch.empty(max(n, 1), dtype=torch.int64, device=row_ptr.device)
    st = _capi.tc_stats()
    T = lib.tc_vertex_triangles(n, nnz, _ptr(row_ptr), _ptr(col), _ptr(levels), ctypes.byref(opt), _ptr(tv),
                                ctypes.byref(st), _ptr(ws), need.value, _stream(stream))
    if T == TC_COUNT_ERROR:
        raise TCError(lib.tc_last_error(), "tc_vertex_triangles")
    return tv[:n], _result(T, st)


def edge_support(row_ptr: torch.Tensor, col: torch.Tensor, levels: torch.Tensor | None = None,
                 options: Options | None = None, stream=None):
    """Triangles through every edge, per input entry (tc_edge_support).
    Returns (sup: int32 tensor of nnz entries viewing the uint32 supports,
    CountResult)."""
    _require_i32_cuda(row_ptr, "row_ptr")
    _require_i32_cuda(col, "col")
    if levels is not None:
        _require_i32_cuda(levels, "levels")
    n, nnz = row_ptr.numel() - 1, col.numel()
    lib = _capi.load()
    opt = (options or Options()).to_c()
    need = ctypes.c_size_t()
    _check(lib.tc_edge_support_ws(n, nnz, ctypes.byref(opt), ctypes.byref(need)), "tc_edge_support_ws")
    ws = workspace(need.value, row_ptr.device)
    sup = torch.empty(max(nnz, 1), dtype=torch.int32, device=row_ptr.device)
    st = _capi.tc_stats()
    T = lib.tc_edge_support(n, nnz, _ptr(row_ptr), _ptr(col), _ptr(levels), ctypes.byref(opt), _ptr(sup),
                            ctypes.byref(st), _ptr(ws), need.value, _stream(stream))
    if T == TC_COUNT_ERROR:
        raise TCError(lib.tc_last_error(), "tc_edge_support")
    return sup[:nnz], _result(T, st)


def relabel_by_degree(row_ptr: torch.Tensor, col: torch.Tensor, stream=None):
    """Degree relabel (tc_relabel_degree).  Returns (row_ptr', col', perm)
    with perm[new id] = old id; new ids follow decreasing degree, ties by
    increasing old id."""
    _require_i32_cuda(row_ptr, "row_ptr")
    _require_i32_cuda(col, "col")
    n, nnz = row_ptr.numel() - 1, col.numel()
    lib = _capi.load()
    need = ctypes.c_size_t()
    _check(lib.tc_relabel_degree_ws(n, nnz, ctypes.byref(need)), "tc_relabel_degree_ws")
    ws = workspace(need.value, row_ptr.device)
    rp2 = torch.empty(n + 1, dtype=torch.int32, device=row_ptr.device)
    col2 = torch.empty(max(nnz, 1), dtype=torch.int32, device=row_ptr.device)
    perm = torch.empty(max(n, 1), dtype=torch.int32, device=row_ptr.device)
    _check(lib.tc_relabel_degree(n, nnz, _ptr(row_ptr), _ptr(col), _ptr(rp2), _ptr(col2), _ptr(perm), _ptr(ws),
                                 need.value, _stream(stream)), "tc_relabel_degree")
    return rp2, col2[:nnz], perm[:n]


def count_cover_edge(row_ptr: torch.Tensor, col: torch.Tensor, levels: torch.Tensor | None = None,
                     options: Options | None = None, stream=None) -> CountResult:
    """Cover-edge count (Algorithm 3) on the same kernels over full rows
    (tc_count_cover_edge); T0 is 0 and T1 = T in the result."""
    _require_i32_cuda(row_ptr, "row_ptr")
    _require_i32_cuda(col, "col")
    if levels is not None:
        _require_i32_cuda(levels, "levels")
    n, nnz = row_ptr.numel() - 1, col.numel()
    lib = _capi.load()
    opt = (options or Options()).to_c()
    need = ctypes.c_size_t()
    _check(lib.tc_count_ws(n, nnz, ctypes.byref(opt), ctypes.byref(need)), "tc_count_ws")
    ws = workspace(need.value, row_ptr.device)
    st = _capi.tc_stats()
    T = lib.tc_count_cover_edge(n, nnz, _ptr(row_ptr), _ptr(col), _ptr(levels), ctypes.byref(opt),
                                ctypes.byref(st), _ptr(ws), need.value, _stream(stream))
    if T == TC_COUNT_ERROR:
        raise TCError(lib.tc_last_error(), "tc_count_cover_edge")
    return _result(T, st)


def count(row_ptr: torch.Tensor, col: torch.Tensor, levels: torch.Tensor | None = None,
          options: Options | None = None, stream=None) -> CountResult:
    """Triangle count T = T0 + T1 with statistics."""
    _require_i32_cuda(row_ptr, "row_ptr")
    _require_i32_cuda(col, "col")
    if levels is not None:
        _require_i32_cuda(levels, "levels")
    c = Counter(row_ptr.numel() - 1, col.numel(), options, row_ptr.device)
    return c(row_ptr, col, levels, stream)
