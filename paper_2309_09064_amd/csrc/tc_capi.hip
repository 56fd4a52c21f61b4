// C ABI of libtc: argument checks on the host before any device work,
// workspace carving, optional device-side input validation, error codes.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "tc_internal.hpp"

namespace tc {

namespace {
thread_local int g_last_error = TC_OK;
constexpr int kMaxDevices = 64;
DeviceInfo g_dev[kMaxDevices];
}  // namespace

void set_error(int code) { g_last_error = code; }
int last_error() { return g_last_error; }

void note_hip_error(hipError_t e, const char *what, const char *file, int line) {
    if (getenv("TC_LOG")) fprintf(stderr, "libtc: %s failed: %s (%s:%d)\n", what, hipGetErrorString(e), file, line);
}

int device_info(DeviceInfo *out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return TC_ERR_NO_DEVICE;
    if (dev < 0 || dev >= kMaxDevices) return TC_ERR_NO_DEVICE;
    DeviceInfo &d = g_dev[dev];
    if (!d.ok) {
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, dev) != hipSuccess) return TC_ERR_NO_DEVICE;
        if (strncmp(p.gcnArchName, "gfx950", 6) != 0) return TC_ERR_NO_DEVICE;
        d.cus = p.multiProcessorCount > 0 ? p.multiProcessorCount : 256;
        d.ok = 1;
    }
    *out = d;
    return TC_OK;
}

namespace {
thread_local Mailbox t_mail;

__global__ void k_mail_u64(const uint64_t *src, uint64_t *dst, int count) {
    if ((int)threadIdx.x < count) dst[threadIdx.x] = src[threadIdx.x];
}
__global__ void k_mail_i32(const int32_t *src, uint64_t *dst) {
    if (threadIdx.x == 0) dst[0] = (uint64_t)(int64_t)src[0];
}
}  // namespace

int mailbox_release() {
    if (!t_mail.host) return TC_OK;
    const hipError_t e = hipHostFree(t_mail.host);
    t_mail = Mailbox{};
    return e == hipSuccess ? TC_OK : TC_ERR_HIP;
}

int mailbox(Mailbox *out) {
    if (!t_mail.host) {
        void *h = nullptr;
        if (hipHostMalloc(&h, 4096, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) return TC_ERR_HIP;
        void *d = nullptr;
        if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess) return TC_ERR_HIP;
        t_mail.host = static_cast<uint64_t *>(h);
        t_mail.dev = static_cast<uint64_t *>(d);
    }
    *out = t_mail;
    return TC_OK;
}

int mail_u64(const uint64_t *src, uint64_t *dst, int count, hipStream_t s) {
    hipLaunchKernelGGL(k_mail_u64, dim3(1), dim3(64), 0, s, src, dst, count);
    TC_HIP_TRY(hipGetLastError());
    return TC_OK;
}

int mail_i32(const int32_t *src, uint64_t *dst, hipStream_t s) {
    hipLaunchKernelGGL(k_mail_i32, dim3(1), dim3(64), 0, s, src, dst);
    TC_HIP_TRY(hipGetLastError());
    return TC_OK;
}

// ---------------------------------------------------------------- validation

namespace {

// bit 0: row_ptr not monotone / wrong ends; bit 1: column out of range;
// bit 2: row not strictly ascending (duplicate or unsorted); bit 3: self-loop;
// bit 4: missing reverse entry; bit 5: levels differ by more than one.
__global__ void k_validate(int32_t n, int64_t nnz, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                           const int32_t *__restrict__ lev, int32_t *__restrict__ bad) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += stride) {
        int32_t b = rp[x], e = rp[x + 1];
        if (e < b || b < 0 || (int64_t)e > nnz || (x == 0 && b != 0) || (x == n - 1 && (int64_t)e != nnz)) {
            atomicOr(bad, 1);
            continue;
        }
        for (int32_t j = b; j < e; ++j) {
            int32_t y = col[j];
            if (y < 0 || y >= n) { atomicOr(bad, 2); continue; }
            if (j > b && col[j - 1] >= y) atomicOr(bad, 4);
            if (y == x) atomicOr(bad, 8);
            int32_t lo = rp[y], hi = rp[y + 1];
            bool found = false;
            if (lo >= 0 && hi <= nnz && lo <= hi) {
                while (lo < hi) {
                    int32_t mid = (lo + hi) >> 1;
                    if (col[mid] < (int32_t)x) lo = mid + 1; else hi = mid;
                }
                found = lo < rp[y + 1] && col[lo] == (int32_t)x;
            }
            if (!found) atomicOr(bad, 16);
            if (lev) {
                int32_t d = lev[x] - lev[y];
                if (d > 1 || d < -1) atomicOr(bad, 32);
            }
        }
    }
}

}  // namespace

int validate_device(int32_t n, int64_t nnz, const int32_t *rp, const int32_t *col, const int32_t *lev,
                    int32_t *scratch, hipStream_t s) {
    TC_HIP_TRY(hipMemsetAsync(scratch, 0, sizeof(int32_t), s));
    if (n > 0) {
        int64_t g = ((int64_t)n + 255) / 256;
        if (g > 16384) g = 16384;
        hipLaunchKernelGGL(k_validate, dim3((unsigned)g), dim3(256), 0, s, n, nnz, rp, col, lev, scratch);
        TC_HIP_TRY(hipGetLastError());
    }
    int32_t bad = 0;
    TC_HIP_TRY(hipMemcpyAsync(&bad, scratch, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    TC_HIP_TRY(hipStreamSynchronize(s));
    if (n == 0 && nnz != 0) bad |= 1;
    return bad ? TC_ERR_INVALID_CSR : TC_OK;
}

namespace {

// ---------------------------------------------------------------- options

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

int make_cfg(const tc_options *opt, CountCfg *cfg, int *flags) {
    CountCfg c;
    *flags = 0;
    if (opt) {
        if (opt->schedule != TC_SCHED_HEURISTIC && opt->schedule != TC_SCHED_TABLE) return TC_ERR_ARG;
        if (opt->force_strategy < TC_STRAT_AUTO || opt->force_strategy >= TC_NUM_STRATEGIES) return TC_ERR_ARG;
        if (opt->wave_slots && (!is_pow2(opt->wave_slots) || opt->wave_slots < 64 || opt->wave_slots > 2048))
            return TC_ERR_ARG;
        if (opt->wg_slots && (!is_pow2(opt->wg_slots) || opt->wg_slots < 1024 || opt->wg_slots > 32768))
            return TC_ERR_ARG;
        if (opt->chunk_work < 0 || opt->grid_blocks < 0 || opt->wave_max_owner < 0) return TC_ERR_ARG;
        c.schedule = opt->schedule;
        c.table = opt->schedule == TC_SCHED_TABLE ? opt->sched_table : nullptr;
        c.force = opt->force_strategy;
        if (opt->wave_slots) c.wave_slots = opt->wave_slots;
        if (opt->wg_slots) c.wg_slots = opt->wg_slots;
        if (opt->chunk_work) c.chunk_work = opt->chunk_work;
        c.grid_blocks = opt->grid_blocks;
        c.wave_max_owner = opt->wave_max_owner;
        if (opt->merge_max_owner < -1 || opt->merge_max_owner > 31) return TC_ERR_ARG;
        c.merge_max_owner = opt->merge_max_owner;
        if (opt->wg_slice_max && (!is_pow2(opt->wg_slice_max) || opt->wg_slice_max < 64 ||
                                  opt->wg_slice_max > c.wg_slots / 2))
            return TC_ERR_ARG;
        c.wg_slice_max = opt->wg_slice_max;
        if (opt->orientation != TC_ORIENT_RANK && opt->orientation != TC_ORIENT_ID) return TC_ERR_ARG;
        c.orientation = opt->orientation;
        if (opt->flags & ~(TC_VALIDATE | TC_TIMING)) return TC_ERR_ARG;
        *flags = opt->flags;
    }
    // the sixteen wavefront tables of a block share the workgroup's LDS
    if (c.wave_slots * 16 > 32768) return TC_ERR_ARG;
    c.timing = (*flags & TC_TIMING) != 0;
    *cfg = c;
    return TC_OK;
}

int check_graph_args(int32_t n, int64_t nnz, const void *rp, const void *col) {
    if (n < 0 || nnz < 0) return TC_ERR_ARG;
    if (nnz >= (int64_t(1) << 31)) return TC_ERR_OVERFLOW;
    if (n > 0 && !rp) return TC_ERR_ARG;
    if (nnz > 0 && !col) return TC_ERR_ARG;
    if (n == 0 && nnz > 0) return TC_ERR_ARG;
    return TC_OK;
}

int check_ws(void *ws, size_t ws_bytes, size_t need) { return check_workspace(ws, ws_bytes, need); }

int fail(int code) {
    set_error(code);
    return code;
}

}  // namespace

int check_workspace(void *ws, size_t ws_bytes, size_t need) {
    if (need > ws_bytes) return TC_ERR_WORKSPACE;
    if (need > 0 && !ws) return TC_ERR_WORKSPACE;
    if (((uintptr_t)ws & 255) != 0) return TC_ERR_WORKSPACE;
    return TC_OK;
}

CountPlanBufs carve_count_plan(Carver &c, int32_t n, int64_t nnz, bool own_levels, bool edge_pos) {
    CountPlanBufs P;
    const int64_t nn = n > 0 ? n : 1;
    const int64_t nz = nnz > 0 ? nnz : 1;
    P.levels = own_levels ? c.take<int32_t>(nn) : nullptr;
    // the list arrays get kListPad ints of padding on both sides: the
    // intersection kernel reads whole 8-element runs that may straddle a
    // list's ends (never used, always inside the allocation)
    P.pb.rp0 = c.take<int32_t>(nn + 1);
    P.pb.c0 = c.take<int32_t>(nz + 2 * kListPad) + (c.base ? kListPad : 0);
    P.pb.up0 = c.take<int32_t>(nn);
    P.pb.rp1 = c.take<int32_t>(nn + 1);
    P.pb.c1 = c.take<int32_t>(nz + 2 * kListPad) + (c.base ? kListPad : 0);
    P.pb.d0 = c.take<int32_t>(nn);
    P.pb.rpu = c.take<int32_t>(nn + 1);
    P.pb.e0x2 = c.take<int64_t>(1);
    P.pb.vrec = c.take<int4>(nn);
    if (edge_pos) {   // per-edge support: input entry of every c0 / c1 entry
        P.pb.pos0 = c.take<int32_t>(nz);
        P.pb.pos1 = c.take<int32_t>(nz);
    }
    P.flag = c.take<int32_t>(64);
    size_t sb = bfs_ws_bytes(n, nnz);
    size_t t = partition_ws_bytes(n, nnz);
    if (t > sb) sb = t;
    t = count_ws_bytes(n, nnz);
    if (t > sb) sb = t;
    P.scratch = c.take<char>(sb);
    P.scratch_bytes = sb;
    return P;
}

int options_cfg(const tc_options *opt, CountCfg *cfg, int *flags) { return make_cfg(opt, cfg, flags); }

}  // namespace tc

using namespace tc;

extern "C" {

int tc_last_error(void) { return tc::last_error(); }

const char *tc_strerror(int code) {
    switch (code) {
    case TC_OK: return "ok";
    case TC_ERR_ARG: return "invalid argument";
    case TC_ERR_RANGE: return "vertex id out of range";
    case TC_ERR_OVERFLOW: return "size does not fit int32 CSR";
    case TC_ERR_CAPACITY: return "output buffer too small";
    case TC_ERR_WORKSPACE: return "workspace missing, too small or misaligned";
    case TC_ERR_HIP: return "HIP runtime error";
    case TC_ERR_NO_DEVICE: return "no gfx950 device";
    case TC_ERR_INVALID_CSR: return "malformed CSR or levels";
    case TC_ERR_TOO_LARGE: return "graph exceeds the fixed scratch of the no-allocation count";
    default: return "unknown error";
    }
}

int tc_version(void) { return 10100; }

int tc_thread_release(void) { return fail(mailbox_release()); }

int tc_build_csr_ws(int32_t n, int64_t m_tuples, size_t *h_ws_bytes) {
    if (!h_ws_bytes || n < 0 || m_tuples < 0) return fail(TC_ERR_ARG);
    if (2 * m_tuples >= (int64_t(1) << 31)) return fail(TC_ERR_OVERFLOW);
    *h_ws_bytes = build_csr_ws_bytes(n, m_tuples);
    return fail(TC_OK);
}

int tc_build_csr(int32_t n, int64_t m_tuples, const int32_t *d_src, const int32_t *d_dst, int32_t *d_row_ptr,
                 int32_t *d_col_idx, int64_t col_cap, int64_t *h_nnz, void *ws, size_t ws_bytes, void *stream) {
    if (n < 0 || m_tuples < 0 || col_cap < 0 || !d_row_ptr || !h_nnz) return fail(TC_ERR_ARG);
    if (m_tuples > 0 && (!d_src || !d_dst)) return fail(TC_ERR_ARG);
    if (col_cap > 0 && !d_col_idx) return fail(TC_ERR_ARG);
    if (2 * m_tuples >= (int64_t(1) << 31)) return fail(TC_ERR_OVERFLOW);
    int rc = check_ws(ws, ws_bytes, build_csr_ws_bytes(n, m_tuples));
    if (rc != TC_OK) return fail(rc);
    DeviceInfo di;
    rc = device_info(&di);
    if (rc != TC_OK) return fail(rc);
    rc = build_csr_run(n, m_tuples, d_src, d_dst, d_row_ptr, d_col_idx, col_cap, h_nnz, ws, ws_bytes,
                       static_cast<hipStream_t>(stream));
    return fail(rc);
}

int tc_bfs_levels_ws(int32_t n, int64_t nnz, size_t *h_ws_bytes) {
    if (!h_ws_bytes) return fail(TC_ERR_ARG);
    int rc = check_graph_args(n, nnz, (const void *)1, (const void *)1);
    if (rc != TC_OK) return fail(rc);
    *h_ws_bytes = bfs_ws_bytes(n, nnz);
    return fail(TC_OK);
}

int tc_bfs_levels(int32_t n, int64_t nnz, const int32_t *d_row_ptr, const int32_t *d_col_idx, int32_t *d_levels,
                  int32_t *h_levels_count, void *ws, size_t ws_bytes, void *stream) {
    int rc = check_graph_args(n, nnz, d_row_ptr, d_col_idx);
    if (rc != TC_OK) return fail(rc);
    if (n > 0 && !d_levels) return fail(TC_ERR_ARG);
    rc = check_ws(ws, ws_bytes, bfs_ws_bytes(n, nnz));
    if (rc != TC_OK) return fail(rc);
    DeviceInfo di;
    rc = device_info(&di);
    if (rc != TC_OK) return fail(rc);
    BfsOut bo;
    rc = bfs_run(n, nnz, d_row_ptr, d_col_idx, d_levels, &bo, ws, ws_bytes, static_cast<hipStream_t>(stream));
    if (rc == TC_OK) {
        hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
        if (e != hipSuccess) rc = TC_ERR_HIP;
    }
    if (rc == TC_OK && h_levels_count) *h_levels_count = bo.levels;
    return fail(rc);
}

int tc_partition_ws(int32_t n, int64_t nnz, size_t *h_ws_bytes) {
    if (!h_ws_bytes) return fail(TC_ERR_ARG);
    int rc = check_graph_args(n, nnz, (const void *)1, (const void *)1);
    if (rc != TC_OK) return fail(rc);
    Carver c(nullptr, 0);
    const int64_t nn = n > 0 ? n : 1;
    c.take<int32_t>(nn);          // d0
    c.take<int32_t>(nn + 1);      // rpu
    c.take<int64_t>(1);           // 2|E0|
    c.take<char>(partition_ws_bytes(n, nnz));
    *h_ws_bytes = c.used();
    return fail(TC_OK);
}

int tc_partition(int32_t n, int64_t nnz, const int32_t *d_row_ptr, const int32_t *d_col_idx, const int32_t *d_levels,
                 int32_t orientation, int32_t *d_rp0, int32_t *d_c0, int32_t *d_up0, int32_t *d_rp1, int32_t *d_c1,
                 int64_t *h_e0, void *ws, size_t ws_bytes, void *stream) {
    int rc = check_graph_args(n, nnz, d_row_ptr, d_col_idx);
    if (rc != TC_OK) return fail(rc);
    if (orientation != TC_ORIENT_RANK && orientation != TC_ORIENT_ID) return fail(TC_ERR_ARG);
    if (!d_rp0 || !d_rp1 || !h_e0 || (n > 0 && (!d_levels || !d_up0)) || (nnz > 0 && (!d_c0 || !d_c1)))
        return fail(TC_ERR_ARG);
    size_t need = 0;
    tc_partition_ws(n, nnz, &need);
    rc = check_ws(ws, ws_bytes, need);
    if (rc != TC_OK) return fail(rc);
    DeviceInfo di;
    rc = device_info(&di);
    if (rc != TC_OK) return fail(rc);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (n == 0) {   // empty graph: both row-pointer arrays are {0}
        if (hipMemsetAsync(d_rp0, 0, sizeof(int32_t), s) != hipSuccess ||
            hipMemsetAsync(d_rp1, 0, sizeof(int32_t), s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
            return fail(TC_ERR_HIP);
        *h_e0 = 0;
        return fail(TC_OK);
    }
    Carver c(ws, ws_bytes);
    const int64_t nn = n > 0 ? n : 1;
    PartBufs pb;
    pb.rp0 = d_rp0;
    pb.c0 = d_c0;
    pb.up0 = d_up0;
    pb.rp1 = d_rp1;
    pb.c1 = d_c1;
    pb.d0 = c.take<int32_t>(nn);
    pb.rpu = c.take<int32_t>(nn + 1);
    pb.e0x2 = c.take<int64_t>(1);
    pb.by_id = orientation == TC_ORIENT_ID ? 1 : 0;
    void *scratch = c.take<char>(partition_ws_bytes(n, nnz));
    rc = partition_run(n, nnz, d_row_ptr, d_col_idx, d_levels, pb, scratch, partition_ws_bytes(n, nnz), s);
    if (rc != TC_OK) return fail(rc);
    int64_t e0x2 = 0;
    if (hipMemcpyAsync(&e0x2, pb.e0x2, sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(TC_ERR_HIP);
    *h_e0 = e0x2 / 2;
    return fail(TC_OK);
}

int tc_count_ws(int32_t n, int64_t nnz, const tc_options *opt, size_t *h_ws_bytes) {
    if (!h_ws_bytes) return fail(TC_ERR_ARG);
    int rc = check_graph_args(n, nnz, (const void *)1, (const void *)1);
    if (rc != TC_OK) return fail(rc);
    CountCfg cfg;
    int flags;
    rc = make_cfg(opt, &cfg, &flags);
    if (rc != TC_OK) return fail(rc);
    Carver c(nullptr, 0);
    carve_count_plan(c, n, nnz, true, false);
    *h_ws_bytes = c.used();
    return fail(TC_OK);
}

static uint64_t count_impl(int32_t n, int64_t nnz, const int32_t *d_row_ptr, const int32_t *d_col_idx,
                    const int32_t *d_levels, const tc_options *opt, tc_stats *stats, uint64_t *d_prof, void *ws,
                    size_t ws_bytes, void *stream,
                    uint64_t *d_tv = nullptr, bool edge = false, uint32_t *d_sup = nullptr, bool cover = false) {
    int rc = check_graph_args(n, nnz, d_row_ptr, d_col_idx);
    if (rc != TC_OK) { fail(rc); return TC_COUNT_ERROR; }
    CountCfg cfg;
    int flags;
    rc = make_cfg(opt, &cfg, &flags);
    if (rc != TC_OK) { fail(rc); return TC_COUNT_ERROR; }
    if (cfg.schedule == TC_SCHED_TABLE && !cfg.table) { fail(TC_ERR_ARG); return TC_COUNT_ERROR; }
    cfg.prof = reinterpret_cast<unsigned long long *>(d_prof);
    cfg.tv = reinterpret_cast<unsigned long long *>(d_tv);
    if (edge || d_tv) {
        // the hit counters beside every hash table halve the LDS per table
        if (cfg.wg_slots > kCountedMaxWgSlots) cfg.wg_slots = kCountedMaxWgSlots;
        if (cfg.wave_slots > kCountedMaxWaveSlots) cfg.wave_slots = kCountedMaxWaveSlots;
    }
    if (edge) {
        cfg.sup = nnz > 0 ? d_sup : nullptr;   // no entries: nothing to count or write
        cfg.rp = d_row_ptr;
        cfg.col = d_col_idx;
    }
    size_t need = 0;
    {
        Carver c(nullptr, 0);
        carve_count_plan(c, n, nnz, true, edge);
        need = c.used();
    }
    rc = check_ws(ws, ws_bytes, need);
    if (rc != TC_OK) { fail(rc); return TC_COUNT_ERROR; }
    DeviceInfo di;
    rc = device_info(&di);
    if (rc != TC_OK) { fail(rc); return TC_COUNT_ERROR; }
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (n == 0) {   // no vertices, no triangles
        if (stats) memset(stats, 0, sizeof(*stats));
        fail(TC_OK);
        return 0;
    }
    Carver c(ws, ws_bytes);
    CountPlanBufs P = carve_count_plan(c, n, nnz, true, edge);
    if (flags & TC_VALIDATE) {
        rc = validate_device(n, nnz, d_row_ptr, d_col_idx, d_levels, P.flag, s);
        if (rc != TC_OK) { fail(rc); return TC_COUNT_ERROR; }
    }
    const bool timing = (flags & TC_TIMING) != 0;
    EventSet ev;   // destroyed on every return
    auto fail_ev = [&](int code) {
        fail(code);
        return TC_COUNT_ERROR;
    };
    if (timing) {
        if (ev.create(3) != TC_OK || hipEventRecord(ev.e[0], s) != hipSuccess) return fail_ev(TC_ERR_HIP);
    }
    BfsOut bo;
    const int32_t *lev = d_levels;
    if (!lev) {
        rc = bfs_run(n, nnz, d_row_ptr, d_col_idx, P.levels, &bo, P.scratch, P.scratch_bytes, s);
        if (rc != TC_OK) return fail_ev(rc);
        lev = P.levels;
    }
    if (timing && hipEventRecord(ev.e[1], s) != hipSuccess) return fail_ev(TC_ERR_HIP);
    P.pb.by_id = cfg.orientation == TC_ORIENT_ID ? 1 : 0;
    rc = partition_run(n, nnz, d_row_ptr, d_col_idx, lev, P.pb, P.scratch, P.scratch_bytes, s);
    if (rc != TC_OK) return fail_ev(rc);
    PartBufs pb = P.pb;
    if (cover) {   // Algorithm 3 runs on full rows; the partition only supplies the horizontal edges
        rc = cover_view_run(n, d_row_ptr, d_col_idx, &pb, s);
        if (rc != TC_OK) return fail_ev(rc);
        cfg.cover_lev = lev;
    }
    if (timing && hipEventRecord(ev.e[2], s) != hipSuccess) return fail_ev(TC_ERR_HIP);
    CountOut co;
    rc = count_run(n, nnz, pb, cfg, &co, P.scratch, P.scratch_bytes, s);
    if (rc != TC_OK) return fail_ev(rc);
    if (stats) {
        memset(stats, 0, sizeof(*stats));
        stats->T0 = co.T0;
        stats->T1 = co.T1;
        stats->e0 = co.e0x2 / 2;
        stats->units = co.units;
        stats->items = co.items;
        stats->probes = co.probes;
        stats->hashed = co.hashed;
        stats->levels = bo.levels;
        stats->bfs_rounds = bo.rounds;
        for (int k = 0; k < TC_NUM_STRATEGIES; ++k) stats->strategy_items[k] = co.strategy_items[k];
        if (timing) {
            (void)hipEventElapsedTime(&stats->ms_bfs, ev.e[0], ev.e[1]);
            (void)hipEventElapsedTime(&stats->ms_partition, ev.e[1], ev.e[2]);
            stats->ms_bucket = co.ms_bucket;
            stats->ms_isect = co.ms_isect;
        }
    }
    fail(TC_OK);
    return co.T0 + co.T1;
}

uint64_t tc_count(int32_t n, int64_t nnz, const int32_t *d_row_ptr, const int32_t *d_col_idx, const int32_t *d_levels,
                  const tc_options *opt, tc_stats *stats, void *ws, size_t ws_bytes, void *stream) {
    return count_impl(n, nnz, d_row_ptr, d_col_idx, d_levels, opt, stats, nullptr, ws, ws_bytes, stream);
}

int tc_schedule_table(int32_t n, int64_t nnz, const tc_options *opt, int32_t *d_table, void *stream) {
    int rc = check_graph_args(n, nnz, (const void *)1, (const void *)1);
    if (rc != TC_OK) return fail(rc);
    if (!d_table) return fail(TC_ERR_ARG);
    CountCfg cfg;
    int flags;
    rc = make_cfg(opt, &cfg, &flags);
    if (rc != TC_OK) return fail(rc);
    if (cfg.schedule == TC_SCHED_TABLE && !cfg.table) return fail(TC_ERR_ARG);
    DeviceInfo di;
    rc = device_info(&di);
    if (rc != TC_OK) return fail(rc);
    return fail(schedule_table_run(n, nnz, cfg, d_table, static_cast<hipStream_t>(stream)));
}

uint64_t tc_vertex_triangles(int32_t n, int64_t nnz, const int32_t *d_row_ptr, const int32_t *d_col_idx,
                             const int32_t *d_levels, const tc_options *opt, uint64_t *d_tv, tc_stats *stats,
                             void *ws, size_t ws_bytes, void *stream) {
    if (!d_tv && n > 0) { fail(TC_ERR_ARG); return TC_COUNT_ERROR; }
    return count_impl(n, nnz, d_row_ptr, d_col_idx, d_levels, opt, stats, nullptr, ws, ws_bytes, stream, d_tv);
}

int tc_edge_support_ws(int32_t n, int64_t nnz, const tc_options *opt, size_t *h_ws_bytes) {
    if (!h_ws_bytes) return fail(TC_ERR_ARG);
    int rc = check_graph_args(n, nnz, (const void *)1, (const void *)1);
    if (rc != TC_OK) return fail(rc);
    CountCfg cfg;
    int flags;
    rc = make_cfg(opt, &cfg, &flags);
    if (rc != TC_OK) return fail(rc);
    Carver c(nullptr, 0);
    carve_count_plan(c, n, nnz, true, true);
    *h_ws_bytes = c.used();
    return fail(TC_OK);
}

uint64_t tc_edge_support(int32_t n, int64_t nnz, const int32_t *d_row_ptr, const int32_t *d_col_idx,
                         const int32_t *d_levels, const tc_options *opt, uint32_t *d_sup, tc_stats *stats, void *ws,
                         size_t ws_bytes, void *stream) {
    if (!d_sup && nnz > 0) { fail(TC_ERR_ARG); return TC_COUNT_ERROR; }
    return count_impl(n, nnz, d_row_ptr, d_col_idx, d_levels, opt, stats, nullptr, ws, ws_bytes, stream, nullptr,
                      true, d_sup);
}

uint64_t tc_count_cover_edge(int32_t n, int64_t nnz, const int32_t *d_row_ptr, const int32_t *d_col_idx,
                             const int32_t *d_levels, const tc_options *opt, tc_stats *stats, void *ws,
                             size_t ws_bytes, void *stream) {
    return count_impl(n, nnz, d_row_ptr, d_col_idx, d_levels, opt, stats, nullptr, ws, ws_bytes, stream, nullptr,
                      false, nullptr, true);
}

int tc_relabel_degree_ws(int32_t n, int64_t nnz, size_t *h_ws_bytes) {
    if (!h_ws_bytes) return fail(TC_ERR_ARG);
    int rc = check_graph_args(n, nnz, (const void *)1, (const void *)1);
    if (rc != TC_OK) return fail(rc);
    *h_ws_bytes = relabel_ws_bytes(n, nnz);
    return fail(TC_OK);
}

int tc_relabel_degree(int32_t n, int64_t nnz, const int32_t *d_row_ptr, const int32_t *d_col_idx,
                      int32_t *d_out_row_ptr, int32_t *d_out_col_idx, int32_t *d_perm, void *ws, size_t ws_bytes,
                      void *stream) {
    int rc = check_graph_args(n, nnz, d_row_ptr, d_col_idx);
    if (rc != TC_OK) return fail(rc);
    if (!d_out_row_ptr || (nnz > 0 && !d_out_col_idx) || (n > 0 && !d_perm)) return fail(TC_ERR_ARG);
    rc = check_ws(ws, ws_bytes, relabel_ws_bytes(n, nnz));
    if (rc != TC_OK) return fail(rc);
    DeviceInfo di;
    rc = device_info(&di);
    if (rc != TC_OK) return fail(rc);
    return fail(relabel_run(n, nnz, d_row_ptr, d_col_idx, d_out_row_ptr, d_out_col_idx, d_perm, ws, ws_bytes,
                            static_cast<hipStream_t>(stream)));
}

uint64_t tc_count_profile(int32_t n, int64_t nnz, const int32_t *d_row_ptr, const int32_t *d_col_idx,
                          const int32_t *d_levels, const tc_options *opt, tc_stats *stats, uint64_t *d_prof,
                          void *ws, size_t ws_bytes, void *stream) {
    if (!d_prof) { fail(TC_ERR_ARG); return TC_COUNT_ERROR; }
    return count_impl(n, nnz, d_row_ptr, d_col_idx, d_levels, opt, stats, d_prof, ws, ws_bytes, stream);
}

}  // extern "C"
