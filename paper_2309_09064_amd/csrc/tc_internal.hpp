// Internal declarations shared by the HIP translation units of libtc.
// Everything here is gfx950-only: 64-wide wavefronts, 160 KB LDS per CU.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/tc.h"

namespace tc {

constexpr int kWave = 64;

// ------------------------------------------------------------------ errors

void set_error(int code);
int last_error();

#define TC_HIP_TRY(expr)                                   \
    do {                                                   \
        hipError_t e_ = (expr);                            \
        if (e_ != hipSuccess) {                            \
            ::tc::note_hip_error(e_, #expr, __FILE__, __LINE__); \
            return TC_ERR_HIP;                             \
        }                                                  \
    } while (0)

#define TC_TRY(expr)                  \
    do {                              \
        int rc_ = (expr);             \
        if (rc_ != TC_OK) return rc_; \
    } while (0)

void note_hip_error(hipError_t e, const char *what, const char *file, int line);

// ------------------------------------------------------------------ workspace

// Carves 256-byte aligned pieces out of the caller's workspace.  With a NULL
// base it only measures (used by the *_ws size queries), so the size query
// and the real carving run the same code.
struct Carver {
    char *base;
    size_t cap;
    size_t off = 0;
    Carver(void *b, size_t c) : base(static_cast<char *>(b)), cap(c) {}
    template <class T>
    T *take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
    size_t used() const { return (off + 255) & ~size_t(255); }
    bool fits() const { return used() <= cap; }
};

// HIP events released on every exit path of the function that holds them.
struct EventSet {
    hipEvent_t e[4] = {nullptr, nullptr, nullptr, nullptr};
    int create(int count) {
        for (int i = 0; i < count && i < 4; ++i)
            if (hipEventCreate(&e[i]) != hipSuccess) return TC_ERR_HIP;
        return TC_OK;
    }
    ~EventSet() {
        for (auto &x : e)
            if (x) (void)hipEventDestroy(x);
    }
};

// ------------------------------------------------------------------ device info

struct DeviceInfo {
    int cus = 256;
    int ok = 0;
};
int device_info(DeviceInfo *out);

// ------------------------------------------------------------------ mailbox

// A 4 KB pinned host buffer, mapped into the device address space, private
// to the calling host thread: allocated on the thread's first call, reused
// by every later one, released by tc_thread_release (or at process end).
// Kernels write small results there; the host reads them after
// synchronising the stream, without a device-to-host copy.
struct Mailbox {
    uint64_t *host = nullptr;
    uint64_t *dev = nullptr;
};
int mailbox(Mailbox *out);
int mailbox_release();
// dst[i] = src[i] for i < count (count <= 64), one tiny kernel.
int mail_u64(const uint64_t *src, uint64_t *dst, int count, hipStream_t s);
int mail_i32(const int32_t *src, uint64_t *dst, hipStream_t s);

// ------------------------------------------------------------------ device helpers

__device__ __forceinline__ int lane_id() { return __lane_id(); }

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

template <class T>
__device__ __forceinline__ T wave_incl_scan(T v) {
    const int l = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        T t = __shfl_up(v, d, kWave);
        if (l >= d) v += t;
    }
    return v;
}

// Orders LDS traffic between lanes of one wavefront (no workgroup barrier).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Last r in [lo, hi] with rp[r] <= e (the CSR row that holds entry e).
template <class P>
__device__ __forceinline__ int64_t row_of(const P *rp, int64_t lo, int64_t hi, int64_t e) {
    while (lo < hi) {
        int64_t mid = (lo + hi + 1) >> 1;
        if ((int64_t)rp[mid] <= e) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// The 8 entries [e0, e1) of a thread's run (e1 - e0 <= 8), 0 past e1: two
// 16-byte loads when the run is whole and 16-byte aligned (a wavefront's
// instruction then covers 1 KB instead of 256 bytes), else one load each.
__device__ __forceinline__ void load_run8(const int32_t *__restrict__ a, int64_t e0, int64_t e1, int32_t (&y)[8]) {
    if (e1 - e0 == 8 && ((uintptr_t)(a + e0) & 15) == 0) {
        const int4 lo = *reinterpret_cast<const int4 *>(a + e0), hi = *reinterpret_cast<const int4 *>(a + e0 + 4);
        y[0] = lo.x; y[1] = lo.y; y[2] = lo.z; y[3] = lo.w;
        y[4] = hi.x; y[5] = hi.y; y[6] = hi.z; y[7] = hi.w;
    } else {
#pragma unroll
        for (int k = 0; k < 8; ++k) y[k] = e0 + k < e1 ? a[e0 + k] : 0;
    }
}

// Rows spanned by the tile of CSR entries [t0, t1) (t0 < t1 <= rp[nrows]):
// one thread searches, the block shares the range through `sh` (2 entries).
// Ends with a barrier.  Threads then search only inside [lo, hi].
template <class P>
__device__ __forceinline__ void tile_rows(const P *rp, int64_t nrows, int64_t t0, int64_t t1, int64_t *sh) {
    if (threadIdx.x == 0) {
        const int64_t lo = row_of(rp, 0, nrows - 1, t0);
        sh[0] = lo;
        sh[1] = row_of(rp, lo, nrows - 1, t1 - 1);
    }
    __syncthreads();
}

// ------------------------------------------------------------------ tiles of entries

// Row passes work on tiles of kTileEntries consecutive CSR entries.  The
// tile table holds, per tile, the rows of its first and last entry, so a
// block finds its rows with two loads instead of a binary search over the
// row pointers (at Kronecker scale 24 that search was 24 dependent loads
// into a 67 MB array per tile).  tlo / thi: int32[tiles(total)].
constexpr int kTileEntries = 2048;
__host__ __device__ constexpr int64_t tiles_of(int64_t entries) { return (entries + kTileEntries - 1) / kTileEntries + 1; }
// Fills the table of the rows 0..n-1 of rp (entries 0..rp[n]), on the device.
int tile_table_run(int32_t n, const int32_t *rp, int32_t *tlo, int32_t *thi, hipStream_t s);

// ------------------------------------------------------------------ fill and scan

// p[i] = value for the first `count` 32-bit words: a kernel, so that it may
// be recorded into a captured graph (where memset nodes are avoided).
int fill_u32(void *p, uint32_t value, int64_t count, hipStream_t s);

// Exclusive prefix sum of n values (int32 or int64 input) into int32 or int64
// output of n+1 entries (out[n] = total).  Three-level reduce-then-scan.
size_t scan_ws_bytes(int64_t n);
int scan_exclusive_i32_to_i32(const int32_t *in, int32_t *out, int64_t n, void *ws, hipStream_t s);
int scan_exclusive_i32_to_i64(const int32_t *in, int64_t *out, int64_t n, void *ws, hipStream_t s);
int scan_exclusive_i64_to_i64(const int64_t *in, int64_t *out, int64_t n, void *ws, hipStream_t s);

// ------------------------------------------------------------------ phases

// Stable LSD radix sort of nk 64-bit keys on their low `bits` bits, 8 bits a
// pass, ping-ponging between a and b; *sorted is whichever holds the result.
// Its scratch (radix_sort_ws_bytes(nk)) also serves any scan of up to nk
// values.
size_t radix_sort_ws_bytes(int64_t nk);
int radix_sort_u64(uint64_t *a, uint64_t *b, int64_t nk, int bits, void *ws, size_t ws_bytes, hipStream_t s,
                   uint64_t **sorted);
int bits_for_ids(int64_t n);   // bits for ids 0 .. n-1 (at least 1)

// Degree relabel (decreasing degree, ties by increasing id)
size_t relabel_ws_bytes(int32_t n, int64_t nnz);
int relabel_run(int32_t n, int64_t nnz, const int32_t *rp, const int32_t *col, int32_t *out_rp, int32_t *out_col,
                int32_t *perm, void *ws, size_t ws_bytes, hipStream_t s);

// CSR build
size_t build_csr_ws_bytes(int32_t n, int64_t m);
int build_csr_run(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, int32_t *row_ptr,
                  int32_t *col, int64_t col_cap, int64_t *h_nnz, void *ws, size_t ws_bytes,
                  hipStream_t s);

// BFS levels
struct BfsOut {
    int32_t levels = 0;
    int32_t rounds = 0;
};
size_t bfs_ws_bytes(int32_t n, int64_t nnz);
int bfs_run(int32_t n, int64_t nnz, const int32_t *rp, const int32_t *col, int32_t *lev, BfsOut *out,
            void *ws, size_t ws_bytes, hipStream_t s);

// Partition into N0 (rank-split rows) and N1
// Padding (ints) on both sides of the N0/N1 list arrays.
constexpr int kListPad = 16;

struct PartBufs {
    int32_t *rp0, *c0, *up0, *rp1, *c1;   // outputs (rp* are n+1)
    int32_t *d0;                          // n: |N0(x)|
    int32_t *rpu;                         // n+1: prefix of up0
    int64_t *e0x2;                        // device scalar: 2|E0|
    int4 *vrec = nullptr;                 // n: {rp0, |N0+|, rp1, |N1|} per vertex, or NULL
    int32_t *pos0 = nullptr, *pos1 = nullptr;   // input entry of every c0 / c1 entry (nnz each), or NULL
    int by_id = 0;                        // N0+ by id (TC_ORIENT_ID) instead of rank
};
size_t partition_ws_bytes(int32_t n, int64_t nnz);
// Turns a partition into the full-row view the cover-edge count runs on
// (up0 zeroed, vrec rewritten, rp1/c1 pointing at the input CSR).
int cover_view_run(int32_t n, const int32_t *rp, const int32_t *col, PartBufs *pb, hipStream_t s);
int partition_run(int32_t n, int64_t nnz, const int32_t *rp, const int32_t *col, const int32_t *lev,
                  const PartBufs &pb, void *ws, size_t ws_bytes, hipStream_t s);

// Counting phase (bucketize + intersect)
struct CountOut {
    uint64_t T0 = 0, T1 = 0;
    int64_t units = 0, items = 0, probes = 0, hashed = 0;
    int64_t e0x2 = 0;   // 2|E0|
    int32_t strategy_items[TC_NUM_STRATEGIES] = {0, 0, 0, 0};
    float ms_bucket = 0.f, ms_isect = 0.f;
};
// Per-vertex and per-edge counts keep a hit counter beside every hash table
// slot, so their tables get half the LDS: at most these many slots.
constexpr int kCountedMaxWgSlots = 16384;
constexpr int kCountedMaxWaveSlots = 1024;

struct CountCfg {
    int schedule = TC_SCHED_HEURISTIC;
    int force = TC_STRAT_AUTO;
    int wave_slots = 2048;
    int wg_slots = 32768;
    int chunk_work = 0;   // 0: by input size (default_chunk_work)
    int grid_blocks = 0;
    int wave_max_owner = 0;
    int wg_slice_max = 0;   // longest owner slice of a workgroup table; 0: wg_slots / 4
    int merge_max_owner = 0;
    int orientation = TC_ORIENT_RANK;   // of the N0+ lists (the partition reads it)
    const int32_t *table = nullptr;   // device per-bucket strategies (schedule)
    unsigned long long *prof = nullptr;   // device per-(bucket, strategy) profile, or NULL
    const int32_t *gid = nullptr;         // batch: graph of every vertex, or NULL
    unsigned long long *batch_counts = nullptr;   // batch: one count per graph (zeroed by the caller)
    unsigned long long *tv = nullptr;   // per-vertex triangle counts, n entries (zeroed by count_run), or NULL
    uint32_t *sup = nullptr;   // per-edge support, one per input entry (zeroed by count_run), or NULL; needs pos0/1
    const int32_t *rp = nullptr, *col = nullptr;   // the input CSR (per-edge support only)
    const int32_t *cover_lev = nullptr;   // cover-edge count (over a cover_view_run view): the levels, or NULL
    bool timing = false;
    bool sync = true;   // false: enqueue only; no host read, no synchronisation (out is not filled)
    unsigned long long *result = nullptr;   // device uint64[4] or NULL: receives {T, T0, T1, |E0|} on the stream
};
// The intersection kernel's launch shape for cfg, resolved once per device
// before any stream capture (count_run then finds it cached).
int count_prepare(int32_t n, int64_t nnz, const CountCfg &cfg);

// Levels of one graph by a single workgroup (no host read): scratch of
// bfs_single_ws_bytes(n).
size_t bfs_single_ws_bytes(int32_t n);
int bfs_single_run(int32_t n, const int32_t *rp, const int32_t *col, int32_t *lev, void *ws, size_t ws_bytes,
                   hipStream_t s);

// ------------------------------------------------------------------ shared by the entry points

// The buffers one count over n vertices and nnz entries takes from a
// workspace: levels (own_levels), the partition's lists and records (with
// the per-entry maps of per-edge support when edge_pos), a flag block and
// the scratch shared by the BFS, partition and counting phases.
struct CountPlanBufs {
    int32_t *levels;
    PartBufs pb;
    void *scratch;
    size_t scratch_bytes;
    int32_t *flag;
};
CountPlanBufs carve_count_plan(Carver &c, int32_t n, int64_t nnz, bool own_levels, bool edge_pos);
// TC_ERR_WORKSPACE unless ws holds `need` bytes and is 256-byte aligned.
int check_workspace(void *ws, size_t ws_bytes, size_t need);
// TC_VALIDATE's device check of a CSR (and levels, when non-NULL) through
// one int of scratch; synchronises the stream.
int validate_device(int32_t n, int64_t nnz, const int32_t *rp, const int32_t *col, const int32_t *lev,
                    int32_t *scratch, hipStream_t s);
// Probe elements per wavefront item when the options leave it at 0: 16384
// below 2^23 input entries, 32768 below 2^24, 65536 from there on.
int default_chunk_work(int64_t nnz);
// Checked options -> configuration (TC_ERR_ARG for invalid options).
int options_cfg(const tc_options *opt, CountCfg *cfg, int *flags);
size_t count_ws_bytes(int32_t n, int64_t nnz);
// The strategy each bucket gets under cfg for a graph of n vertices and nnz
// entries (force, table or heuristic, after the feasibility rules).
int schedule_table_run(int32_t n, int64_t nnz, const CountCfg &cfg, int32_t *table, hipStream_t s);
int count_run(int32_t n, int64_t nnz, const PartBufs &pb, const CountCfg &cfg, CountOut *out,
              void *ws, size_t ws_bytes, hipStream_t s);

}  // namespace tc
