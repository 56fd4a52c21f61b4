// Device-wide exclusive prefix sums (reduce-then-scan, three levels at most).
// A tile is 256 threads x 8 consecutive values; sums are kept in int64.
#include "tc_internal.hpp"

namespace tc {
namespace {

constexpr int kThreads = 256;
constexpr int kPer = 8;
constexpr int kTile = kThreads * kPer;
constexpr int kWaves = kThreads / kWave;

__device__ __forceinline__ int64_t block_excl_scan(int64_t v, int64_t *total) {
    __shared__ int64_t wsum[kWaves];
    const int t = threadIdx.x;
    const int w = t / kWave;
    int64_t inc = wave_incl_scan(v);
    if (lane_id() == kWave - 1) wsum[w] = inc;
    __syncthreads();
    int64_t before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) {
        int64_t s = wsum[i];
        before += (i < w) ? s : 0;
        all += s;
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

// A thread's kPer consecutive elements [base, base + kPer), 0 past n: by
// 16-byte loads when the run is whole and 16-byte aligned (a wavefront's
// instruction then covers 1 KB instead of 256 or 512 bytes), else one load
// each.  In-place scans read a thread's elements before it stores them, and
// no other thread touches them.
template <class T>
__device__ __forceinline__ void load_per(const T *p, int64_t base, int64_t n, int64_t (&v)[kPer]) {
    static_assert(kPer == 8 && (sizeof(T) == 4 || sizeof(T) == 8), "runs of 8 four- or eight-byte elements");
    if (base + kPer <= n && ((uintptr_t)(p + base) & 15) == 0) {
        const int4 *q = reinterpret_cast<const int4 *>(p + base);
        if (sizeof(T) == 4) {
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int4 a = q[j];
                v[4 * j] = (int64_t)(T)a.x; v[4 * j + 1] = (int64_t)(T)a.y;
                v[4 * j + 2] = (int64_t)(T)a.z; v[4 * j + 3] = (int64_t)(T)a.w;
            }
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int4 a = q[j];
                v[2 * j] = (int64_t)(T)(((uint64_t)(uint32_t)a.y << 32) | (uint32_t)a.x);
                v[2 * j + 1] = (int64_t)(T)(((uint64_t)(uint32_t)a.w << 32) | (uint32_t)a.z);
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < kPer; ++i) v[i] = base + i < n ? (int64_t)p[base + i] : 0;
    }
}

template <class T>
__device__ __forceinline__ void store_per(T *p, int64_t base, int64_t n, const int64_t (&r)[kPer]) {
    if (base + kPer <= n && ((uintptr_t)(p + base) & 15) == 0) {
        int4 *q = reinterpret_cast<int4 *>(p + base);
        if (sizeof(T) == 4) {
#pragma unroll
            for (int j = 0; j < 2; ++j)
                q[j] = make_int4((int32_t)(T)r[4 * j], (int32_t)(T)r[4 * j + 1], (int32_t)(T)r[4 * j + 2],
                                 (int32_t)(T)r[4 * j + 3]);
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint64_t a = (uint64_t)(T)r[2 * j], b = (uint64_t)(T)r[2 * j + 1];
                q[j] = make_int4((int32_t)(uint32_t)a, (int32_t)(uint32_t)(a >> 32), (int32_t)(uint32_t)b,
                                 (int32_t)(uint32_t)(b >> 32));
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < kPer; ++i)
            if (base + i < n) p[base + i] = (T)r[i];
    }
}

template <class Tin>
__global__ __launch_bounds__(kThreads) void k_scan_reduce(const Tin *__restrict__ in, int64_t n,
                                                           int64_t *__restrict__ sums) {
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kPer;
    int64_t v[kPer];
    load_per(in, base, n, v);
    int64_t acc = 0;
#pragma unroll
    for (int i = 0; i < kPer; ++i) acc += v[i];
    int64_t tot;
    (void)block_excl_scan(acc, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

template <class Tin, class Tout>
__global__ __launch_bounds__(kThreads) void k_scan_apply(const Tin *in, int64_t n, const int64_t *offs,
                                                          Tout *out) {
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kPer;
    int64_t v[kPer];
    load_per(in, base, n, v);
    int64_t acc = 0;
#pragma unroll
    for (int i = 0; i < kPer; ++i) acc += v[i];
    int64_t tot;
    int64_t run = block_excl_scan(acc, &tot);
    const int64_t off = offs ? offs[blockIdx.x] : 0;
    run += off;
    int64_t r[kPer];
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        r[i] = run;
        run += v[i];
    }
    store_per(out, base, n, r);
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = (Tout)(off + tot);
}

int64_t nblocks(int64_t n) { return (n + kTile - 1) / kTile; }

__global__ void k_fill_u32(uint32_t *__restrict__ p, uint32_t v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <class Tin, class Tout>
int scan_impl(const Tin *in, Tout *out, int64_t n, int64_t *ws, hipStream_t s) {
    if (n <= kTile) {
        hipLaunchKernelGGL((k_scan_apply<Tin, Tout>), dim3(1), dim3(kThreads), 0, s, in, n,
                           (const int64_t *)nullptr, out);
        TC_HIP_TRY(hipGetLastError());
        return TC_OK;
    }
    const int64_t nb = nblocks(n);
    int64_t *sums = ws;                 // nb + 1 entries
    int64_t *rest = ws + ((nb + 1 + 31) & ~int64_t(31));
    hipLaunchKernelGGL((k_scan_reduce<Tin>), dim3((unsigned)nb), dim3(kThreads), 0, s, in, n, sums);
    TC_HIP_TRY(hipGetLastError());
    TC_TRY((scan_impl<int64_t, int64_t>(sums, sums, nb, rest, s)));
    hipLaunchKernelGGL((k_scan_apply<Tin, Tout>), dim3((unsigned)nb), dim3(kThreads), 0, s, in, n,
                       (const int64_t *)sums, out);
    TC_HIP_TRY(hipGetLastError());
    return TC_OK;
}

}  // namespace

size_t scan_ws_bytes(int64_t n) {
    size_t total = 0;
    while (n > kTile) {
        int64_t nb = nblocks(n);
        total += (size_t)((nb + 1 + 31) & ~int64_t(31)) * sizeof(int64_t);
        n = nb;
    }
    return total + 256;
}

// For every non-empty row x: the tiles whose first entry, or whose last
// entry, lies in the row get x as their first, or last, row.  Every entry
// belongs to one row, so each tile is written once for each end.
__global__ void k_tile_table(int32_t n, const int32_t *__restrict__ rp, int32_t *__restrict__ tlo,
                             int32_t *__restrict__ thi) {
    const int64_t total = rp[n];
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a = rp[x], b = rp[x + 1];
        if (b <= a) continue;
        for (int64_t t = a / kTileEntries; t <= (b - 1) / kTileEntries; ++t) {
            const int64_t first = t * kTileEntries;
            const int64_t last = ((t + 1) * kTileEntries < total ? (t + 1) * kTileEntries : total) - 1;
            if (first >= a) tlo[t] = (int32_t)x;
            if (last < b) thi[t] = (int32_t)x;
        }
    }
}

int tile_table_run(int32_t n, const int32_t *rp, int32_t *tlo, int32_t *thi, hipStream_t s) {
    if (n <= 0) return TC_OK;
    int64_t g = ((int64_t)n + kThreads - 1) / kThreads;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_tile_table, dim3((unsigned)g), dim3(kThreads), 0, s, n, rp, tlo, thi);
    TC_HIP_TRY(hipGetLastError());
    return TC_OK;
}

int fill_u32(void *p, uint32_t value, int64_t count, hipStream_t s) {
    if (count <= 0) return TC_OK;
    int64_t g = (count + kThreads - 1) / kThreads;
    if (g > 16384) g = 16384;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)g), dim3(kThreads), 0, s, static_cast<uint32_t *>(p), value, count);
    TC_HIP_TRY(hipGetLastError());
    return TC_OK;
}

int scan_exclusive_i32_to_i32(const int32_t *in, int32_t *out, int64_t n, void *ws, hipStream_t s) {
    return scan_impl<int32_t, int32_t>(in, out, n, static_cast<int64_t *>(ws), s);
}
int scan_exclusive_i32_to_i64(const int32_t *in, int64_t *out, int64_t n, void *ws, hipStream_t s) {
    return scan_impl<int32_t, int64_t>(in, out, n, static_cast<int64_t *>(ws), s);
}
int scan_exclusive_i64_to_i64(const int64_t *in, int64_t *out, int64_t n, void *ws, hipStream_t s) {
    return scan_impl<int64_t, int64_t>(in, out, n, static_cast<int64_t *>(ws), s);
}

}  // namespace tc
