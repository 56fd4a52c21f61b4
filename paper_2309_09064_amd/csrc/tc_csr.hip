// Simple undirected CSR from raw tuples: key generation, a stable LSD radix
// sort on (u, v) keys, duplicate removal and row pointers.  This builds the
// paper's input format (CSR with sorted rows); it is not part of the timed
// count.
#include "tc_internal.hpp"

namespace tc {
namespace {

constexpr int kThreads = 256;
constexpr int kRounds = 16;                 // keys per thread per tile
constexpr int kTileKeys = kThreads * kRounds;
constexpr int kWaves = kThreads / kWave;
constexpr uint64_t kSentinel = ~0ull;

int bits_for(int64_t n) {
    int b = 1;
    while ((int64_t(1) << b) < n) ++b;
    return b;
}

// Two keys per tuple (both directions); self-loops and out-of-range tuples
// become sentinels, which sort last.
__global__ void k_make_keys(const int32_t *__restrict__ src, const int32_t *__restrict__ dst, int64_t m,
                            int32_t n, int bv, uint64_t *__restrict__ keys, int32_t *__restrict__ err) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x) {
        int32_t u = src[i], v = dst[i];
        uint64_t a = kSentinel, b = kSentinel;
        if (u < 0 || u >= n || v < 0 || v >= n) {
            atomicOr(err, 1);
        } else if (u != v) {
            a = ((uint64_t)u << bv) | (uint64_t)v;
            b = ((uint64_t)v << bv) | (uint64_t)u;
        }
        keys[2 * i] = a;
        keys[2 * i + 1] = b;
    }
}

// Per-tile digit histogram, digit-major: hist[d * nblk + blk].
__global__ __launch_bounds__(kThreads) void k_rs_hist(const uint64_t *__restrict__ keys, int64_t nkeys,
                                                       int shift, int32_t *__restrict__ hist) {
    __shared__ int32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTileKeys;
    for (int r = 0; r < kRounds; ++r) {
        int64_t i = base + (int64_t)r * kThreads + threadIdx.x;
        if (i < nkeys) atomicAdd(&h[(keys[i] >> shift) & 255u], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: keys of a tile keep their order within each digit.  Each
// round ranks 256 keys: a wave finds lanes with an equal digit by eight
// ballots, waves are ordered through LDS counters.
__global__ __launch_bounds__(kThreads) void k_rs_scatter(const uint64_t *__restrict__ in,
                                                          uint64_t *__restrict__ out, int64_t nkeys,
                                                          int shift, const int32_t *__restrict__ hoff) {
    __shared__ int32_t run[256];
    __shared__ int32_t cnt[kWaves][256];
    const int t = threadIdx.x;
    const int w = t / kWave;
    const int l = lane_id();
    run[t] = hoff[(int64_t)t * gridDim.x + blockIdx.x];
#pragma unroll
    for (int k = 0; k < kWaves; ++k) cnt[k][t] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTileKeys;
    const uint64_t lt = (l == 0) ? 0ull : (~0ull >> (64 - l));
    for (int r = 0; r < kRounds; ++r) {
        const int64_t i = base + (int64_t)r * kThreads + t;
        const bool valid = i < nkeys;
        uint64_t key = valid ? in[i] : 0ull;
        uint32_t d = (uint32_t)(key >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            bool bit = (d >> b) & 1u;
            uint64_t bal = __ballot(bit);
            peers &= bit ? bal : ~bal;
        }
        const int rank = __popcll(peers & lt);
        if (valid && rank == 0) cnt[w][d] = __popcll(peers);
        __syncthreads();   // every wave's digit counts are visible
        if (valid) {
            int before = run[d];
            for (int k = 0; k < w; ++k) before += cnt[k][d];
            out[before + rank] = key;
        }
        __syncthreads();
        int add = 0;
#pragma unroll
        for (int k = 0; k < kWaves; ++k) {
            add += cnt[k][t];
            cnt[k][t] = 0;
        }
        run[t] += add;
        __syncthreads();
    }
}

__global__ void k_uniq_flags(const uint64_t *__restrict__ keys, int64_t nkeys, int32_t *__restrict__ flag) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nkeys;
         i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t k = keys[i];
        flag[i] = (k != kSentinel) && (i == 0 || keys[i - 1] != k);
    }
}

__global__ void k_uniq_scatter(const uint64_t *__restrict__ keys, int64_t nkeys, const int32_t *__restrict__ flag,
                               const int32_t *__restrict__ pos, int bv, int32_t *__restrict__ col,
                               int32_t *__restrict__ deg) {
    const uint64_t vmask = (1ull << bv) - 1;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nkeys;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (flag[i]) {
            uint64_t k = keys[i];
            col[pos[i]] = (int32_t)(k & vmask);
            atomicAdd(&deg[(int64_t)(k >> bv)], 1);
        }
    }
}

unsigned grid_for(int64_t work, int threads) {
    int64_t g = (work + threads - 1) / threads;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (unsigned)g;
}

struct CsrLayout {
    uint64_t *ka, *kb;
    int32_t *flag, *pos, *deg, *err;
    void *sort;   // radix sort scratch, also the scans' scratch
    size_t sort_bytes;
};

CsrLayout carve_csr(Carver &c, int32_t n, int64_t m) {
    const int64_t nk = 2 * m;
    CsrLayout L;
    L.ka = c.take<uint64_t>(nk > 0 ? nk : 1);
    L.kb = c.take<uint64_t>(nk > 0 ? nk : 1);
    L.flag = c.take<int32_t>(nk + 1);
    L.pos = c.take<int32_t>(nk + 1);
    L.deg = c.take<int32_t>((int64_t)n + 1);
    L.err = c.take<int32_t>(64);
    int64_t biggest = nk > (int64_t)n ? nk : (int64_t)n;
    L.sort_bytes = radix_sort_ws_bytes(biggest);
    L.sort = c.take<char>(L.sort_bytes);
    return L;
}

struct SortLayout {
    int32_t *hist;
    void *scan;
};

SortLayout carve_sort(Carver &c, int64_t nk) {
    const int64_t nblk = (nk + kTileKeys - 1) / kTileKeys;
    SortLayout L;
    L.hist = c.take<int32_t>(256 * nblk + 1);
    L.scan = c.take<char>(scan_ws_bytes(256 * nblk > nk ? 256 * nblk : nk));
    return L;
}

}  // namespace

int bits_for_ids(int64_t n) { return bits_for(n); }

size_t radix_sort_ws_bytes(int64_t nk) {
    Carver c(nullptr, 0);
    carve_sort(c, nk);
    return c.used();
}

int radix_sort_u64(uint64_t *a, uint64_t *b, int64_t nk, int bits, void *ws, size_t ws_bytes, hipStream_t s,
                   uint64_t **sorted) {
    Carver c(ws, ws_bytes);
    SortLayout L = carve_sort(c, nk);
    if (!c.fits()) return TC_ERR_WORKSPACE;
    *sorted = a;
    if (nk <= 0) return TC_OK;
    const int64_t nblk = (nk + kTileKeys - 1) / kTileKeys;
    for (int shift = 0; shift < bits; shift += 8) {
        hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)nblk), dim3(kThreads), 0, s, a, nk, shift, L.hist);
        TC_HIP_TRY(hipGetLastError());
        TC_TRY(scan_exclusive_i32_to_i32(L.hist, L.hist, 256 * nblk, L.scan, s));
        hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)nblk), dim3(kThreads), 0, s, a, b, nk, shift, L.hist);
        TC_HIP_TRY(hipGetLastError());
        uint64_t *t = a;
        a = b;
        b = t;
    }
    *sorted = a;
    return TC_OK;
}

size_t build_csr_ws_bytes(int32_t n, int64_t m) {
    Carver c(nullptr, 0);
    carve_csr(c, n, m);
    return c.used();
}

int build_csr_run(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, int32_t *row_ptr,
                  int32_t *col, int64_t col_cap, int64_t *h_nnz, void *ws, size_t ws_bytes,
                  hipStream_t s) {
    Carver c(ws, ws_bytes);
    CsrLayout L = carve_csr(c, n, m);
    if (!c.fits()) return TC_ERR_WORKSPACE;
    const int64_t nk = 2 * m;
    TC_HIP_TRY(hipMemsetAsync(L.err, 0, sizeof(int32_t), s));
    TC_HIP_TRY(hipMemsetAsync(L.deg, 0, sizeof(int32_t) * ((size_t)n + 1), s));
    int64_t nnz = 0;
    if (nk > 0) {
        hipLaunchKernelGGL(k_make_keys, dim3(grid_for(m, 256)), dim3(256), 0, s, src, dst, m, n,
                           bits_for(n), L.ka, L.err);
        TC_HIP_TRY(hipGetLastError());
        const int bv = bits_for(n);
        uint64_t *a = nullptr;
        TC_TRY(radix_sort_u64(L.ka, L.kb, nk, 2 * bv, L.sort, L.sort_bytes, s, &a));
        hipLaunchKernelGGL(k_uniq_flags, dim3(grid_for(nk, 256)), dim3(256), 0, s, a, nk, L.flag);
        TC_HIP_TRY(hipGetLastError());
        TC_TRY(scan_exclusive_i32_to_i32(L.flag, L.pos, nk, L.sort, s));
        int32_t hv[2] = {0, 0};
        TC_HIP_TRY(hipMemcpyAsync(&hv[0], L.pos + nk, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        TC_HIP_TRY(hipMemcpyAsync(&hv[1], L.err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        TC_HIP_TRY(hipStreamSynchronize(s));
        if (hv[1]) return TC_ERR_RANGE;
        nnz = hv[0];
        if (h_nnz) *h_nnz = nnz;
        if (nnz > col_cap) return TC_ERR_CAPACITY;
        hipLaunchKernelGGL(k_uniq_scatter, dim3(grid_for(nk, 256)), dim3(256), 0, s, a, nk, L.flag, L.pos,
                           bv, col, L.deg);
        TC_HIP_TRY(hipGetLastError());
    } else if (h_nnz) {
        *h_nnz = 0;
    }
    TC_TRY(scan_exclusive_i32_to_i32(L.deg, row_ptr, n, L.sort, s));
    TC_HIP_TRY(hipStreamSynchronize(s));
    if (h_nnz) *h_nnz = nnz;
    return TC_OK;
}

}  // namespace tc
