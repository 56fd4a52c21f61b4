// BFS levels with the serial semantics of Algorithm 4's first loop: each
// component is searched from its smallest vertex id.  The roots are found as
// connected components whose labels converge to the minimum id (links always
// hook the larger root under the smaller; the sampling-then-finish order of
// Sutton, Ben-Nun and Bar-Yossef's Afforest), then one multi-source
// level-synchronous BFS runs from all roots at once.  Hop distances are
// unique, so the result does not depend on the order of the parallel work.
#include "tc_internal.hpp"

namespace tc {
namespace {

constexpr int kThreads = 256;
constexpr int kRun = 8;           // CSR entries per thread in edge passes
constexpr int kSamples = 256;

__device__ __forceinline__ void link(int32_t *comp, int32_t u, int32_t v) {
    int32_t p1 = comp[u], p2 = comp[v];
    while (p1 != p2) {
        int32_t high = p1 > p2 ? p1 : p2;
        int32_t low = p1 + p2 - high;
        int32_t ph = comp[high];
        if (ph == low) break;
        if (ph == high && atomicCAS(&comp[high], high, low) == high) break;
        p1 = comp[comp[high]];
        p2 = comp[low];
    }
}

__global__ void k_cc_init(int32_t n, int32_t *comp) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        comp[v] = (int32_t)v;
}

__global__ void k_cc_link_round(int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                int r, int32_t *comp) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        int32_t b = rp[v], e = rp[v + 1];
        if (e - b > r) link(comp, (int32_t)v, col[b + r]);
    }
}

__global__ void k_cc_compress(int32_t n, int32_t *comp) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        int32_t c = comp[v];
        while (c != comp[c]) c = comp[c];
        comp[v] = c;
    }
}

// Most frequent label among kSamples hashed vertices (one block): every
// thread counts the samples equal to its own, ties go to the smaller label.
__global__ __launch_bounds__(kSamples) void k_cc_sample_mode(int32_t n, const int32_t *comp, int32_t *giant) {
    __shared__ int32_t smp[kSamples];
    __shared__ int64_t best[kSamples / kWave];
    const int t = threadIdx.x;
    uint32_t h = (uint32_t)t * 2654435761u + 0x9E3779B9u;
    h ^= h >> 15;
    h *= 2246822519u;
    h ^= h >> 13;
    smp[t] = comp[(int64_t)h % n];
    __syncthreads();
    const int32_t mine = smp[t];
    int32_t c = 0;
    for (int i = 0; i < kSamples; ++i) c += smp[i] == mine;
    // larger count wins, then smaller label: pack as (count, -label)
    int64_t key = ((int64_t)c << 32) | (uint32_t)(0x7fffffff - mine);
    for (int d = kWave / 2; d > 0; d >>= 1) {
        int64_t o = __shfl_xor(key, d, kWave);
        key = o > key ? o : key;
    }
    if (lane_id() == 0) best[t / kWave] = key;
    __syncthreads();
    if (t == 0) {
        int64_t b = best[0];
        for (int i = 1; i < kSamples / kWave; ++i) b = best[i] > b ? best[i] : b;
        *giant = 0x7fffffff - (int32_t)(b & 0xffffffff);
    }
}

// Finish the linking: every edge whose row is outside the sampled giant
// component, except the first two entries of each row (already linked).
__global__ __launch_bounds__(kThreads) void k_cc_link_rest(int32_t n, int64_t nnz, const int32_t *__restrict__ rp,
                                                            const int32_t *__restrict__ col, const int32_t *giant,
                                                            int32_t *comp) {
    __shared__ int64_t rows[2];
    const int32_t g = *giant;
    constexpr int64_t kTile = (int64_t)kThreads * kRun;
    for (int64_t t0 = (int64_t)blockIdx.x * kTile; t0 < nnz; t0 += (int64_t)gridDim.x * kTile) {
        tile_rows(rp, n, t0, t0 + kTile < nnz ? t0 + kTile : nnz, rows);
        const int64_t e0 = t0 + (int64_t)threadIdx.x * kRun;
        if (e0 < nnz) {
            const int64_t e1 = e0 + kRun < nnz ? e0 + kRun : nnz;
            int64_t x = row_of(rp, rows[0], rows[1], e0);
            int64_t xe = rp[x + 1];
            bool skip = comp[x] == g;
            for (int64_t e = e0; e < e1; ++e) {
                while (e >= xe) { ++x; xe = rp[x + 1]; skip = comp[x] == g; }
                if (!skip && e - rp[x] >= 2) link(comp, (int32_t)x, col[e]);
            }
        }
        __syncthreads();   // `rows` is rewritten for the next tile
    }
}

// Level 0: the roots (label == own id); every other vertex starts unvisited.
__global__ void k_bfs_init(int32_t n, const int32_t *__restrict__ comp, int32_t *__restrict__ lev) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        lev[v] = comp[v] == (int32_t)v ? 0 : -1;
}

// Frontier of `level`: flag[v] = 1 for vertices on that level with an edge.
__global__ void k_level_flags(int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ lev,
                              int32_t level, int32_t *__restrict__ flag) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        flag[v] = lev[v] == level && rp[v + 1] > rp[v];
}

__global__ void k_compact(int32_t n, const int32_t *__restrict__ flag, const int32_t *__restrict__ pos,
                          int32_t *__restrict__ front) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        if (flag[v]) front[pos[v]] = (int32_t)v;
}

__global__ void k_front_deg(int32_t f, const int32_t *__restrict__ front, const int32_t *__restrict__ rp,
                            int32_t *__restrict__ fdeg) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < f; i += (int64_t)gridDim.x * blockDim.x) {
        int32_t u = front[i];
        fdeg[i] = rp[u + 1] - rp[u];
    }
}

// Top-down expansion over the concatenated adjacency of the frontier: each
// thread takes kRun consecutive (frontier vertex, neighbour) pairs and sets
// unvisited neighbours to the next level.  Every writer stores the same
// value, so plain stores suffice.
__global__ __launch_bounds__(kThreads) void k_bfs_expand(int32_t f, const int32_t *__restrict__ front,
                                                          const int64_t *__restrict__ fpre,
                                                          const int32_t *__restrict__ rp,
                                                          const int32_t *__restrict__ col, int32_t next_level,
                                                          int32_t *lev) {
    __shared__ int64_t rows[2];
    const int64_t E = fpre[f];
    constexpr int64_t kTile = (int64_t)kThreads * kRun;
    for (int64_t t0 = (int64_t)blockIdx.x * kTile; t0 < E; t0 += (int64_t)gridDim.x * kTile) {
        tile_rows(fpre, f, t0, t0 + kTile < E ? t0 + kTile : E, rows);
        const int64_t e0 = t0 + (int64_t)threadIdx.x * kRun;
        if (e0 < E) {
            const int64_t e1 = e0 + kRun < E ? e0 + kRun : E;
            int64_t i = row_of(fpre, rows[0], rows[1], e0);
            int64_t iend = fpre[i + 1];
            int64_t base = (int64_t)rp[front[i]] - fpre[i];
            for (int64_t e = e0; e < e1; ++e) {
                while (e >= iend) { ++i; iend = fpre[i + 1]; base = (int64_t)rp[front[i]] - fpre[i]; }
                const int32_t w = col[base + e];
                if (lev[w] < 0) lev[w] = next_level;
            }
        }
        __syncthreads();   // `rows` is rewritten for the next tile
    }
}

// Bottom-up step: every unvisited vertex looks for a neighbour on the current
// level and stops at the first one.  Rows longer than kBigRow are scanned by
// the whole wavefront, 64 neighbours per step.  A vertex set here holds
// next_level != level, so concurrent readers looking for `level` are unaffected.
constexpr int32_t kBigRow = 64;

__global__ __launch_bounds__(kThreads) void k_bfs_bottom_up(int32_t n, const int32_t *__restrict__ rp,
                                                             const int32_t *__restrict__ col, int32_t level,
                                                             int32_t *lev) {
    const int l = lane_id();
    for (int64_t vb = (int64_t)blockIdx.x * blockDim.x; vb < n; vb += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = vb + threadIdx.x;
        bool todo = false;
        int32_t b = 0, e = 0;
        if (v < n && lev[v] < 0) {
            b = rp[v];
            e = rp[v + 1];
            todo = e > b;
        }
        const bool big = todo && e - b > kBigRow;
        bool found = false;
        if (todo && !big) {
            for (int32_t j = b; j < e; ++j)
                if (lev[col[j]] == level) { found = true; break; }
        }
        uint64_t bm = __ballot(big);
        while (bm) {
            const int src = __ffsll((unsigned long long)bm) - 1;
            bm &= bm - 1;
            const int32_t sb = __shfl(b, src, kWave), se = __shfl(e, src, kWave);
            bool hit = false;
            for (int32_t j = sb; j < se && !hit; j += kWave) {
                const bool h = j + l < se && lev[col[j + l]] == level;
                hit = __ballot(h) != 0;
            }
            if (l == src) found = hit;
        }
        if (found) lev[v] = level + 1;
    }
}

unsigned grid_for(int64_t work, int threads, int64_t cap = 65536) {
    int64_t g = (work + threads - 1) / threads;
    if (g > cap) g = cap;
    if (g < 1) g = 1;
    return (unsigned)g;
}

struct BfsLayout {
    int32_t *comp, *front, *flag, *pos, *fdeg, *giant;
    int64_t *fpre;
    void *scan;
};

BfsLayout carve_bfs(Carver &c, int32_t n) {
    BfsLayout L;
    const int64_t nn = n > 0 ? n : 1;
    L.comp = c.take<int32_t>(nn);
    L.front = c.take<int32_t>(nn);
    L.flag = c.take<int32_t>(nn);
    L.pos = c.take<int32_t>(nn + 1);
    L.fdeg = c.take<int32_t>(nn);
    L.fpre = c.take<int64_t>(nn + 1);
    L.giant = c.take<int32_t>(64);
    L.scan = c.take<char>(scan_ws_bytes(nn));
    return L;
}

}  // namespace

size_t bfs_ws_bytes(int32_t n, int64_t nnz) {
    (void)nnz;
    Carver c(nullptr, 0);
    carve_bfs(c, n);
    return c.used();
}

int bfs_run(int32_t n, int64_t nnz, const int32_t *rp, const int32_t *col, int32_t *lev, BfsOut *out,
            void *ws, size_t ws_bytes, hipStream_t s) {
    Carver c(ws, ws_bytes);
    BfsLayout L = carve_bfs(c, n);
    if (!c.fits()) return TC_ERR_WORKSPACE;
    if (out) *out = BfsOut{};
    if (n == 0) return TC_OK;
    DeviceInfo di;
    TC_TRY(device_info(&di));
    const unsigned gv = grid_for(n, kThreads);
    hipLaunchKernelGGL(k_cc_init, dim3(gv), dim3(kThreads), 0, s, n, L.comp);
    for (int r = 0; r < 2; ++r) {
        hipLaunchKernelGGL(k_cc_link_round, dim3(gv), dim3(kThreads), 0, s, n, rp, col, r, L.comp);
        hipLaunchKernelGGL(k_cc_compress, dim3(gv), dim3(kThreads), 0, s, n, L.comp);
    }
    hipLaunchKernelGGL(k_cc_sample_mode, dim3(1), dim3(kSamples), 0, s, n, L.comp, L.giant);
    if (nnz > 0) {
        const unsigned ge = grid_for((nnz + kRun - 1) / kRun, kThreads, (int64_t)di.cus * 8);
        hipLaunchKernelGGL(k_cc_link_rest, dim3(ge), dim3(kThreads), 0, s, n, nnz, rp, col, L.giant, L.comp);
    }
    hipLaunchKernelGGL(k_cc_compress, dim3(gv), dim3(kThreads), 0, s, n, L.comp);
    TC_HIP_TRY(hipGetLastError());

    hipLaunchKernelGGL(k_bfs_init, dim3(gv), dim3(kThreads), 0, s, n, L.comp, lev);
    TC_HIP_TRY(hipGetLastError());
    Mailbox mb;
    TC_TRY(mailbox(&mb));
    int32_t level = 0, rounds = 0;
    const unsigned gb = grid_for(n, kThreads, (int64_t)di.cus * 8);
    for (;;) {
        // frontier of `level` (vertices with an edge), compacted in id order
        hipLaunchKernelGGL(k_level_flags, dim3(gv), dim3(kThreads), 0, s, n, rp, lev, level, L.flag);
        TC_HIP_TRY(hipGetLastError());
        TC_TRY(scan_exclusive_i32_to_i32(L.flag, L.pos, n, L.scan, s));
        TC_TRY(mail_i32(L.pos + n, mb.dev, s));
        TC_HIP_TRY(hipStreamSynchronize(s));
        const int32_t f = (int32_t)mb.host[0];
        if (f == 0) break;
        ++rounds;
        if ((int64_t)f * 16 > (int64_t)n) {
            // large frontier: bottom-up, every unvisited vertex checks its row
            hipLaunchKernelGGL(k_bfs_bottom_up, dim3(gb), dim3(kThreads), 0, s, n, rp, col, level, lev);
            TC_HIP_TRY(hipGetLastError());
        } else {
            hipLaunchKernelGGL(k_compact, dim3(gv), dim3(kThreads), 0, s, n, L.flag, L.pos, L.front);
            hipLaunchKernelGGL(k_front_deg, dim3(grid_for(f, kThreads)), dim3(kThreads), 0, s, f, L.front, rp,
                               L.fdeg);
            TC_HIP_TRY(hipGetLastError());
            TC_TRY(scan_exclusive_i32_to_i64(L.fdeg, L.fpre, f, L.scan, s));
            hipLaunchKernelGGL(k_bfs_expand, dim3((unsigned)di.cus * 8), dim3(kThreads), 0, s, f, L.front, L.fpre,
                               rp, col, level + 1, lev);
            TC_HIP_TRY(hipGetLastError());
        }
        ++level;
    }
    // `level` is the number of expansions; the last one found nothing unless
    // no vertex has an edge, so the deepest level equals level - 1 (or 0).
    if (out) {
        out->levels = level > 0 ? level : 1;
        out->rounds = rounds;
    }
    return TC_OK;
}

}  // namespace tc
