// BFS levels with the serial semantics of Algorithm 4's first loop: each
// component is searched from its smallest vertex id.  Two passes:
//  1. the smallest vertex with an edge is necessarily the root of its
//     component (every smaller id is isolated), and isolated vertices are
//     their own roots at level 0, so a level-synchronous BFS from that one
//     vertex labels its component at once (on these graphs the giant
//     component: all but 0.1% of the vertices with edges);
//  2. only if vertices are left unvisited, their roots are found as
//     connected components whose labels converge to the minimum id (links
//     always hook the larger root under the smaller; the sampling-then-
//     finish order of Sutton, Ben-Nun and Bar-Noy's Afforest), restricted
//     to those vertices, and one multi-source BFS runs from all of them.
// Hop distances are unique, so the result does not depend on the order of
// the parallel work.
#include "tc_internal.hpp"

namespace tc {
namespace {

constexpr int kThreads = 256;
constexpr int kRun = 8;           // CSR entries per thread in edge passes

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

__global__ void k_cc_link_round(int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                int r, int32_t *comp) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        if (comp[v] < 0) continue;   // labelled by the first pass
        int32_t b = rp[v], e = rp[v + 1];
        if (e - b > r) link(comp, (int32_t)v, col[b + r]);
    }
}

__global__ void k_cc_compress(int32_t n, int32_t *comp) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        int32_t c = comp[v];
        if (c < 0) continue;   // labelled by the first pass
        while (c != comp[c]) c = comp[c];
        comp[v] = c;
    }
}

// Finish the linking: every edge whose row's label is not *skip (the first
// pass's vertices carry -1), except the first two entries of each row
// (already linked by the rounds).
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

// The smallest vertex with an edge (*first starts above n).  Launched on at
// most kFirstBlocks blocks that stride over the vertices: each thread stops
// at its first vertex with an edge, the block takes the minimum, and one
// atomic per block follows (one per wavefront over a vertex-sized grid
// serialised some 16K atomics on the one word).
constexpr int kFirstBlocks = 256;
__global__ __launch_bounds__(kThreads) void k_first_active(int32_t n, const int32_t *__restrict__ rp,
                                                            int32_t *first) {
    __shared__ int32_t s_min[kThreads / kWave];
    int32_t best = INT32_MAX;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        if (rp[v + 1] > rp[v]) {
            best = (int32_t)v;
            break;   // later vertices of this thread are larger
        }
    for (int d = kWave / 2; d > 0; d >>= 1) best = min(best, __shfl_xor(best, d, kWave));
    if (lane_id() == 0) s_min[threadIdx.x / kWave] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kThreads / kWave; ++w) best = min(best, s_min[w]);
        if (best != INT32_MAX) atomicMin(first, best);
    }
}

// Finish the linking of a small second pass: a thread per vertex of the pass
// links the rest of its row (entries from the third; the rounds linked the
// first two).  For a large second pass the tiled k_cc_link_rest is used.
__global__ void k_cc_link_rows(int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                               int32_t *comp) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        if (comp[v] < 0) continue;   // labelled by the first pass
        for (int32_t e = rp[v] + 2; e < rp[v + 1]; ++e) link(comp, (int32_t)v, col[e]);
    }
}

// First pass, level 0: that vertex and every isolated vertex; the rest
// starts unvisited.
__global__ void k_bfs_init_first(int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ first,
                                 int32_t *__restrict__ lev) {
    const int32_t f = *first;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        lev[v] = ((int32_t)v == f || rp[v + 1] == rp[v]) ? 0 : -1;
}

// Unvisited vertices after the first pass: their count, and their labels for
// the second pass (own id; -1 marks the first pass's vertices).
__global__ void k_rest_init(int32_t n, const int32_t *__restrict__ lev, int32_t *__restrict__ comp,
                            int32_t *__restrict__ count) {
    int32_t c = 0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const bool rest = lev[v] < 0;
        comp[v] = rest ? (int32_t)v : -1;
        c += rest;
    }
    if (c) atomicAdd(count, c);
}

// Second pass, level 0: the roots (label == own id) among the unvisited.
__global__ void k_bfs_init_rest(int32_t n, const int32_t *__restrict__ comp, int32_t *__restrict__ lev) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        if (comp[v] == (int32_t)v) lev[v] = 0;
}

// Frontier of `level`: the vertices on that level with an edge (in the
// second pass, only those of the pass: comp[v] >= 0), as bits (below) and,
// per 64-bit word of them, their number wcnt[v / 64] (a top-down level
// compacts the frontier from a prefix sum of n / 64 word counts).  Each block
// also writes the number and the degree sum of its frontier vertices to
// part[2 * blockIdx.x] and part[2 * blockIdx.x + 1] (launched on at most
// kFlagBlocks blocks; k_front_mail adds them up).
constexpr int kFlagBlocks = 1024;
// The frontier also as bits, one per vertex (bits[v / 64] bit v % 64): the
// bottom-up pass tests its neighbours there, an array of n / 8 bytes that
// stays in L2, instead of gathering their levels.
__global__ __launch_bounds__(kThreads) void k_level_flags(int32_t n, const int32_t *__restrict__ rp,
                                                           const int32_t *__restrict__ lev, int32_t level,
                                                           const int32_t *__restrict__ only,
                                                           int32_t *__restrict__ wcnt,
                                                           unsigned long long *__restrict__ bits,
                                                           unsigned long long *__restrict__ part) {
    __shared__ unsigned long long s_sum[kThreads / kWave][2];
    unsigned long long c = 0, d = 0;
    // a wavefront takes 64 consecutive vertices (the grid stride is a
    // multiple of 64): one bit word per wavefront and step
    for (int64_t vb = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~(kWave - 1)); vb < n;
         vb += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = vb + lane_id();
        bool in = false;
        int32_t deg = 0;
        if (v < n) {
            deg = rp[v + 1] - rp[v];
            in = lev[v] == level && deg > 0 && (only == nullptr || only[v] >= 0);
        }
        const uint64_t word = __ballot(in);
        if (lane_id() == 0) {
            bits[vb >> 6] = word;
            wcnt[vb >> 6] = __popcll(word);
        }
        c += in ? 1ull : 0ull;
        d += in ? (unsigned long long)deg : 0ull;
    }
    c = wave_sum(c);
    d = wave_sum(d);
    if (lane_id() == 0) {
        s_sum[threadIdx.x / kWave][0] = c;
        s_sum[threadIdx.x / kWave][1] = d;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kThreads / kWave; ++w) {
            c += s_sum[w][0];
            d += s_sum[w][1];
        }
        part[2 * blockIdx.x] = c;
        part[2 * blockIdx.x + 1] = d;
    }
}

// Mailbox: dst[0] = frontier size, dst[1] = the frontier's degree sum, from
// the nparts blocks' partial sums.  One block.
__global__ __launch_bounds__(kThreads) void k_front_mail(const unsigned long long *__restrict__ part, int nparts,
                                                          uint64_t *dst) {
    __shared__ unsigned long long s_sum[kThreads / kWave][2];
    unsigned long long c = 0, d = 0;
    for (int i = threadIdx.x; i < nparts; i += kThreads) {
        c += part[2 * i];
        d += part[2 * i + 1];
    }
    c = wave_sum(c);
    d = wave_sum(d);
    if (lane_id() == 0) {
        s_sum[threadIdx.x / kWave][0] = c;
        s_sum[threadIdx.x / kWave][1] = d;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kThreads / kWave; ++w) {
            c += s_sum[w][0];
            d += s_sum[w][1];
        }
        dst[0] = c;
        dst[1] = d;
    }
}

// The frontier list in id order: vertex v of the bits goes to the prefix of
// the word counts before its word plus the set bits below it in the word.
__global__ void k_compact(int32_t n, const unsigned long long *__restrict__ bits, const int32_t *__restrict__ wpos,
                          int32_t *__restrict__ front) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const unsigned long long word = bits[v >> 6];
        const int b = (int)(v & 63);
        if ((word >> b) & 1ull) front[wpos[v >> 6] + __popcll(word & ((1ull << b) - 1ull))] = (int32_t)v;
    }
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

__device__ __forceinline__ bool in_frontier(const unsigned long long *__restrict__ bits, int32_t y) {
    return (bits[y >> 6] >> (y & 63)) & 1ull;
}

__global__ __launch_bounds__(kThreads) void k_bfs_bottom_up(int32_t n, const int32_t *__restrict__ rp,
                                                             const int32_t *__restrict__ col, int32_t level,
                                                             const unsigned long long *__restrict__ bits,
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
                if (in_frontier(bits, col[j])) { found = true; break; }
        }
        uint64_t bm = __ballot(big);
        while (bm) {
            const int src = __ffsll((unsigned long long)bm) - 1;
            bm &= bm - 1;
            const int32_t sb = __shfl(b, src, kWave), se = __shfl(e, src, kWave);
            bool hit = false;
            for (int32_t j = sb; j < se && !hit; j += kWave) {
                const bool h = j + l < se && in_frontier(bits, col[j + l]);
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
    int32_t *comp, *front, *wcnt, *wpos, *fdeg, *giant;   // wcnt, wpos: per 64-bit word of bits
    unsigned long long *bits;   // the frontier, one bit per vertex
    int64_t *fpre;
    unsigned long long *part;   // per-block frontier sizes and degree sums
    void *scan;
};

BfsLayout carve_bfs(Carver &c, int32_t n) {
    BfsLayout L;
    const int64_t nn = n > 0 ? n : 1;
    L.comp = c.take<int32_t>(nn);
    L.front = c.take<int32_t>(nn);
    L.wcnt = c.take<int32_t>((nn + 63) / 64);
    L.bits = c.take<unsigned long long>((nn + 63) / 64);
    L.wpos = c.take<int32_t>((nn + 63) / 64 + 1);
    L.fdeg = c.take<int32_t>(nn);
    L.fpre = c.take<int64_t>(nn + 1);
    L.giant = c.take<int32_t>(64);
    L.part = c.take<unsigned long long>(2 * kFlagBlocks);
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
    Mailbox mb;
    TC_TRY(mailbox(&mb));
    const unsigned gb = grid_for(n, kThreads, (int64_t)di.cus * 8);
    int32_t rounds = 0;
    // level-synchronous BFS from the vertices at level 0 (restricted to
    // only[v] >= 0 when `only` is given); returns the number of expansions
    // Direction switch after Beamer, Asanovic and Patterson's
    // direction-optimising BFS: bottom-up once the frontier's edges exceed
    // 1/kAlpha of the edges not yet explored, or the frontier holds more
    // than n/16 vertices.  Every choice gives the same levels.
    constexpr int64_t kAlpha = 14;
    int64_t m_unexplored = nnz;   // across both passes: the second starts with the rest's edges
    const unsigned gf = gv < kFlagBlocks ? gv : kFlagBlocks;
    auto level_loop = [&](const int32_t *only, int32_t *levels_out) -> int {
        int32_t level = 0;
        for (;;) {
            // frontier of `level` (vertices with an edge), compacted in id order
            hipLaunchKernelGGL(k_level_flags, dim3(gf), dim3(kThreads), 0, s, n, rp, lev, level, only, L.wcnt,
                               L.bits, L.part);
            hipLaunchKernelGGL(k_front_mail, dim3(1), dim3(kThreads), 0, s, L.part, (int)gf, mb.dev);
            TC_HIP_TRY(hipGetLastError());
            TC_HIP_TRY(hipStreamSynchronize(s));
            const int32_t f = (int32_t)mb.host[0];
            const int64_t m_front = (int64_t)mb.host[1];
            if (f == 0) break;
            ++rounds;
            const bool bottom_up = m_front * kAlpha > m_unexplored || (int64_t)f * 16 > (int64_t)n;
            m_unexplored -= m_front;
            if (bottom_up) {
                // large frontier: bottom-up, every unvisited vertex checks its row
                hipLaunchKernelGGL(k_bfs_bottom_up, dim3(gb), dim3(kThreads), 0, s, n, rp, col, level, L.bits, lev);
                TC_HIP_TRY(hipGetLastError());
            } else {
                // positions in the frontier list: only top-down levels need them
                TC_TRY(scan_exclusive_i32_to_i32(L.wcnt, L.wpos, ((int64_t)n + 63) / 64, L.scan, s));
                hipLaunchKernelGGL(k_compact, dim3(gv), dim3(kThreads), 0, s, n, L.bits, L.wpos, L.front);
                hipLaunchKernelGGL(k_front_deg, dim3(grid_for(f, kThreads)), dim3(kThreads), 0, s, f, L.front, rp,
                                   L.fdeg);
                TC_HIP_TRY(hipGetLastError());
                TC_TRY(scan_exclusive_i32_to_i64(L.fdeg, L.fpre, f, L.scan, s));
                hipLaunchKernelGGL(k_bfs_expand, dim3((unsigned)di.cus * 8), dim3(kThreads), 0, s, f, L.front,
                                   L.fpre, rp, col, level + 1, lev);
                TC_HIP_TRY(hipGetLastError());
            }
            ++level;
        }
        // `level` is the number of expansions; the last one found nothing
        // unless no vertex has an edge, so the deepest level is level - 1
        *levels_out = level > 0 ? level : 1;
        return TC_OK;
    };

    // pass 1: from the smallest vertex with an edge, isolated vertices at 0
    TC_HIP_TRY(hipMemsetAsync(L.giant, 0x7f, sizeof(int32_t), s));   // above any vertex id
    hipLaunchKernelGGL(k_first_active, dim3(gv < kFirstBlocks ? gv : kFirstBlocks), dim3(kThreads), 0, s, n, rp, L.giant);
    hipLaunchKernelGGL(k_bfs_init_first, dim3(gv), dim3(kThreads), 0, s, n, rp, L.giant, lev);
    TC_HIP_TRY(hipGetLastError());
    int32_t levels1 = 1, levels2 = 1;
    TC_TRY(level_loop(nullptr, &levels1));

    // pass 2: the components the first pass did not reach
    TC_HIP_TRY(hipMemsetAsync(L.giant + 1, 0, sizeof(int32_t), s));
    hipLaunchKernelGGL(k_rest_init, dim3(gb), dim3(kThreads), 0, s, n, lev, L.comp, L.giant + 1);
    TC_HIP_TRY(hipGetLastError());
    TC_TRY(mail_i32(L.giant + 1, mb.dev, s));
    TC_HIP_TRY(hipStreamSynchronize(s));
    if (mb.host[0] > 0) {
        for (int r = 0; r < 2; ++r) {
            hipLaunchKernelGGL(k_cc_link_round, dim3(gv), dim3(kThreads), 0, s, n, rp, col, r, L.comp);
            hipLaunchKernelGGL(k_cc_compress, dim3(gv), dim3(kThreads), 0, s, n, L.comp);
        }
        if ((int64_t)mb.host[0] * 64 < (int64_t)n) {
            hipLaunchKernelGGL(k_cc_link_rows, dim3(gv), dim3(kThreads), 0, s, n, rp, col, L.comp);
        } else if (nnz > 0) {
            // rows of the first pass carry label -1: pass that label as the one to skip
            TC_HIP_TRY(hipMemsetAsync(L.giant + 2, 0xff, sizeof(int32_t), s));
            const unsigned ge = grid_for((nnz + kRun - 1) / kRun, kThreads, (int64_t)di.cus * 8);
            hipLaunchKernelGGL(k_cc_link_rest, dim3(ge), dim3(kThreads), 0, s, n, nnz, rp, col, L.giant + 2,
                               L.comp);
        }
        hipLaunchKernelGGL(k_cc_compress, dim3(gv), dim3(kThreads), 0, s, n, L.comp);
        hipLaunchKernelGGL(k_bfs_init_rest, dim3(gv), dim3(kThreads), 0, s, n, L.comp, lev);
        TC_HIP_TRY(hipGetLastError());
        TC_TRY(level_loop(L.comp, &levels2));
    }
    if (out) {
        out->levels = levels1 > levels2 ? levels1 : levels2;
        out->rounds = rounds;
    }
    return TC_OK;
}

}  // namespace tc
