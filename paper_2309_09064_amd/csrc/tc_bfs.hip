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
constexpr int kSamples = 1024;

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

// Most frequent label among kSamples hashed vertices (one block).
__global__ __launch_bounds__(kSamples) void k_cc_sample_mode(int32_t n, const int32_t *comp, int32_t *giant) {
    __shared__ int32_t s[kSamples];
    __shared__ int32_t best_len[kSamples / kWave];
    __shared__ int32_t best_val[kSamples / kWave];
    const int t = threadIdx.x;
    uint32_t h = (uint32_t)t * 2654435761u + 0x9E3779B9u;
    h ^= h >> 15;
    h *= 2246822519u;
    h ^= h >> 13;
    s[t] = comp[(int64_t)h % n];
    __syncthreads();
    for (int k = 2; k <= kSamples; k <<= 1) {         // bitonic sort
        for (int j = k >> 1; j > 0; j >>= 1) {
            int p = t ^ j;
            if (p > t) {
                int32_t a = s[t], b = s[p];
                bool up = (t & k) == 0;
                if ((a > b) == up) { s[t] = b; s[p] = a; }
            }
            __syncthreads();
        }
    }
    // run length ending at t, if t ends a run
    int len = 0;
    if (t == kSamples - 1 || s[t] != s[t + 1]) {
        int i = t;
        while (i >= 0 && s[i] == s[t]) --i;
        len = t - i;
    }
    int32_t val = s[t];
    for (int d = kWave / 2; d > 0; d >>= 1) {
        int ol = __shfl_xor(len, d, kWave);
        int32_t ov = __shfl_xor(val, d, kWave);
        if (ol > len || (ol == len && ov < val)) { len = ol; val = ov; }
    }
    if (lane_id() == 0) { best_len[t / kWave] = len; best_val[t / kWave] = val; }
    __syncthreads();
    if (t == 0) {
        int bl = -1;
        int32_t bv = 0;
        for (int i = 0; i < kSamples / kWave; ++i)
            if (best_len[i] > bl || (best_len[i] == bl && best_val[i] < bv)) { bl = best_len[i]; bv = best_val[i]; }
        *giant = bv;
    }
}

// Finish the linking: every edge whose row is outside the sampled giant
// component, except the first two entries of each row (already linked).
__global__ __launch_bounds__(kThreads) void k_cc_link_rest(int32_t n, int64_t nnz, const int32_t *__restrict__ rp,
                                                            const int32_t *__restrict__ col, const int32_t *giant,
                                                            int32_t *comp) {
    const int32_t g = *giant;
    const int64_t nruns = (nnz + kRun - 1) / kRun;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nruns; r += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e0 = r * kRun;
        const int64_t e1 = e0 + kRun < nnz ? e0 + kRun : nnz;
        int64_t x = row_of(rp, 0, n - 1, e0);
        int64_t xe = rp[x + 1];
        bool skip = comp[x] == g;
        for (int64_t e = e0; e < e1; ++e) {
            while (e >= xe) { ++x; xe = rp[x + 1]; skip = comp[x] == g; }
            if (!skip && e - rp[x] >= 2) link(comp, (int32_t)x, col[e]);
        }
    }
}

// Level 0: roots (label == own id).  Roots with edges seed the frontier.
__global__ void k_bfs_init(int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ comp,
                           int32_t *__restrict__ lev, int32_t *__restrict__ front, int32_t *__restrict__ fcount) {
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n; base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = base + threadIdx.x;
        bool seed = false;
        if (v < n) {
            bool root = comp[v] == (int32_t)v;
            lev[v] = root ? 0 : -1;
            seed = root && rp[v + 1] > rp[v];
        }
        uint64_t bal = __ballot(seed);
        int32_t wbase = 0;
        if (lane_id() == 0 && bal) wbase = atomicAdd(fcount, __popcll(bal));
        wbase = __shfl(wbase, 0, kWave);
        if (seed) {
            int l = lane_id();
            uint64_t lt = l == 0 ? 0ull : (~0ull >> (64 - l));
            front[wbase + __popcll(bal & lt)] = (int32_t)v;
        }
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
// thread takes kRun consecutive (frontier vertex, neighbour) pairs.
__global__ __launch_bounds__(kThreads) void k_bfs_expand(int32_t f, const int32_t *__restrict__ front,
                                                          const int64_t *__restrict__ fpre,
                                                          const int32_t *__restrict__ rp,
                                                          const int32_t *__restrict__ col, int32_t next_level,
                                                          int32_t *lev, int32_t *__restrict__ next,
                                                          int32_t *__restrict__ ncount) {
    const int64_t E = fpre[f];
    const int64_t nruns = (E + kRun - 1) / kRun;
    const int l = lane_id();
    const uint64_t lt = l == 0 ? 0ull : (~0ull >> (64 - l));
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t rb = (int64_t)blockIdx.x * blockDim.x; rb < nruns; rb += stride) {
        const int64_t r = rb + threadIdx.x;
        const bool active = r < nruns;
        int64_t e0 = r * kRun;
        int64_t i = 0, iend = 0, base = 0;
        if (active) {
            i = row_of(fpre, 0, f - 1, e0);
            iend = fpre[i + 1];
            base = (int64_t)rp[front[i]] - fpre[i];
        }
        for (int k = 0; k < kRun; ++k) {
            const int64_t e = e0 + k;
            bool found = false;
            int32_t w = 0;
            if (active && e < E) {
                while (e >= iend) { ++i; iend = fpre[i + 1]; base = (int64_t)rp[front[i]] - fpre[i]; }
                w = col[base + e];
                if (lev[w] < 0 && atomicCAS(&lev[w], -1, next_level) == -1) found = true;
            }
            uint64_t bal = __ballot(found);
            if (bal) {
                int32_t wbase = 0;
                if (l == 0) wbase = atomicAdd(ncount, __popcll(bal));
                wbase = __shfl(wbase, 0, kWave);
                if (found) next[wbase + __popcll(bal & lt)] = w;
            }
        }
    }
}

unsigned grid_for(int64_t work, int threads, int64_t cap = 65536) {
    int64_t g = (work + threads - 1) / threads;
    if (g > cap) g = cap;
    if (g < 1) g = 1;
    return (unsigned)g;
}

struct BfsLayout {
    int32_t *comp, *fa, *fb, *fdeg, *cnt, *giant;
    int64_t *fpre;
    void *scan;
};

BfsLayout carve_bfs(Carver &c, int32_t n) {
    BfsLayout L;
    const int64_t nn = n > 0 ? n : 1;
    L.comp = c.take<int32_t>(nn);
    L.fa = c.take<int32_t>(nn);
    L.fb = c.take<int32_t>(nn);
    L.fdeg = c.take<int32_t>(nn);
    L.fpre = c.take<int64_t>(nn + 1);
    L.cnt = c.take<int32_t>(64);
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

    TC_HIP_TRY(hipMemsetAsync(L.cnt, 0, 2 * sizeof(int32_t), s));
    hipLaunchKernelGGL(k_bfs_init, dim3(gv), dim3(kThreads), 0, s, n, rp, L.comp, lev, L.fa, L.cnt);
    TC_HIP_TRY(hipGetLastError());
    int32_t *cur = L.fa, *nxt = L.fb;
    int ci = 0;
    int32_t level = 0, rounds = 0;
    for (;;) {
        int32_t f = 0;
        TC_HIP_TRY(hipMemcpyAsync(&f, L.cnt + ci, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        TC_HIP_TRY(hipStreamSynchronize(s));
        if (f == 0) break;
        ++rounds;
        TC_HIP_TRY(hipMemsetAsync(L.cnt + (ci ^ 1), 0, sizeof(int32_t), s));
        hipLaunchKernelGGL(k_front_deg, dim3(grid_for(f, kThreads)), dim3(kThreads), 0, s, f, cur, rp, L.fdeg);
        TC_HIP_TRY(hipGetLastError());
        TC_TRY(scan_exclusive_i32_to_i64(L.fdeg, L.fpre, f, L.scan, s));
        hipLaunchKernelGGL(k_bfs_expand, dim3((unsigned)di.cus * 8), dim3(kThreads), 0, s, f, cur, L.fpre, rp,
                           col, level + 1, lev, nxt, L.cnt + (ci ^ 1));
        TC_HIP_TRY(hipGetLastError());
        int32_t *t = cur; cur = nxt; nxt = t;
        ci ^= 1;
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
