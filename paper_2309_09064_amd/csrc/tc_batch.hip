// Batched counting: many graphs of uneven size, each given as its own CSR
// with local ids, counted by one pass of the pipeline over their disjoint
// union.  The batch is cut into groups of consecutive graphs whose union fits
// int32 ids and entry positions; per group:
//   1. the group CSR: row pointers and ids rebased to the group (one kernel
//      each), with every id clamped into its own graph so that a malformed
//      input can never reach outside the buffers (TC_VALIDATE reports it);
//   2. BFS levels with the serial semantics of Algorithm 4's first loop, one
//      workgroup per graph (largest graphs first), so no host read and no
//      device-wide barrier is needed between levels;
//   3. the partition, bucketing and the persistent intersection kernel of
//      the single-graph path, each hit added to its graph's counter.
// Nothing in that sequence reads results on the host, so it can be captured
// into a graph once and replayed (tc_batch_plan_*).
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "tc_internal.hpp"

namespace tc {
namespace {

constexpr int kThreads = 256;
constexpr int kRun = 8;
constexpr int kBfsThreads = 1024;
constexpr int kBfsWaves = kBfsThreads / kWave;
constexpr int kBfsRun = 8;
constexpr int kBfsLdsVerts = 65536;   // graphs up to this size keep their visited bits in LDS (8 KB)
constexpr int64_t kGroupMax = (int64_t(1) << 31) - 1024;   // vertices or entries of one group

// Largest g in [lo, hi] with off[g] <= x.
template <class T>
__device__ __forceinline__ int32_t last_le(const T *off, int32_t lo, int32_t hi, int64_t x) {
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if ((int64_t)off[mid] <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Group row pointers and the graph of every group vertex.  Packed vertex
// pv = v0 + v of graph g (voff[g] <= pv < voff[g+1]) has its local row
// pointers at row_ptr[voff[g] + g + (pv - voff[g])].  bad (or NULL) gets bit
// 0 for local row pointers that do not run from 0 to the graph's entries.
__global__ void k_batch_rp(int32_t g0, int32_t g1, int64_t v0, int64_t nv, int64_t e0, int64_t ne,
                           const int64_t *__restrict__ voff, const int64_t *__restrict__ eoff,
                           const int32_t *__restrict__ row_ptr, int32_t *__restrict__ rp_g, int32_t *__restrict__ gid,
                           int32_t *__restrict__ bad) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
        const int64_t pv = v0 + v;
        const int32_t g = last_le(voff, g0, g1 - 1, pv);
        const int64_t i = pv - voff[g];
        const int64_t at = voff[g] + g + i;
        const int64_t ng_e = eoff[g + 1] - eoff[g];
        int64_t a = row_ptr[at], b = row_ptr[at + 1];
        if (bad && ((i == 0 && a != 0) || b < a || b > ng_e || (pv + 1 == voff[g + 1] && b != ng_e)))
            atomicOr(bad, 1);
        a = a < 0 ? 0 : (a > ng_e ? ng_e : a);   // kept inside the graph's entries
        rp_g[v] = (int32_t)(eoff[g] - e0 + a);
        gid[v] = g - g0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) rp_g[nv] = (int32_t)ne;
}

// Group ids: the local id y of entry e of graph g becomes voff[g] - v0 + y.
// bad (or NULL) gets bit 1 for a local id outside [0, n_g); such an id is
// clamped into its graph.  A block takes tiles of kThreads * kRun entries,
// thread t entries t, t + kThreads, ... (each load and store of a wavefront
// contiguous).  One thread finds the graphs of the tile's first and last
// entries: a tile inside one graph (most entries) needs no search at all,
// and otherwise an entry searches only that range of graphs.
__global__ __launch_bounds__(kThreads) void k_batch_col(int32_t g0, int32_t g1, int64_t v0, int64_t e0, int64_t ne,
                                                         const int64_t *__restrict__ voff,
                                                         const int64_t *__restrict__ eoff,
                                                         const int32_t *__restrict__ col, int32_t *__restrict__ col_g,
                                                         int32_t *__restrict__ bad) {
    constexpr int64_t kTile = (int64_t)kThreads * kRun;
    __shared__ int32_t s_g[2];
    for (int64_t t0 = (int64_t)blockIdx.x * kTile; t0 < ne; t0 += (int64_t)gridDim.x * kTile) {
        if (threadIdx.x == 0) {
            const int64_t t1 = t0 + kTile < ne ? t0 + kTile : ne;
            s_g[0] = last_le(eoff, g0, g1 - 1, e0 + t0);
            s_g[1] = last_le(eoff, s_g[0], g1 - 1, e0 + t1 - 1);
        }
        __syncthreads();
        const int32_t glo = s_g[0], ghi = s_g[1];
        __syncthreads();   // s_g is rewritten for the next tile
        const int32_t base0 = (int32_t)(voff[glo] - v0), ng0 = (int32_t)(voff[glo + 1] - voff[glo]);
#pragma unroll
        for (int k = 0; k < kRun; ++k) {
            const int64_t e = t0 + (int64_t)k * kThreads + threadIdx.x;
            if (e >= ne) break;
            int32_t base = base0, ng = ng0;
            if (ghi != glo) {
                const int32_t g = last_le(eoff, glo, ghi, e0 + e);
                base = (int32_t)(voff[g] - v0);
                ng = (int32_t)(voff[g + 1] - voff[g]);
            }
            int32_t y = col[e0 + e];
            if (y < 0 || y >= ng) {
                if (bad) atomicOr(bad, 2);
                y = y < 0 ? 0 : ng - 1;
            }
            col_g[e] = base + y;
        }
    }
}

// A level as other waves of the workgroup left it: levels are set by
// compare-and-swap at the device's cache, so they are read at device scope
// rather than from a line this CU may hold.
__device__ __forceinline__ int32_t level_of(const int32_t *lev, int32_t v) {
    return __hip_atomic_load(lev + v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// BFS levels of every graph of a group, one workgroup per graph, graphs
// taken in `order` (largest first).  Per graph: isolated vertices are roots
// at level 0; then, repeatedly, the smallest unvisited vertex is the root of
// its component (Algorithm 4's loop over v in id order) and a
// level-synchronous BFS from it labels the component.  A level expands the
// concatenated rows of its frontier, kBfsRun entries a thread, and a vertex
// joins the next frontier through the one atomic that claims it, so every
// vertex is expanded once.  Graphs of at most kBfsLdsVerts vertices keep a
// visited bit per vertex in LDS: the per-entry test and the claim are LDS
// operations, and only the claiming thread writes the level to memory;
// larger graphs test and claim with the levels themselves.  fa, fb and pre
// are scratch of (vertices), (vertices) and (vertices + graphs) ints;
// *levels_max receives the largest level count.
// Held to 64 vector registers (eight wavefronts per SIMD), so that two
// graphs' workgroups share a CU.
__global__ __launch_bounds__(kBfsThreads, 8) void k_bfs_batch(int32_t graphs, const int32_t *__restrict__ order,
                                                            int32_t g0, int64_t v0, const int64_t *__restrict__ voff,
                                                            const int32_t *__restrict__ rp,
                                                            const int32_t *__restrict__ col, int32_t *lev,
                                                            int32_t *fa, int32_t *fb, int32_t *pre,
                                                            int32_t *levels_max) {
    __shared__ int32_t s_front, s_next, s_root;
    __shared__ int32_t s_wsum[kBfsWaves];
    __shared__ uint32_t s_vis[kBfsLdsVerts / 32];   // visited bits of a small graph's vertices
    const int t = threadIdx.x;
    for (int32_t k = blockIdx.x; k < graphs; k += gridDim.x) {
        const int32_t gi = order[k];
        const int32_t vb = (int32_t)(voff[g0 + gi] - v0), ve = (int32_t)(voff[g0 + gi + 1] - v0);
        int32_t *P = pre + vb + gi;   // room for (ve - vb) + 1 prefix values
        const bool in_lds = ve - vb <= kBfsLdsVerts;
        for (int32_t v = vb + t; v < ve; v += kBfsThreads) lev[v] = rp[v + 1] == rp[v] ? 0 : -1;
        if (in_lds) {   // isolated vertices start visited, like their level 0
            for (int32_t wd = t; wd < (ve - vb + 31) / 32; wd += kBfsThreads) {
                uint32_t bits = 0;
                for (int j = 0; j < 32; ++j) {
                    const int32_t v = vb + wd * 32 + j;
                    if (v < ve && rp[v + 1] == rp[v]) bits |= 1u << j;
                }
                s_vis[wd] = bits;
            }
        }
        __syncthreads();
        int32_t next = vb;
        int32_t deepest = 0;
        for (;;) {
            // the smallest unvisited vertex at or after `next` (every one has
            // an edge: isolated vertices are already at level 0)
            int32_t root = -1;
            while (next < ve) {
                if (t == 0) s_root = INT32_MAX;
                __syncthreads();
                const int32_t v = next + t;
                if (v < ve && level_of(lev, v) < 0) atomicMin(&s_root, v);
                __syncthreads();
                const int32_t m = s_root;
                __syncthreads();   // s_root is reset by the next round
                if (m != INT32_MAX) {
                    root = m;
                    break;
                }
                next += kBfsThreads;
            }
            if (root < 0) break;
            next = root + 1;
            int32_t *F = fa + vb, *N = fb + vb;
            if (t == 0) {
                lev[root] = 0;
                if (in_lds) s_vis[(root - vb) >> 5] |= 1u << ((root - vb) & 31);
                F[0] = root;
                s_front = 1;
            }
            __syncthreads();
            int32_t level = 0;
            for (;;) {
                const int32_t f = s_front;
                if (f == 0) break;
                // exclusive prefix of the frontier's degrees: thread t sums a
                // contiguous chunk, a block scan orders the chunks
                const int32_t per = (f + kBfsThreads - 1) / kBfsThreads;
                const int32_t c0 = t * per < f ? t * per : f, c1 = c0 + per < f ? c0 + per : f;
                int32_t sum = 0;
                for (int32_t i = c0; i < c1; ++i) sum += rp[F[i] + 1] - rp[F[i]];
                const int32_t inc = wave_incl_scan(sum);
                if (lane_id() == kWave - 1) s_wsum[t / kWave] = inc;
                if (t == 0) s_next = 0;
                __syncthreads();
                int32_t run = inc - sum;
                for (int i = 0; i < t / kWave; ++i) run += s_wsum[i];
                for (int32_t i = c0; i < c1; ++i) {
                    P[i] = run;
                    run += rp[F[i] + 1] - rp[F[i]];
                }
                if (c1 == f && c0 < c1) P[f] = run;
                __syncthreads();
                const int32_t E = P[f];
                for (int64_t r = t; r * kBfsRun < E; r += kBfsThreads) {
                    const int32_t a = (int32_t)(r * kBfsRun), b = a + kBfsRun < E ? a + kBfsRun : E;
                    int32_t i = last_le(P, 0, f - 1, a);
                    int32_t iend = P[i + 1];
                    int32_t base = rp[F[i]] - P[i];
                    // the run's neighbour ids, then their levels, then the
                    // compare-and-swaps: independent loads in flight rather
                    // than one dependent chain per entry.  The levels are
                    // read at workgroup scope (a line this CU holds may be
                    // stale): a stale -1 only costs the compare-and-swap,
                    // which decides.
                    int32_t w[kBfsRun], lw[kBfsRun];
#pragma unroll
                    for (int k = 0; k < kBfsRun; ++k) {
                        const int32_t e = a + k;
                        w[k] = -1;
                        if (e < b) {
                            while (e >= iend) {
                                ++i;
                                iend = P[i + 1];
                                base = rp[F[i]] - P[i];
                            }
                            w[k] = col[base + e];
                        }
                    }
                    if (in_lds) {
                        // the visited bit: tested, then claimed by one atomic
                        // or (a stale clear bit only costs the atomic); ids
                        // outside the graph, which validation rejects, are
                        // skipped rather than indexed
                        const uint32_t nv_g = (uint32_t)(ve - vb);
#pragma unroll
                        for (int k = 0; k < kBfsRun; ++k) {
                            const uint32_t o = (uint32_t)(w[k] - vb);
                            lw[k] = w[k] >= 0 && o < nv_g
                                        ? (int32_t)((__hip_atomic_load(&s_vis[o >> 5], __ATOMIC_RELAXED,
                                                                       __HIP_MEMORY_SCOPE_WORKGROUP) >> (o & 31)) & 1u)
                                        : 1;
                        }
#pragma unroll
                        for (int k = 0; k < kBfsRun; ++k)
                            if (!lw[k]) {
                                const uint32_t o = (uint32_t)(w[k] - vb), bit = 1u << (o & 31);
                                if (!(atomicOr(&s_vis[o >> 5], bit) & bit)) {
                                    lev[w[k]] = level + 1;
                                    N[atomicAdd(&s_next, 1)] = w[k];
                                }
                            }
                    } else {
#pragma unroll
                        for (int k = 0; k < kBfsRun; ++k)
                            lw[k] = w[k] >= 0 ? __hip_atomic_load(lev + w[k], __ATOMIC_RELAXED,
                                                                  __HIP_MEMORY_SCOPE_WORKGROUP)
                                              : 0;
#pragma unroll
                        for (int k = 0; k < kBfsRun; ++k)
                            if (lw[k] < 0 && atomicCAS(&lev[w[k]], -1, level + 1) == -1)
                                N[atomicAdd(&s_next, 1)] = w[k];
                    }
                }
                __syncthreads();   // the next frontier is complete
                if (t == 0) s_front = s_next;
                int32_t *tmp = F;
                F = N;
                N = tmp;
                ++level;
                __syncthreads();
            }
            deepest = level > deepest ? level : deepest;
        }
        if (t == 0) atomicMax(levels_max, deepest > 0 ? deepest : 1);
        __syncthreads();   // shared state is reused by the next graph
    }
}

// Copies the group's part of the packed levels (caller-given levels).
__global__ void k_copy_i32(const int32_t *__restrict__ src, int32_t *__restrict__ dst, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

unsigned grid_for(int64_t work, int threads, int64_t cap) {
    int64_t g = (work + threads - 1) / threads;
    if (g > cap) g = cap;
    if (g < 1) g = 1;
    return (unsigned)g;
}

struct Group {
    int32_t g0, g1;   // graphs [g0, g1)
    int64_t v0, v1;   // packed vertices
    int64_t e0, e1;   // packed entries
};

// Checks the offsets and cuts the batch into groups of consecutive graphs
// whose vertices and entries each stay within `cap` (a graph larger than cap
// gets a group of its own; every graph must fit int32 on its own).
int make_groups(int32_t graphs, const int64_t *voff, const int64_t *eoff, int64_t cap, std::vector<Group> *out) {
    out->clear();
    if (graphs < 0 || !voff || !eoff) return TC_ERR_ARG;
    if (voff[0] != 0 || eoff[0] != 0) return TC_ERR_ARG;
    for (int32_t g = 0; g < graphs; ++g) {
        const int64_t nv = voff[g + 1] - voff[g], ne = eoff[g + 1] - eoff[g];
        if (nv < 0 || ne < 0) return TC_ERR_ARG;
        if (nv == 0 && ne != 0) return TC_ERR_ARG;
        if (nv > kGroupMax || ne > kGroupMax) return TC_ERR_OVERFLOW;
    }
    if (cap <= 0 || cap > kGroupMax) cap = kGroupMax;
    int32_t g = 0;
    while (g < graphs) {
        Group G{g, g + 1, voff[g], voff[g + 1], eoff[g], eoff[g + 1]};
        while (G.g1 < graphs && voff[G.g1 + 1] - G.v0 <= cap && eoff[G.g1 + 1] - G.e0 <= cap) {
            ++G.g1;
            G.v1 = voff[G.g1];
            G.e1 = eoff[G.g1];
        }
        out->push_back(G);
        g = G.g1;
    }
    return TC_OK;
}

struct BatchLayout {
    int64_t *voff, *eoff;   // device copies of the offsets
    int32_t *order;         // per group, its graphs largest first (group-relative)
    int32_t *rp_g, *col_g, *gid, *lev;
    int32_t *fa, *fb, *pre;
    int32_t *flag;          // [0] input check bits, [1] largest level count
    CountPlanBufs plan;
};

BatchLayout carve_batch(Carver &c, int32_t graphs, int64_t max_v, int64_t max_e, int64_t max_g) {
    BatchLayout L;
    L.voff = c.take<int64_t>((size_t)graphs + 1);
    L.eoff = c.take<int64_t>((size_t)graphs + 1);
    L.order = c.take<int32_t>(graphs > 0 ? graphs : 1);
    const int64_t nv = max_v > 0 ? max_v : 1;
    L.rp_g = c.take<int32_t>(nv + 1);
    L.col_g = c.take<int32_t>(max_e > 0 ? max_e : 1);
    L.gid = c.take<int32_t>(nv);
    L.lev = c.take<int32_t>(nv);
    L.fa = c.take<int32_t>(nv);
    L.fb = c.take<int32_t>(nv);
    L.pre = c.take<int32_t>(nv + max_g + 1);
    L.flag = c.take<int32_t>(64);
    L.plan = carve_count_plan(c, (int32_t)nv, max_e, false, false);
    return L;
}

struct BatchShape {
    std::vector<Group> groups;
    int64_t max_v = 0, max_e = 0, max_g = 0;
};

int batch_shape(int32_t graphs, const int64_t *voff, const int64_t *eoff, const tc_options *opt, BatchShape *sh) {
    const int64_t cap = opt ? opt->batch_group_entries : 0;
    if (cap < 0) return TC_ERR_ARG;
    TC_TRY(make_groups(graphs, voff, eoff, cap, &sh->groups));
    for (const Group &G : sh->groups) {
        sh->max_v = std::max(sh->max_v, G.v1 - G.v0);
        sh->max_e = std::max(sh->max_e, G.e1 - G.e0);
        sh->max_g = std::max(sh->max_g, (int64_t)(G.g1 - G.g0));
    }
    return TC_OK;
}

size_t batch_ws_bytes(int32_t graphs, const BatchShape &sh) {
    Carver c(nullptr, 0);
    carve_batch(c, graphs, sh.max_v, sh.max_e, sh.max_g);
    return c.used();
}

// Host part shared by the eager call and the plan: copies the offsets and
// the largest-first order of every group into the workspace (synchronously:
// the host arrays may go away after the call).
int upload_batch(int32_t graphs, const int64_t *voff, const int64_t *eoff, const BatchShape &sh,
                 const BatchLayout &L, hipStream_t s) {
    std::vector<int32_t> order((size_t)(graphs > 0 ? graphs : 1));
    for (const Group &G : sh.groups) {
        int32_t *o = order.data() + G.g0;
        for (int32_t i = 0; i < G.g1 - G.g0; ++i) o[i] = i;
        std::stable_sort(o, o + (G.g1 - G.g0), [&](int32_t a, int32_t b) {
            return eoff[G.g0 + a + 1] - eoff[G.g0 + a] > eoff[G.g0 + b + 1] - eoff[G.g0 + b];
        });
    }
    TC_HIP_TRY(hipMemcpyAsync(L.voff, voff, sizeof(int64_t) * ((size_t)graphs + 1), hipMemcpyHostToDevice, s));
    TC_HIP_TRY(hipMemcpyAsync(L.eoff, eoff, sizeof(int64_t) * ((size_t)graphs + 1), hipMemcpyHostToDevice, s));
    if (graphs > 0)
        TC_HIP_TRY(hipMemcpyAsync(L.order, order.data(), sizeof(int32_t) * (size_t)graphs, hipMemcpyHostToDevice, s));
    TC_HIP_TRY(hipStreamSynchronize(s));
    return TC_OK;
}

// Enqueues the whole batch: counts zeroed, then every group's rebase, BFS
// (unless levels are given), partition and intersections.  With
// check = true the input checks run and are read back per group (eager
// calls only); co (optional) accumulates the groups' statistics and needs
// cfg.sync.
int enqueue_batch(int32_t graphs, const BatchShape &sh, const BatchLayout &L, const int32_t *d_row_ptr,
                  const int32_t *d_col_idx, const int32_t *d_levels, const CountCfg &base_cfg, uint64_t *d_counts,
                  bool check, CountOut *co, int32_t *levels_out, hipStream_t s) {
    DeviceInfo di;
    TC_TRY(device_info(&di));
    if (graphs > 0) TC_TRY(fill_u32(d_counts, 0, 2 * (int64_t)graphs, s));
    TC_TRY(fill_u32(L.flag, 0, 64, s));
    for (const Group &G : sh.groups) {
        const int64_t nv = G.v1 - G.v0, ne = G.e1 - G.e0;
        const int32_t ng = G.g1 - G.g0;
        if (nv == 0) continue;   // only empty graphs: their counts stay 0
        int32_t *bad = check ? L.flag : nullptr;
        hipLaunchKernelGGL(k_batch_rp, dim3(grid_for(nv, kThreads, 65536)), dim3(kThreads), 0, s, G.g0, G.g1, G.v0,
                           nv, G.e0, ne, L.voff, L.eoff, d_row_ptr, L.rp_g, L.gid, bad);
        TC_HIP_TRY(hipGetLastError());
        if (ne > 0) {
            hipLaunchKernelGGL(k_batch_col, dim3(grid_for((ne + kRun - 1) / kRun, kThreads, (int64_t)di.cus * 16)),
                               dim3(kThreads), 0, s, G.g0, G.g1, G.v0, G.e0, ne, L.voff, L.eoff, d_col_idx, L.col_g,
                               bad);
            TC_HIP_TRY(hipGetLastError());
        }
        if (check) {
            TC_TRY(validate_device((int32_t)nv, ne, L.rp_g, L.col_g, nullptr, L.flag + 2, s));
            int32_t b = 0;
            TC_HIP_TRY(hipMemcpyAsync(&b, L.flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
            TC_HIP_TRY(hipStreamSynchronize(s));
            if (b) return TC_ERR_INVALID_CSR;
        }
        if (d_levels) {
            hipLaunchKernelGGL(k_copy_i32, dim3(grid_for(nv, kThreads, 65536)), dim3(kThreads), 0, s, d_levels + G.v0,
                               L.lev, nv);
        } else {
            hipLaunchKernelGGL(k_bfs_batch, dim3((unsigned)std::min<int64_t>(ng, 65535)), dim3(kBfsThreads), 0, s, ng,
                               L.order + G.g0, G.g0, G.v0, L.voff, L.rp_g, L.col_g, L.lev, L.fa, L.fb, L.pre,
                               L.flag + 1);
        }
        TC_HIP_TRY(hipGetLastError());
        if (check && d_levels) {
            TC_TRY(validate_device((int32_t)nv, ne, L.rp_g, L.col_g, L.lev, L.flag + 2, s));
        }
        PartBufs pb = L.plan.pb;
        pb.by_id = base_cfg.orientation == TC_ORIENT_ID ? 1 : 0;
        TC_TRY(partition_run((int32_t)nv, ne, L.rp_g, L.col_g, L.lev, pb, L.plan.scratch, L.plan.scratch_bytes, s));
        CountCfg cfg = base_cfg;
        cfg.gid = L.gid;
        cfg.batch_counts = reinterpret_cast<unsigned long long *>(d_counts + G.g0);
        CountOut one;
        TC_TRY(count_run((int32_t)nv, ne, L.plan.pb, cfg, &one, L.plan.scratch, L.plan.scratch_bytes, s));
        if (co && cfg.sync) {
            co->T0 += one.T0;
            co->T1 += one.T1;
            co->e0x2 += one.e0x2;
            co->units += one.units;
            co->items += one.items;
            co->probes += one.probes;
            co->hashed += one.hashed;
            for (int k = 0; k < TC_NUM_STRATEGIES; ++k) co->strategy_items[k] += one.strategy_items[k];
            co->ms_bucket += one.ms_bucket;
            co->ms_isect += one.ms_isect;
        }
    }
    if (levels_out) {
        int32_t lv = 0;
        TC_HIP_TRY(hipMemcpyAsync(&lv, L.flag + 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        TC_HIP_TRY(hipStreamSynchronize(s));
        *levels_out = lv;
    }
    return TC_OK;
}

// Levels only: every group's rebase and BFS, the group's levels copied to
// d_levels at its packed vertices.
int enqueue_levels(const BatchShape &sh, const BatchLayout &L, const int32_t *d_row_ptr, const int32_t *d_col_idx,
                   int32_t *d_levels, hipStream_t s) {
    DeviceInfo di;
    TC_TRY(device_info(&di));
    TC_TRY(fill_u32(L.flag, 0, 64, s));
    for (const Group &G : sh.groups) {
        const int64_t nv = G.v1 - G.v0, ne = G.e1 - G.e0;
        const int32_t ng = G.g1 - G.g0;
        if (nv == 0) continue;
        hipLaunchKernelGGL(k_batch_rp, dim3(grid_for(nv, kThreads, 65536)), dim3(kThreads), 0, s, G.g0, G.g1, G.v0,
                           nv, G.e0, ne, L.voff, L.eoff, d_row_ptr, L.rp_g, L.gid, (int32_t *)nullptr);
        if (ne > 0)
            hipLaunchKernelGGL(k_batch_col, dim3(grid_for((ne + kRun - 1) / kRun, kThreads, (int64_t)di.cus * 16)),
                               dim3(kThreads), 0, s, G.g0, G.g1, G.v0, G.e0, ne, L.voff, L.eoff, d_col_idx, L.col_g,
                               (int32_t *)nullptr);
        hipLaunchKernelGGL(k_bfs_batch, dim3((unsigned)std::min<int64_t>(ng, 65535)), dim3(kBfsThreads), 0, s, ng,
                           L.order + G.g0, G.g0, G.v0, L.voff, L.rp_g, L.col_g, d_levels + G.v0, L.fa, L.fb, L.pre,
                           L.flag + 1);
        TC_HIP_TRY(hipGetLastError());
    }
    return TC_OK;
}

__global__ void k_single_graph(int32_t n, int64_t *voff, int32_t *order) {
    if (threadIdx.x == 0) {
        voff[0] = 0;
        voff[1] = n;
        order[0] = 0;
    }
}

}  // namespace

// Levels of one graph by the one-workgroup BFS kernel: no host read, no
// device-wide barrier (the no-allocation count computes its levels so).
size_t bfs_single_ws_bytes(int32_t n) {
    Carver c(nullptr, 0);
    const int64_t nv = n > 0 ? n : 1;
    c.take<int64_t>(2);
    c.take<int32_t>(1);
    c.take<int32_t>(nv);
    c.take<int32_t>(nv);
    c.take<int32_t>(nv + 2);
    c.take<int32_t>(64);
    return c.used();
}

int bfs_single_run(int32_t n, const int32_t *rp, const int32_t *col, int32_t *lev, void *ws, size_t ws_bytes,
                   hipStream_t s) {
    if (n <= 0) return TC_OK;
    Carver c(ws, ws_bytes);
    const int64_t nv = n;
    int64_t *voff = c.take<int64_t>(2);
    int32_t *order = c.take<int32_t>(1);
    int32_t *fa = c.take<int32_t>(nv);
    int32_t *fb = c.take<int32_t>(nv);
    int32_t *pre = c.take<int32_t>(nv + 2);
    int32_t *flag = c.take<int32_t>(64);
    if (!c.fits()) return TC_ERR_WORKSPACE;
    hipLaunchKernelGGL(k_single_graph, dim3(1), dim3(64), 0, s, n, voff, order);
    TC_TRY(fill_u32(flag, 0, 64, s));
    hipLaunchKernelGGL(k_bfs_batch, dim3(1), dim3(kBfsThreads), 0, s, 1, order, 0, (int64_t)0, voff, rp, col, lev, fa,
                       fb, pre, flag);
    TC_HIP_TRY(hipGetLastError());
    return TC_OK;
}

namespace {

int batch_cfg(const tc_options *opt, CountCfg *cfg, int *flags) {
    TC_TRY(options_cfg(opt, cfg, flags));
    if (cfg->schedule == TC_SCHED_TABLE && !cfg->table) return TC_ERR_ARG;
    return TC_OK;
}

int fail(int code) {
    set_error(code);
    return code;
}

}  // namespace
}  // namespace tc

using namespace tc;

struct tc_batch_plan {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int device = 0;
};

extern "C" {

int tc_count_batched_ws(int32_t graphs, const int64_t *h_vtx_off, const int64_t *h_edge_off, const tc_options *opt,
                        size_t *h_ws_bytes) {
    if (!h_ws_bytes) return fail(TC_ERR_ARG);
    CountCfg cfg;
    int flags;
    int rc = options_cfg(opt, &cfg, &flags);
    if (rc != TC_OK) return fail(rc);
    BatchShape sh;
    rc = batch_shape(graphs, h_vtx_off, h_edge_off, opt, &sh);
    if (rc != TC_OK) return fail(rc);
    *h_ws_bytes = batch_ws_bytes(graphs, sh);
    return fail(TC_OK);
}

uint64_t tc_count_batched(int32_t graphs, const int64_t *h_vtx_off, const int64_t *h_edge_off,
                          const int32_t *d_row_ptr, const int32_t *d_col_idx, const int32_t *d_levels,
                          const tc_options *opt, uint64_t *d_counts, tc_stats *stats, void *ws, size_t ws_bytes,
                          void *stream) {
    CountCfg cfg;
    int flags;
    int rc = batch_cfg(opt, &cfg, &flags);
    BatchShape sh;
    if (rc == TC_OK) rc = batch_shape(graphs, h_vtx_off, h_edge_off, opt, &sh);
    if (rc == TC_OK && graphs > 0 && !d_counts) rc = TC_ERR_ARG;
    if (rc == TC_OK && graphs > 0 && h_vtx_off[graphs] > 0 && !d_row_ptr) rc = TC_ERR_ARG;
    if (rc == TC_OK && graphs > 0 && h_edge_off[graphs] > 0 && !d_col_idx) rc = TC_ERR_ARG;
    if (rc == TC_OK) rc = check_workspace(ws, ws_bytes, batch_ws_bytes(graphs, sh));
    DeviceInfo di;
    if (rc == TC_OK) rc = device_info(&di);
    if (rc != TC_OK) {
        fail(rc);
        return TC_COUNT_ERROR;
    }
    if (stats) memset(stats, 0, sizeof(*stats));
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (graphs == 0) {
        fail(TC_OK);
        return 0;
    }
    Carver c(ws, ws_bytes);
    const BatchLayout L = carve_batch(c, graphs, sh.max_v, sh.max_e, sh.max_g);
    rc = upload_batch(graphs, h_vtx_off, h_edge_off, sh, L, s);
    CountOut co;
    int32_t levels = 0;
    if (rc == TC_OK)
        rc = enqueue_batch(graphs, sh, L, d_row_ptr, d_col_idx, d_levels, cfg, d_counts, (flags & TC_VALIDATE) != 0,
                           &co, &levels, s);
    if (rc != TC_OK) {
        fail(rc);
        return TC_COUNT_ERROR;
    }
    if (stats) {
        stats->T0 = co.T0;
        stats->T1 = co.T1;
        stats->e0 = co.e0x2 / 2;
        stats->units = co.units;
        stats->items = co.items;
        stats->probes = co.probes;
        stats->hashed = co.hashed;
        stats->levels = d_levels ? 0 : levels;
        for (int k = 0; k < TC_NUM_STRATEGIES; ++k) stats->strategy_items[k] = co.strategy_items[k];
        stats->ms_bucket = co.ms_bucket;
        stats->ms_isect = co.ms_isect;
    }
    fail(TC_OK);
    return co.T0 + co.T1;
}

int tc_bfs_levels_batched(int32_t graphs, const int64_t *h_vtx_off, const int64_t *h_edge_off,
                          const int32_t *d_row_ptr, const int32_t *d_col_idx, int32_t *d_levels,
                          int32_t *h_levels_count, void *ws, size_t ws_bytes, void *stream) {
    BatchShape sh;
    int rc = batch_shape(graphs, h_vtx_off, h_edge_off, nullptr, &sh);
    if (rc != TC_OK) return fail(rc);
    if (graphs > 0 && h_vtx_off[graphs] > 0 && (!d_row_ptr || !d_levels)) return fail(TC_ERR_ARG);
    if (graphs > 0 && h_edge_off[graphs] > 0 && !d_col_idx) return fail(TC_ERR_ARG);
    rc = check_workspace(ws, ws_bytes, batch_ws_bytes(graphs, sh));
    if (rc != TC_OK) return fail(rc);
    DeviceInfo di;
    rc = device_info(&di);
    if (rc != TC_OK) return fail(rc);
    if (graphs == 0) {
        if (h_levels_count) *h_levels_count = 0;
        return fail(TC_OK);
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    Carver c(ws, ws_bytes);
    const BatchLayout L = carve_batch(c, graphs, sh.max_v, sh.max_e, sh.max_g);
    rc = upload_batch(graphs, h_vtx_off, h_edge_off, sh, L, s);
    if (rc == TC_OK) rc = enqueue_levels(sh, L, d_row_ptr, d_col_idx, d_levels, s);
    int32_t lv = 0;
    if (rc == TC_OK && (hipMemcpyAsync(&lv, L.flag + 1, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
                        hipStreamSynchronize(s) != hipSuccess))
        rc = TC_ERR_HIP;
    if (rc == TC_OK && h_levels_count) *h_levels_count = lv;
    return fail(rc);
}

int tc_batch_plan_create(int32_t graphs, const int64_t *h_vtx_off, const int64_t *h_edge_off,
                         const int32_t *d_row_ptr, const int32_t *d_col_idx, const tc_options *opt,
                         uint64_t *d_counts, void *ws, size_t ws_bytes, void *stream, tc_batch_plan **out) {
    if (!out) return fail(TC_ERR_ARG);
    *out = nullptr;
    CountCfg cfg;
    int flags;
    int rc = batch_cfg(opt, &cfg, &flags);
    if (rc != TC_OK) return fail(rc);
    if (flags & (TC_TIMING | TC_VALIDATE)) return fail(TC_ERR_ARG);   // both read results on the host
    BatchShape sh;
    rc = batch_shape(graphs, h_vtx_off, h_edge_off, opt, &sh);
    if (rc != TC_OK) return fail(rc);
    if (graphs > 0 && !d_counts) return fail(TC_ERR_ARG);
    if (graphs > 0 && h_vtx_off[graphs] > 0 && !d_row_ptr) return fail(TC_ERR_ARG);
    if (graphs > 0 && h_edge_off[graphs] > 0 && !d_col_idx) return fail(TC_ERR_ARG);
    rc = check_workspace(ws, ws_bytes, batch_ws_bytes(graphs, sh));
    if (rc != TC_OK) return fail(rc);
    DeviceInfo di;
    rc = device_info(&di);
    if (rc != TC_OK) return fail(rc);
    hipStream_t s = static_cast<hipStream_t>(stream);
    tc_batch_plan *p = new (std::nothrow) tc_batch_plan;
    if (!p) return fail(TC_ERR_HIP);
    if (hipGetDevice(&p->device) != hipSuccess) {
        delete p;
        return fail(TC_ERR_HIP);
    }
    Carver c(ws, ws_bytes);
    const BatchLayout L = carve_batch(c, graphs, sh.max_v, sh.max_e, sh.max_g);
    if (graphs > 0) rc = upload_batch(graphs, h_vtx_off, h_edge_off, sh, L, s);
    // launch shapes are resolved before the capture (host-side queries)
    for (const Group &G : sh.groups)
        if (rc == TC_OK) {
            CountCfg gc = cfg;
            gc.gid = L.gid;
            rc = count_prepare((int32_t)(G.v1 - G.v0), G.e1 - G.e0, gc);
        }
    // capture on a private stream: the caller's may be the legacy default
    // stream, which cannot be captured
    hipStream_t cs = nullptr;
    if (rc == TC_OK && hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) rc = TC_ERR_HIP;
    if (rc == TC_OK && hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) rc = TC_ERR_HIP;
    if (rc == TC_OK) {
        cfg.sync = false;
        const int er = enqueue_batch(graphs, sh, L, d_row_ptr, d_col_idx, nullptr, cfg, d_counts, false, nullptr,
                                     nullptr, cs);
        const hipError_t ee = hipStreamEndCapture(cs, &p->graph);
        rc = er != TC_OK ? er : (ee != hipSuccess ? TC_ERR_HIP : TC_OK);
    }
    if (rc == TC_OK && hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) != hipSuccess) rc = TC_ERR_HIP;
    if (cs) (void)hipStreamDestroy(cs);
    if (rc != TC_OK) {
        if (p->exec) (void)hipGraphExecDestroy(p->exec);
        if (p->graph) (void)hipGraphDestroy(p->graph);
        delete p;
        return fail(rc);
    }
    *out = p;
    return fail(TC_OK);
}

int tc_batch_plan_launch(tc_batch_plan *plan, void *stream) {
    if (!plan || !plan->exec) return fail(TC_ERR_ARG);
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != plan->device) return fail(TC_ERR_ARG);
    if (hipGraphLaunch(plan->exec, static_cast<hipStream_t>(stream)) != hipSuccess) return fail(TC_ERR_HIP);
    return fail(TC_OK);
}

int tc_batch_plan_destroy(tc_batch_plan *plan) {
    if (!plan) return fail(TC_OK);
    int rc = TC_OK;
    if (plan->exec && hipGraphExecDestroy(plan->exec) != hipSuccess) rc = TC_ERR_HIP;
    if (plan->graph && hipGraphDestroy(plan->graph) != hipSuccess) rc = TC_ERR_HIP;
    delete plan;
    return fail(rc);
}

}  // extern "C"
