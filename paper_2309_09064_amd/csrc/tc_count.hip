// Counting phase of Algorithm 4 on the partitioned graph.
//
// Every horizontal edge {x, y} needs two intersections:
//   kind 0 (T0, triangles inside G0):   |N0+(x) & N0+(y)|    (Algorithm 2)
//   kind 1 (T1, one horizontal edge):   |N1(x)  & N1(y)|     (Algorithm 4)
// For each kind the endpoint with the larger list owns the edge (ties: larger
// id); the owner's list is hashed once and every owned partner's list is
// streamed through it, so an intersection costs the smaller list (the paper's
// min(d(u), d(v)) argument in Section II).  An intersection with an empty side
// is skipped.
//
// Work unit = (owner x, kind).  A unit is split into items that cover a range
// of x's N0 row (its partners); items are grouped by a bucket
// (kind, log2 owner size, log2 mean partner size) and each bucket is given an
// intersection strategy by the schedule.  One persistent kernel drains two
// queues: workgroup items first (a workgroup shares one LDS table), then
// wavefront items (each wavefront has a private LDS table, or searches the
// owner list in global memory).  Every strategy computes the same exact
// integer, so the schedule never changes a count.
#include "tc_internal.hpp"

namespace tc {
namespace {

constexpr int kRun = 8;                 // CSR entries per thread in row passes
constexpr int kThreads = 256;
constexpr int kIsectThreads = 512;      // 8 wavefronts per persistent block
constexpr int kIsectWaves = kIsectThreads / kWave;
constexpr int kBuckets = 2 * 32 * 32;
constexpr int kMinPartnersPerItem = 8;
constexpr int32_t kEmpty = -1;

struct Item {
    int32_t owner;
    int32_t code;   // kind | strategy << 1
    int32_t jb, je; // range of c0 positions (owner's N0 row) holding partners
};

__device__ __forceinline__ int32_t list_size(int kind, const int32_t *up0, const int32_t *rp1, int32_t v) {
    return kind == 0 ? up0[v] : rp1[v + 1] - rp1[v];
}

__device__ __forceinline__ const int32_t *list_ptr(int kind, const int32_t *rp0, const int32_t *c0,
                                                   const int32_t *rp1, const int32_t *c1, int32_t v) {
    return kind == 0 ? c0 + rp0[v] : c1 + rp1[v];
}

__device__ __forceinline__ bool owns(int32_t sx, int32_t sy, int32_t x, int32_t y) {
    return sy > 0 && (sx > sy || (sx == sy && x > y));
}

__device__ __forceinline__ int ilog2(int64_t v) { return v <= 1 ? 0 : 63 - __clzll((unsigned long long)v); }

__device__ __forceinline__ int bucket_of(int kind, int32_t sx, int64_t work, int32_t cnt) {
    int ob = ilog2(sx);
    int pb = ilog2(work / cnt);
    ob = ob > 31 ? 31 : ob;
    pb = pb > 31 ? 31 : pb;
    return (kind * 32 + ob) * 32 + pb;
}

struct SchedCfg {
    const int32_t *table;  // per-bucket strategy (nullable -> heuristic)
    int32_t force;         // >= 0: this strategy everywhere it is feasible
    int32_t wave_ob_max;   // largest owner-size class a wavefront table holds
    int32_t wg_ob_max;     // largest owner-size class the workgroup table holds
    int32_t heur_wave_ob;  // heuristic: wavefront table up to this class
    int32_t chunk_work;    // probe elements per wavefront item
};

// Strategy of a bucket.  Feasibility depends only on the owner-size class
// ob = floor(log2 |owner list|): a table of 2^k slots takes classes
// ob <= k - 2, i.e. lists shorter than half the table.
__device__ __forceinline__ int strategy_for(const SchedCfg &c, int b) {
    const int ob = (b >> 5) & 31;
    int s;
    if (c.force >= 0) s = c.force;
    else if (c.table) s = c.table[b];
    else s = ob <= c.heur_wave_ob ? TC_STRAT_WAVE_HASH : (ob <= c.wg_ob_max ? TC_STRAT_WG_HASH : TC_STRAT_BSEARCH);
    if (s == TC_STRAT_WAVE_HASH && ob > c.wave_ob_max) s = ob <= c.wg_ob_max ? TC_STRAT_WG_HASH : TC_STRAT_BSEARCH;
    if (s == TC_STRAT_WG_HASH && ob > c.wg_ob_max) s = TC_STRAT_BSEARCH;
    if (s < 0 || s >= TC_NUM_STRATEGIES) s = TC_STRAT_BSEARCH;
    return s;
}

// ---------------------------------------------------------------- ownership

// Per owner and kind: number of owned partners and their total list length.
__global__ __launch_bounds__(kThreads) void k_own(int32_t n, const int64_t *__restrict__ e0x2p,
                                                   const int32_t *__restrict__ rp0,
                                                   const int32_t *__restrict__ c0, const int32_t *__restrict__ up0,
                                                   const int32_t *__restrict__ rp1, int32_t *__restrict__ cnt,
                                                   unsigned long long *__restrict__ work) {
    const int64_t e0x2 = *e0x2p;
    const int64_t nruns = (e0x2 + kRun - 1) / kRun;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nruns; r += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e0 = r * kRun;
        const int64_t e1 = e0 + kRun < e0x2 ? e0 + kRun : e0x2;
        int64_t x = row_of(rp0, 0, n - 1, e0);
        int64_t xe = rp0[x + 1];
        int32_t s0x = up0[x], s1x = rp1[x + 1] - rp1[x];
        int32_t n0 = 0, n1 = 0;
        unsigned long long w0 = 0, w1 = 0;
        auto flush = [&]() {
            if (n0) { atomicAdd(&cnt[2 * x], n0); atomicAdd(&work[2 * x], w0); }
            if (n1) { atomicAdd(&cnt[2 * x + 1], n1); atomicAdd(&work[2 * x + 1], w1); }
            n0 = n1 = 0;
            w0 = w1 = 0;
        };
        for (int64_t e = e0; e < e1; ++e) {
            while (e >= xe) {
                flush();
                ++x;
                xe = rp0[x + 1];
                s0x = up0[x];
                s1x = rp1[x + 1] - rp1[x];
            }
            const int32_t y = c0[e];
            const int32_t s0y = up0[y], s1y = rp1[y + 1] - rp1[y];
            if (owns(s0x, s0y, (int32_t)x, y)) { ++n0; w0 += (unsigned)s0y; }
            if (owns(s1x, s1y, (int32_t)x, y)) { ++n1; w1 += (unsigned)s1y; }
        }
        flush();
    }
}

// Items per unit; count pass (fill == 0) histograms items per bucket, fill
// pass writes them.  Stats: [0] units, [1] probes, [2] hashed, [3..6] items
// per strategy.
template <int kFill>
__global__ __launch_bounds__(kThreads) void k_items(int32_t n, const int32_t *__restrict__ rp0,
                                                     const int32_t *__restrict__ up0,
                                                     const int32_t *__restrict__ rp1, const int32_t *__restrict__ cnt,
                                                     const unsigned long long *__restrict__ work, SchedCfg sc,
                                                     int32_t *__restrict__ bucket_items,
                                                     const int32_t *__restrict__ bucket_off,
                                                     int32_t *__restrict__ bucket_cur, Item *__restrict__ items,
                                                     unsigned long long *__restrict__ stats) {
    __shared__ int32_t hist[kFill ? 1 : kBuckets];
    if (!kFill) {
        for (int i = threadIdx.x; i < kBuckets; i += blockDim.x) hist[i] = 0;
        __syncthreads();
    }
    unsigned long long units = 0, probes = 0, hashed = 0, ps0 = 0, ps1 = 0, ps2 = 0, ps3 = 0;
    const int64_t total = 2 * (int64_t)n;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < total; u += (int64_t)gridDim.x * blockDim.x) {
        const int32_t c = cnt[u];
        if (c == 0) continue;
        const int32_t x = (int32_t)(u >> 1);
        const int kind = (int)(u & 1);
        const unsigned long long w = work[u];
        const int32_t sx = kind == 0 ? up0[x] : rp1[x + 1] - rp1[x];
        const int b = bucket_of(kind, sx, (int64_t)w, c);
        const int s = strategy_for(sc, b);
        const int64_t target = (int64_t)sc.chunk_work * (s == TC_STRAT_WG_HASH ? kIsectWaves : 1);
        const int32_t jb = rp0[x], je = rp0[x + 1];
        int64_t nch = ((int64_t)w + target - 1) / target;
        const int64_t cap = (je - jb + kMinPartnersPerItem - 1) / kMinPartnersPerItem;
        if (nch > cap) nch = cap;
        if (nch < 1) nch = 1;
        if (!kFill) {
            atomicAdd(&hist[b], (int32_t)nch);
            ++units;
            probes += w;
            hashed += (unsigned long long)sx * (unsigned long long)nch;
            const unsigned long long nc = (unsigned long long)nch;
            ps0 += s == 0 ? nc : 0;
            ps1 += s == 1 ? nc : 0;
            ps2 += s == 2 ? nc : 0;
            ps3 += s == 3 ? nc : 0;
        } else {
            const int32_t pos = bucket_off[b] + atomicAdd(&bucket_cur[b], (int32_t)nch);
            const int64_t len = je - jb;
            for (int64_t k = 0; k < nch; ++k) {
                Item it;
                it.owner = x;
                it.code = kind | (s << 1);
                it.jb = jb + (int32_t)(len * k / nch);
                it.je = jb + (int32_t)(len * (k + 1) / nch);
                items[pos + k] = it;
            }
        }
    }
    if (!kFill) {
        __syncthreads();
        for (int i = threadIdx.x; i < kBuckets; i += blockDim.x)
            if (hist[i]) atomicAdd(&bucket_items[i], hist[i]);
        units = wave_sum(units);
        probes = wave_sum(probes);
        hashed = wave_sum(hashed);
        ps0 = wave_sum(ps0);
        ps1 = wave_sum(ps1);
        ps2 = wave_sum(ps2);
        ps3 = wave_sum(ps3);
        if (lane_id() == 0) {
            atomicAdd(&stats[0], units);
            atomicAdd(&stats[1], probes);
            atomicAdd(&stats[2], hashed);
            atomicAdd(&stats[3], ps0);
            atomicAdd(&stats[4], ps1);
            atomicAdd(&stats[5], ps2);
            atomicAdd(&stats[6], ps3);
        }
    }
}

// Queue layout (one thread): workgroup-table buckets first, then the rest;
// inside each queue larger owners first.  q[2] = workgroup items, q[3] = all.
__global__ void k_bucket_order(const int32_t *__restrict__ bucket_items, SchedCfg sc,
                               int32_t *__restrict__ bucket_off, int32_t *__restrict__ q) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int32_t off = 0;
    for (int pass = 0; pass < 2; ++pass) {
        for (int ob = 31; ob >= 0; --ob)
            for (int pb = 31; pb >= 0; --pb)
                for (int kind = 0; kind < 2; ++kind) {
                    const int b = (kind * 32 + ob) * 32 + pb;
                    const bool wg = strategy_for(sc, b) == TC_STRAT_WG_HASH;
                    if (wg != (pass == 0)) continue;
                    bucket_off[b] = off;
                    off += bucket_items[b];
                }
        if (pass == 0) q[2] = off;
    }
    q[3] = off;
}

// ---------------------------------------------------------------- probes

__device__ __forceinline__ uint32_t hash_slot(int32_t v, int shift) {
    return ((uint32_t)v * 0x9E3779B1u) >> shift;
}

__device__ __forceinline__ void hash_insert(int32_t *tab, uint32_t mask, int shift, int32_t v) {
    uint32_t h = hash_slot(v, shift);
    while (atomicCAS(&tab[h], kEmpty, v) != kEmpty) h = (h + 1) & mask;
}

__device__ __forceinline__ uint32_t hash_has(const int32_t *tab, uint32_t mask, int shift, int32_t v) {
    uint32_t h = hash_slot(v, shift);
    for (;;) {
        int32_t t = tab[h];
        if (t == v) return 1u;
        if (t == kEmpty) return 0u;
        h = (h + 1) & mask;
    }
}

__device__ __forceinline__ uint32_t bsearch_has(const int32_t *a, int32_t len, int32_t v) {
    int32_t lo = 0, hi = len;
    while (lo < hi) {
        int32_t mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1; else hi = mid;
    }
    return (lo < len && a[lo] == v) ? 1u : 0u;
}

// first index with a[i] >= v (lower) or a[i] > v (upper)
__device__ __forceinline__ int32_t lower_idx(const int32_t *a, int32_t len, int32_t v) {
    int32_t lo = 0, hi = len;
    while (lo < hi) {
        int32_t mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}
__device__ __forceinline__ int32_t upper_idx(const int32_t *a, int32_t len, int32_t v) {
    int32_t lo = 0, hi = len;
    while (lo < hi) {
        int32_t mid = (lo + hi) >> 1;
        if (a[mid] <= v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Wave-parallel merge of sorted a (owner, length la) and b (partner, lb):
// lane l merges its 1/64 slice of a with the matching value range of b.
__device__ __forceinline__ uint32_t merge_count(const int32_t *a, int32_t la, const int32_t *b, int32_t lb) {
    const int l = lane_id();
    const int32_t a0 = (int32_t)((int64_t)la * l / kWave), a1 = (int32_t)((int64_t)la * (l + 1) / kWave);
    if (a0 >= a1) return 0u;
    int32_t i = a0;
    int32_t j = lower_idx(b, lb, a[a0]);
    const int32_t je = upper_idx(b, lb, a[a1 - 1]);
    uint32_t hits = 0;
    while (i < a1 && j < je) {
        int32_t x = a[i], y = b[j];
        if (x < y) ++i;
        else if (x > y) ++j;
        else { ++hits; ++i; ++j; }
    }
    return hits;
}

struct Graph {
    const int32_t *rp0, *c0, *up0, *rp1, *c1;
};

// Streams every owned partner list of c0 positions [jb, je) of owner x
// through `probe`; positions are split over `nw` cooperating wavefronts,
// this wavefront being number `w`.
template <class Probe>
__device__ __forceinline__ uint32_t stream_partners(const Graph &g, int kind, int32_t x, int32_t sx, int32_t jb,
                                                    int32_t je, int w, int nw, Probe probe) {
    const int l = lane_id();
    uint32_t hits = 0;
    for (int32_t base = jb + w * kWave; base < je; base += nw * kWave) {
        const int32_t p = base + l;
        int32_t y = 0, sy = 0, yb = 0;
        bool mine = false;
        if (p < je) {
            y = g.c0[p];
            if (kind == 0) { sy = g.up0[y]; yb = g.rp0[y]; }
            else { yb = g.rp1[y]; sy = g.rp1[y + 1] - yb; }
            mine = owns(sx, sy, x, y);
        }
        uint64_t m = __ballot(mine);
        const int32_t *lists = kind == 0 ? g.c0 : g.c1;
        while (m) {
            const int src = __ffsll((unsigned long long)m) - 1;
            m &= m - 1;
            const int32_t len = __shfl(sy, src, kWave);
            const int32_t *b = lists + __shfl(yb, src, kWave);
            hits += probe(b, len);
        }
    }
    return hits;
}

// Probe a list with all lanes, four elements in flight per lane.
template <class Has>
__device__ __forceinline__ uint32_t probe_list(const int32_t *b, int32_t len, Has has) {
    const int l = lane_id();
    uint32_t hits = 0;
    for (int32_t i = l; i < len; i += 4 * kWave) {
        int32_t v0 = b[i];
        int32_t v1 = i + kWave < len ? b[i + kWave] : -1;
        int32_t v2 = i + 2 * kWave < len ? b[i + 2 * kWave] : -1;
        int32_t v3 = i + 3 * kWave < len ? b[i + 3 * kWave] : -1;
        hits += has(v0);
        if (v1 >= 0) hits += has(v1);
        if (v2 >= 0) hits += has(v2);
        if (v3 >= 0) hits += has(v3);
    }
    return hits;
}

__device__ __forceinline__ int table_log2(int32_t sx, int max_log2) {
    int lg = 6;   // at least 64 slots
    while (lg < max_log2 && (1 << lg) < 2 * sx) ++lg;
    return lg;
}

__global__ __launch_bounds__(kIsectThreads) void k_isect(Graph g, const Item *__restrict__ items,
                                                          int32_t *__restrict__ q, int wg_log2, int wave_log2,
                                                          unsigned long long *__restrict__ tri) {
    extern __shared__ int32_t lds[];
    const int32_t n_wg = q[2], n_all = q[3];
    __shared__ int32_t s_item;
    const int w = threadIdx.x / kWave;
    const int l = lane_id();
    uint64_t acc[2] = {0, 0};

    // ---- workgroup items: one shared table per block
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(&q[0], 1);
        __syncthreads();
        const int32_t it = s_item;
        if (it >= n_wg) break;
        const Item item = items[it];
        const int kind = item.code & 1;
        const int32_t x = item.owner;
        const int32_t *a = list_ptr(kind, g.rp0, g.c0, g.rp1, g.c1, x);
        const int32_t sx = list_size(kind, g.up0, g.rp1, x);
        const int lg = table_log2(sx, wg_log2);
        const uint32_t mask = (1u << lg) - 1;
        const int shift = 32 - lg;
        for (int i = threadIdx.x; i <= (int)mask; i += kIsectThreads) lds[i] = kEmpty;
        __syncthreads();
        for (int i = threadIdx.x; i < sx; i += kIsectThreads) hash_insert(lds, mask, shift, a[i]);
        __syncthreads();
        acc[kind] += stream_partners(g, kind, x, sx, item.jb, item.je, w, kIsectWaves,
                                     [&](const int32_t *b, int32_t len) {
                                         return probe_list(b, len, [&](int32_t v) {
                                             return hash_has(lds, mask, shift, v);
                                         });
                                     });
        __syncthreads();   // table reuse and s_item rewrite
    }

    // ---- wavefront items
    int32_t *tab = lds + (w << wave_log2);
    for (;;) {
        int32_t it = 0;
        if (l == 0) it = atomicAdd(&q[1], 1);
        it = __shfl(it, 0, kWave) + n_wg;
        if (it >= n_all) break;
        const Item item = items[it];
        const int kind = item.code & 1;
        const int strat = item.code >> 1;
        const int32_t x = item.owner;
        const int32_t *a = list_ptr(kind, g.rp0, g.c0, g.rp1, g.c1, x);
        const int32_t sx = list_size(kind, g.up0, g.rp1, x);
        if (strat == TC_STRAT_WAVE_HASH) {
            const int lg = table_log2(sx, wave_log2);
            const uint32_t mask = (1u << lg) - 1;
            const int shift = 32 - lg;
            for (int i = l; i <= (int)mask; i += kWave) tab[i] = kEmpty;
            wave_lds_sync();
            for (int i = l; i < sx; i += kWave) hash_insert(tab, mask, shift, a[i]);
            wave_lds_sync();
            acc[kind] += stream_partners(g, kind, x, sx, item.jb, item.je, 0, 1, [&](const int32_t *b, int32_t len) {
                return probe_list(b, len, [&](int32_t v) { return hash_has(tab, mask, shift, v); });
            });
            wave_lds_sync();
        } else if (strat == TC_STRAT_MERGE) {
            acc[kind] += stream_partners(g, kind, x, sx, item.jb, item.je, 0, 1, [&](const int32_t *b, int32_t len) {
                return merge_count(a, sx, b, len);
            });
        } else {
            acc[kind] += stream_partners(g, kind, x, sx, item.jb, item.je, 0, 1, [&](const int32_t *b, int32_t len) {
                return probe_list(b, len, [&](int32_t v) { return bsearch_has(a, sx, v); });
            });
        }
    }

    uint64_t t0 = wave_sum(acc[0]);
    uint64_t t1 = wave_sum(acc[1]);
    if (l == 0) {
        if (t0) atomicAdd(&tri[0], (unsigned long long)t0);
        if (t1) atomicAdd(&tri[1], (unsigned long long)t1);
    }
}

unsigned grid_for(int64_t work, int threads, int64_t cap) {
    int64_t g = (work + threads - 1) / threads;
    if (g > cap) g = cap;
    if (g < 1) g = 1;
    return (unsigned)g;
}

struct CountLayout {
    int32_t *cnt;
    unsigned long long *work;
    int32_t *bucket_items, *bucket_off, *bucket_cur, *q;
    Item *items;
    unsigned long long *stats;   // [0..6] unit stats, [8..9] T0/T1
};

int64_t item_capacity(int32_t n, int64_t nnz) {
    // per unit: at most ceil(|N0(x)| / kMinPartnersPerItem) items
    return 2 * ((int64_t)n + nnz / kMinPartnersPerItem) + 64;
}

CountLayout carve_count(Carver &c, int32_t n, int64_t nnz) {
    CountLayout L;
    const int64_t nn = n > 0 ? n : 1;
    L.cnt = c.take<int32_t>(2 * nn);
    L.work = c.take<unsigned long long>(2 * nn);
    L.bucket_items = c.take<int32_t>(kBuckets + 1);
    L.bucket_off = c.take<int32_t>(kBuckets + 1);
    L.bucket_cur = c.take<int32_t>(kBuckets);
    L.q = c.take<int32_t>(64);
    L.items = c.take<Item>(item_capacity(n, nnz));
    L.stats = c.take<unsigned long long>(16);
    return L;
}

}  // namespace

size_t count_ws_bytes(int32_t n, int64_t nnz) {
    Carver c(nullptr, 0);
    carve_count(c, n, nnz);
    return c.used();
}

int ilog2_host(int v) {
    int k = 0;
    while ((1 << (k + 1)) <= v) ++k;
    return k;
}

int count_run(int32_t n, int64_t nnz, const PartBufs &pb, const CountCfg &cfg, CountOut *out, void *ws,
              size_t ws_bytes, hipStream_t s) {
    Carver c(ws, ws_bytes);
    CountLayout L = carve_count(c, n, nnz);
    if (!c.fits()) return TC_ERR_WORKSPACE;
    DeviceInfo di;
    TC_TRY(device_info(&di));
    const int wave_log2 = ilog2_host(cfg.wave_slots);
    const int wg_log2 = ilog2_host(cfg.wg_slots);
    SchedCfg sc;
    sc.table = cfg.table;
    sc.force = cfg.force;
    sc.wave_ob_max = wave_log2 - 2;
    sc.wg_ob_max = wg_log2 - 2;
    sc.heur_wave_ob = cfg.wave_max_owner > 0 ? ilog2_host(cfg.wave_max_owner) : wave_log2 - 2;
    sc.chunk_work = cfg.chunk_work;

    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    if (cfg.timing) {
        for (auto &e : ev) TC_HIP_TRY(hipEventCreate(&e));
        TC_HIP_TRY(hipEventRecord(ev[0], s));
    }
    const int64_t nn = n > 0 ? n : 1;
    TC_HIP_TRY(hipMemsetAsync(L.cnt, 0, sizeof(int32_t) * 2 * nn, s));
    TC_HIP_TRY(hipMemsetAsync(L.work, 0, sizeof(unsigned long long) * 2 * nn, s));
    TC_HIP_TRY(hipMemsetAsync(L.bucket_items, 0, sizeof(int32_t) * (kBuckets + 1), s));
    TC_HIP_TRY(hipMemsetAsync(L.bucket_cur, 0, sizeof(int32_t) * kBuckets, s));
    TC_HIP_TRY(hipMemsetAsync(L.q, 0, sizeof(int32_t) * 64, s));
    TC_HIP_TRY(hipMemsetAsync(L.stats, 0, sizeof(unsigned long long) * 16, s));
    const unsigned gp = (unsigned)di.cus * 8;
    if (n > 0) {
        hipLaunchKernelGGL(k_own, dim3(gp), dim3(kThreads), 0, s, n, pb.e0x2, pb.rp0, pb.c0, pb.up0, pb.rp1, L.cnt,
                           L.work);
        TC_HIP_TRY(hipGetLastError());
        const unsigned gu = grid_for(2 * (int64_t)n, kThreads, (int64_t)di.cus * 4);
        hipLaunchKernelGGL((k_items<0>), dim3(gu), dim3(kThreads), 0, s, n, pb.rp0, pb.up0, pb.rp1, L.cnt, L.work,
                           sc, L.bucket_items, L.bucket_off, L.bucket_cur, L.items, L.stats);
        TC_HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_bucket_order, dim3(1), dim3(64), 0, s, L.bucket_items, sc, L.bucket_off, L.q);
        TC_HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL((k_items<1>), dim3(gu), dim3(kThreads), 0, s, n, pb.rp0, pb.up0, pb.rp1, L.cnt, L.work,
                           sc, L.bucket_items, L.bucket_off, L.bucket_cur, L.items, L.stats);
        TC_HIP_TRY(hipGetLastError());
    }
    if (cfg.timing) TC_HIP_TRY(hipEventRecord(ev[1], s));
    if (n > 0) {
        int lds_slots = 1 << wg_log2;
        if ((kIsectWaves << wave_log2) > lds_slots) lds_slots = kIsectWaves << wave_log2;
        const size_t lds_bytes = (size_t)lds_slots * sizeof(int32_t);
        TC_HIP_TRY(hipFuncSetAttribute((const void *)k_isect, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds_bytes));
        int per_cu = (int)((160 * 1024) / (lds_bytes + 1024));
        if (per_cu > 4) per_cu = 4;
        if (per_cu < 1) per_cu = 1;
        const unsigned gi = cfg.grid_blocks > 0 ? (unsigned)cfg.grid_blocks : (unsigned)(di.cus * per_cu);
        Graph g{pb.rp0, pb.c0, pb.up0, pb.rp1, pb.c1};
        hipLaunchKernelGGL(k_isect, dim3(gi), dim3(kIsectThreads), lds_bytes, s, g, L.items, L.q, wg_log2,
                           wave_log2, L.stats + 8);
        TC_HIP_TRY(hipGetLastError());
    }
    if (cfg.timing) TC_HIP_TRY(hipEventRecord(ev[2], s));
    unsigned long long h[16];
    TC_HIP_TRY(hipMemcpyAsync(h, L.stats, sizeof(h), hipMemcpyDeviceToHost, s));
    TC_HIP_TRY(hipStreamSynchronize(s));
    if (out) {
        out->T0 = h[8];
        out->T1 = h[9];
        out->units = (int64_t)h[0];
        out->probes = (int64_t)h[1];
        out->hashed = (int64_t)h[2];
        int64_t items = 0;
        for (int k = 0; k < TC_NUM_STRATEGIES; ++k) {
            out->strategy_items[k] = (int32_t)h[3 + k];
            items += (int64_t)h[3 + k];
        }
        out->items = items;
        if (cfg.timing) {
            TC_HIP_TRY(hipEventElapsedTime(&out->ms_bucket, ev[0], ev[1]));
            TC_HIP_TRY(hipEventElapsedTime(&out->ms_isect, ev[1], ev[2]));
        }
    }
    if (cfg.timing)
        for (auto &e : ev) (void)hipEventDestroy(e);
    return TC_OK;
}

}  // namespace tc
