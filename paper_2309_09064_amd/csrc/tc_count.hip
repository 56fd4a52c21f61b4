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
#include <stdio.h>
#include <stdlib.h>

#include <mutex>

#include "tc_internal.hpp"

namespace tc {
namespace {

constexpr int kRun = 8;                 // CSR entries per thread in row passes (load_run8)
constexpr int kThreads = 256;
constexpr int kIsectThreads = 1024;     // 16 wavefronts per persistent block
constexpr int kIsectWaves = kIsectThreads / kWave;
constexpr int kBuckets = 2 * 32 * 32;
constexpr int kOwnRowsMax = 512;           // rows a tile may span and still count in LDS
constexpr int kMinPartnersPerItem = 8;     // wavefront items
constexpr int kMinPartnersPerWgItem = 4096; // workgroup items
constexpr int kWgItemWaves = 4 * kIsectWaves; // a workgroup item holds this many wavefront items of work
constexpr int32_t kEmpty = -1;
constexpr int32_t kNoKey = -2;   // window padding: never stored, never equal to kEmpty
// By default a workgroup table (2^wg_log2 slots) holds at most 2^(wg_log2 -
// kWgCapShift) owner elements (load 1/4: fewer slices than at 1/8, still
// short probe sequences; measured faster on Kronecker scale 22 and Chung-Lu
// 2^20); longer owner lists are cut into value-range slices.
constexpr int kWgCapShift = 2;
// Claim counters of the intersection pass: kClaimStreams streams (one per
// XCD), each with a wavefront-item and a lane-group counter in its own
// 128-byte line after the first kQueueInts ints of the queue block.
constexpr int kClaimStreams = 8;
constexpr int kQueueInts = 64;
constexpr int kClaimStride = 32;
constexpr int kQueueBlockInts = kQueueInts + kClaimStreams * kClaimStride;
constexpr int kLaneMergeOb = 4;            // merge items with owner lists below 32: one lane each
constexpr int kLanePartners = 32;          // row positions per lane item (owner classes 0-2)

// Row positions per lane item of owner class ob.  A merging lane walks both
// lists of each of its partners in turn, up to 2^(ob+2) steps per partner,
// and its wavefront holds the group of 64 items until the slowest lane is
// done, so the partner count halves per class above 2: every lane's walk
// stays within about 512 steps.  Per-element cost profiles cannot see such
// a walk's latency, only its share of the wavefront's time.  The register
// and LDS forms of the counting modes (`batched`) cost a few load latencies
// per batch of partners whatever the class, so their items all take
// kLanePartners positions.
__host__ __device__ constexpr int lane_partners(int ob, bool batched = false) {
    return ob <= 2 || batched ? kLanePartners : kLanePartners >> (ob - 2);
}

struct Item {
    int32_t owner;
    int32_t code;   // kind | strategy << 1 | bucket << 3 | owner slice << 14
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
    int32_t wg_ob_max;     // largest owner-size class the workgroup table holds whole
    int32_t wg_cap_log2;   // log2 of the owner elements one workgroup table holds
    int32_t wg_slicing;    // longer owner lists are sliced (else they are searched; also for half slices)
    int32_t heur_wave_ob;  // heuristic: wavefront table up to this class
    int32_t heur_merge_ob; // heuristic: lane merge up to this class (-1: never)
    int32_t chunk_work;    // probe elements per wavefront item
    int32_t lane_batched;  // lane items take the register / LDS forms (counting modes, 2048-slot wavefront tables)
};

// Strategy of a bucket.  Feasibility depends only on the owner-size class
// ob = floor(log2 |owner list|): a table of 2^k slots takes classes
// ob <= k - 2, i.e. lists shorter than half the table.  The workgroup hash
// takes any owner while slicing is on: a list longer than half its table is
// cut into value-range slices that each fill at most half of it, one work
// item per slice.
// A table entry holds the strategy in bits 0-1 and, in bit 2, the tile
// choice of the workgroup hash: slices of half the usual size (more items,
// a quarter-full table's pending probes halved).  Other values mean binary
// search.
constexpr int32_t kTileHalf = 4;
__device__ __forceinline__ int strategy_for(const SchedCfg &c, int b) {
    const int ob = (b >> 5) & 31;
    const bool wg_ok = ob <= c.wg_ob_max || c.wg_slicing;
    int s;
    if (c.force >= 0) s = c.force;
    else if (c.table) s = (uint32_t)c.table[b] < 8u ? (c.table[b] & 3) : TC_STRAT_BSEARCH;
    else if (ob <= c.heur_merge_ob) s = TC_STRAT_MERGE;
    else s = ob <= c.heur_wave_ob ? TC_STRAT_WAVE_HASH : (wg_ok ? TC_STRAT_WG_HASH : TC_STRAT_BSEARCH);
    if (s == TC_STRAT_WAVE_HASH && ob > c.wave_ob_max) s = wg_ok ? TC_STRAT_WG_HASH : TC_STRAT_BSEARCH;
    if (s == TC_STRAT_WG_HASH && !wg_ok) s = TC_STRAT_BSEARCH;
    if (s < 0 || s >= TC_NUM_STRATEGIES) s = TC_STRAT_BSEARCH;
    return s;
}

constexpr int kHalfShift = 14;           // item code bit: the item's owner is cut into half-size slices
constexpr int kSliceShift = 15;          // slice index in the item code's top 17 bits
constexpr int kMaxSlicesLog2 = 32 - kSliceShift;

// Half-size workgroup slices for bucket b: asked for by its table entry,
// the bucket takes the workgroup hash, and its owner lists are long enough
// to be cut finer (at least half a slice).
__device__ __forceinline__ int tile_half(const SchedCfg &c, int b, int s) {
    if (c.force >= 0 || !c.table || s != TC_STRAT_WG_HASH || !c.wg_slicing) return 0;
    const int32_t v = c.table[b];
    return (uint32_t)v < 8u && (v & kTileHalf) && ((b >> 5) & 31) >= c.wg_cap_log2 - 1 ? 1 : 0;
}

// Slices of an owner list of sx elements under the workgroup hash.
__device__ __forceinline__ int32_t owner_slices(int32_t sx, int cap_log2) {
    return (int32_t)(((int64_t)sx + (1 << cap_log2) - 1) >> cap_log2);
}

// ---------------------------------------------------------------- ownership

// Per owner and kind: number of owned partners and their total list length.
// Per c0 entry (x, y) and kind k it also writes the partner record the
// intersection pass needs: y's kind-k list {offset, size} where x owns the
// edge for kind k, {0, 0} where it does not (an owned partner's list is never
// empty).  The pass then reads 8 coalesced bytes per position and kind
// instead of gathering y's 16-byte vertex record, a 128-byte line per owned
// partner: this pass gathers those records anyway.
__global__ __launch_bounds__(kThreads) void k_own(int32_t n, const int64_t *__restrict__ e0x2p,
                                                   const int32_t *__restrict__ rp0,
                                                   const int32_t *__restrict__ c0, const int32_t *__restrict__ up0,
                                                   const int32_t *__restrict__ rp1, const int4 *__restrict__ vrec,
                                                   int32_t *__restrict__ cnt, unsigned long long *__restrict__ work,
                                                   int2 *__restrict__ prec0, int2 *__restrict__ prec1,
                                                   const int32_t *__restrict__ tlo, const int32_t *__restrict__ thi) {
    __shared__ int32_t acc_n[2][kOwnRowsMax];
    __shared__ unsigned long long acc_w[2][kOwnRowsMax];
    constexpr int kHalf = kWave * kRun / 2;   // entries in half a wavefront's span
    __shared__ int4 stg[kThreads / kWave][kHalf / 2];   // per wavefront: one kind's records of half its span
    const int64_t e0x2 = *e0x2p;
    constexpr int64_t kTile = (int64_t)kThreads * kRun;
    static_assert(kTile == kTileEntries, "a tile of this pass is a tile of the tile table");
    for (int64_t t0 = (int64_t)blockIdx.x * kTile; t0 < e0x2; t0 += (int64_t)gridDim.x * kTile) {
        const int64_t r_lo = tlo[t0 / kTile], r_hi = thi[t0 / kTile];
        const int64_t nr = r_hi - r_lo + 1;
        const bool local = nr <= kOwnRowsMax;   // count in LDS, flush once per row
        if (local)
            for (int64_t i = threadIdx.x; i < nr; i += kThreads) {
                acc_n[0][i] = acc_n[1][i] = 0;
                acc_w[0][i] = acc_w[1][i] = 0;
            }
        __syncthreads();
        const int64_t e0 = t0 + (int64_t)threadIdx.x * kRun;
        // the run's partner records and which of them the row's vertex owns
        // (bit k per kind): the stores below select from them, so that no
        // second copy of the records stays live through the row walk
        int4 ry[kRun];
        uint32_t own0 = 0, own1 = 0;
        if (e0 < e0x2) {
            const int64_t e1 = e0 + kRun < e0x2 ? e0 + kRun : e0x2;
            int64_t x = row_of(rp0, r_lo, r_hi, e0);
            int64_t xe = rp0[x + 1];
            int32_t s0x = up0[x], s1x = rp1[x + 1] - rp1[x];
            int32_t n0 = 0, n1 = 0;
            unsigned long long w0 = 0, w1 = 0;
            auto flush = [&]() {
                if (local) {
                    const int64_t i = x - r_lo;
                    if (n0) { atomicAdd(&acc_n[0][i], n0); atomicAdd(&acc_w[0][i], w0); }
                    if (n1) { atomicAdd(&acc_n[1][i], n1); atomicAdd(&acc_w[1][i], w1); }
                } else {
                    if (n0) { atomicAdd(&cnt[2 * x], n0); atomicAdd(&work[2 * x], w0); }
                    if (n1) { atomicAdd(&cnt[2 * x + 1], n1); atomicAdd(&work[2 * x + 1], w1); }
                }
                n0 = n1 = 0;
                w0 = w1 = 0;
            };
            // the run's partners and their list sizes, issued before the
            // row walk (two memory latencies per thread, not per entry)
            int32_t y[kRun];
            load_run8(c0, e0, e1, y);
#pragma unroll
            for (int k = 0; k < kRun; ++k) ry[k] = e0 + k < e1 ? vrec[y[k]] : make_int4(0, 0, 0, 0);
#pragma unroll
            for (int k = 0; k < kRun; ++k) {
                const int64_t e = e0 + k;
                if (e >= e1) break;
                while (e >= xe) {
                    flush();
                    ++x;
                    xe = rp0[x + 1];
                    s0x = up0[x];
                    s1x = rp1[x + 1] - rp1[x];
                }
                const bool o0 = owns(s0x, ry[k].y, (int32_t)x, y[k]);
                const bool o1 = owns(s1x, ry[k].w, (int32_t)x, y[k]);
                if (o0) { ++n0; w0 += (unsigned)ry[k].y; }
                if (o1) { ++n1; w1 += (unsigned)ry[k].w; }
                own0 |= (uint32_t)o0 << k;
                own1 |= (uint32_t)o1 << k;
            }
            flush();
        } else {
#pragma unroll
            for (int k = 0; k < kRun; ++k) ry[k] = make_int4(0, 0, 0, 0);
        }
        // the records leave through LDS, half a wavefront's span at a time,
        // so that every store instruction writes 1 KB of consecutive entries
        // (a thread's own run is 64 bytes: its direct stores would touch a
        // 16-byte piece of every 64 bytes per instruction)
        {
            const int w = (int)threadIdx.x / kWave, l = lane_id();
            const int64_t wb = t0 + (int64_t)w * (2 * kHalf);   // first entry of the wavefront's span
            if (wb < e0x2) {                                   // uniform in the wavefront
                const bool full = wb + 2 * kHalf <= e0x2;
                // kind 0 stores {rp0, |N0+|} of the owned partners, kind 1
                // {rp1, |N1|}; {0, 0} elsewhere
                auto rec = [&](int kind, int k) -> int2 {
                    const bool o = (((kind ? own1 : own0) >> k) & 1u) != 0;
                    return o ? (kind ? make_int2(ry[k].z, ry[k].w) : make_int2(ry[k].x, ry[k].y)) : make_int2(0, 0);
                };
                auto put = [&](int kind, int2 *dst) {
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        if ((l >> 5) == h) {
#pragma unroll
                            for (int k = 0; k < kRun; k += 2) {
                                const int2 a = rec(kind, k), b = rec(kind, k + 1);
                                stg[w][(l & 31) * (kRun / 2) + k / 2] = make_int4(a.x, a.y, b.x, b.y);
                            }
                        }
                        wave_lds_sync();
#pragma unroll
                        for (int j = 0; j < kHalf / 2 / kWave; ++j) {
                            const int q = l + kWave * j;                // 16-byte piece of the half span
                            const int4 v = stg[w][q];
                            const int64_t i = (int64_t)h * kHalf + 2 * q;   // entry in the wavefront's span
                            if (full) {
                                *reinterpret_cast<int4 *>(dst + i) = v;
                            } else {
                                if (wb + i < e0x2) dst[i] = make_int2(v.x, v.y);
                                if (wb + i + 1 < e0x2) dst[i + 1] = make_int2(v.z, v.w);
                            }
                        }
                        wave_lds_sync();   // the region is rewritten next
                    }
                };
                put(0, prec0 + wb);
                put(1, prec1 + wb);
            }
        }
        __syncthreads();
        if (local) {
            for (int64_t i = threadIdx.x; i < nr; i += kThreads) {
                const int64_t r = r_lo + i;
                const bool edge = r == r_lo || r == r_hi;
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    const int32_t c = acc_n[k][i];
                    if (edge) {
                        if (c) { atomicAdd(&cnt[2 * r + k], c); atomicAdd(&work[2 * r + k], acc_w[k][i]); }
                    } else {
                        cnt[2 * r + k] = c;
                        work[2 * r + k] = acc_w[k][i];
                    }
                }
            }
        }
        __syncthreads();   // LDS is reused by the next tile
    }
}

// Items per unit.  The count pass (kFill = 0) histograms items per bucket;
// the fill pass writes them.  A block handles 4096 units: LDS atomics order
// the block's items inside each bucket, then one global atomic per (block,
// bucket) reserves the block's range.  Stats: [0] units, [1] probes,
// [2] hashed, [3..6] items per strategy.
constexpr int kItemThreads = 1024;
constexpr int kUnitsPerThread = 4;

template <int kFill>
__global__ __launch_bounds__(kItemThreads) void k_items(int32_t n, const int32_t *__restrict__ rp0,
                                                         const int32_t *__restrict__ up0,
                                                         const int32_t *__restrict__ rp1,
                                                         const int32_t *__restrict__ cnt,
                                                         const unsigned long long *__restrict__ work, SchedCfg sc,
                                                         int32_t *__restrict__ bucket_items,
                                                         const int32_t *__restrict__ bucket_off,
                                                         int32_t *__restrict__ bucket_cur, Item *__restrict__ items,
                                                         unsigned long long *__restrict__ stats,
                                                         unsigned long long *__restrict__ prof) {
    __shared__ int32_t hist[kBuckets];
    __shared__ int32_t bbase[kFill ? kBuckets : 1];
    for (int i = threadIdx.x; i < kBuckets; i += kItemThreads) hist[i] = 0;
    __syncthreads();
    const int64_t total = 2 * (int64_t)n;
    const int64_t u0 = ((int64_t)blockIdx.x * kItemThreads + threadIdx.x) * kUnitsPerThread;
    int bk[kUnitsPerThread], loc[kUnitsPerThread], st[kUnitsPerThread];
    int32_t nchs[kUnitsPerThread], nsls[kUnitsPerThread];
    unsigned long long units = 0, probes = 0, hashed = 0, ps0 = 0, ps1 = 0, ps2 = 0, ps3 = 0;
#pragma unroll
    for (int k = 0; k < kUnitsPerThread; ++k) {
        const int64_t u = u0 + k;
        bk[k] = -1;
        nchs[k] = 0;
        nsls[k] = 1;
        loc[k] = 0;
        st[k] = 0;
        const int32_t c = u < total ? cnt[u] : 0;
        if (c == 0) continue;
        const int32_t x = (int32_t)(u >> 1);
        const int kind = (int)(u & 1);
        const unsigned long long w = work[u];
        const int32_t sx = kind == 0 ? up0[x] : rp1[x + 1] - rp1[x];
        const int b = bucket_of(kind, sx, (int64_t)w, c);
        const int s = strategy_for(sc, b);
        const int64_t target = (int64_t)sc.chunk_work * (s == TC_STRAT_WG_HASH ? kWgItemWaves : 1);
        const int32_t jb = rp0[x], je = rp0[x + 1];
        const int32_t minp = s == TC_STRAT_WG_HASH ? kMinPartnersPerWgItem : kMinPartnersPerItem;
        // a sliced owner: each slice streams about w / nsl elements; the
        // items of a unit stay at most slices + partner chunks in number
        const int32_t nsl = s == TC_STRAT_WG_HASH ? owner_slices(sx, sc.wg_cap_log2 - tile_half(sc, b, s)) : 1;
        int64_t nch = ((int64_t)w / nsl + target - 1) / target;
        int64_t cap = (je - jb + minp - 1) / minp;
        if (nsl > 1) cap = (cap + nsl - 1) / nsl;
        if (nch > cap) nch = cap;
        if (s == TC_STRAT_MERGE && ((b >> 5) & 31) <= kLaneMergeOb) {   // one lane walks an item's partners
            const int lp = lane_partners((b >> 5) & 31, sc.lane_batched != 0);
            nch = (je - jb + lp - 1) / lp;
        }
        if (nch < 1) nch = 1;
        bk[k] = b;
        st[k] = s;
        nchs[k] = (int32_t)nch;
        nsls[k] = nsl;
        loc[k] = atomicAdd(&hist[b], (int32_t)nch * nsl);
        if (!kFill && prof)   // profile: the bucket's elements (partners streamed + owner list)
            atomicAdd(&prof[(b * TC_NUM_STRATEGIES + s) * 3 + 1], w + (unsigned long long)sx);
        if (!kFill) {
            const unsigned long long nc = (unsigned long long)nch * (unsigned long long)nsl;
            ++units;
            probes += w;
            hashed += (unsigned long long)sx * nc;
            ps0 += s == 0 ? nc : 0;
            ps1 += s == 1 ? nc : 0;
            ps2 += s == 2 ? nc : 0;
            ps3 += s == 3 ? nc : 0;
        }
    }
    __syncthreads();
    if (!kFill) {
        for (int i = threadIdx.x; i < kBuckets; i += kItemThreads)
            if (hist[i]) atomicAdd(&bucket_items[i], hist[i]);
        __shared__ unsigned long long red[kItemThreads / kWave][7];
        const unsigned long long v[7] = {wave_sum(units), wave_sum(probes), wave_sum(hashed), wave_sum(ps0),
                                         wave_sum(ps1), wave_sum(ps2), wave_sum(ps3)};
        if (lane_id() == 0)
            for (int k = 0; k < 7; ++k) red[threadIdx.x / kWave][k] = v[k];
        __syncthreads();
        if (threadIdx.x < 7) {
            unsigned long long a = 0;
            for (int i = 0; i < kItemThreads / kWave; ++i) a += red[i][threadIdx.x];
            if (a) atomicAdd(&stats[threadIdx.x], a);
        }
        return;
    }
    for (int i = threadIdx.x; i < kBuckets; i += kItemThreads)
        bbase[i] = hist[i] ? bucket_off[i] + atomicAdd(&bucket_cur[i], hist[i]) : 0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kUnitsPerThread; ++k) {
        if (bk[k] < 0) continue;
        const int64_t u = u0 + k;
        const int32_t x = (int32_t)(u >> 1);
        const int32_t jb = rp0[x], je = rp0[x + 1];
        const int64_t len = je - jb;
        const int32_t pos = bbase[bk[k]] + loc[k];
        const int32_t code =
            (int32_t)(u & 1) | (st[k] << 1) | (bk[k] << 3) | (tile_half(sc, bk[k], st[k]) << kHalfShift);
        for (int32_t si = 0; si < nsls[k]; ++si)
            for (int32_t c = 0; c < nchs[k]; ++c) {
                Item it;
                it.owner = x;
                it.code = (int32_t)((uint32_t)code | ((uint32_t)si << kSliceShift));
                it.jb = jb + (int32_t)(len * c / nchs[k]);
                it.je = jb + (int32_t)(len * (c + 1) / nchs[k]);
                items[pos + si * nchs[k] + c] = it;
            }
    }
}

// Queue layout: workgroup-table buckets first, then the rest; inside each
// queue larger owners first.  One block: place every bucket's item count at
// its queue position, exclusive-scan the 4096 positions, read offsets back.
// q[2] = workgroup items, q[3] = all items.  (q[0] is the intersection
// pass's workgroup-item counter; its stream counters follow the first
// kQueueInts ints.)
// Three sections: workgroup-table items, then wavefront items, then the
// lane items (merge strategy with owner lists below 2^(kLaneMergeOb + 1)),
// which wavefronts take 64 at a time, one per lane.
__device__ __forceinline__ int queue_pos(const SchedCfg &sc, int b) {
    const int ob = (b >> 5) & 31, pb = b & 31, kind = b >> 10;
    const int s = strategy_for(sc, b);
    const int section = s == TC_STRAT_WG_HASH ? 0 : (s == TC_STRAT_MERGE && ob <= kLaneMergeOb ? 2 : 1);
    return section * kBuckets + ((31 - ob) * 32 + (31 - pb)) * 2 + kind;
}

__global__ __launch_bounds__(1024) void k_bucket_order(const int32_t *__restrict__ bucket_items, SchedCfg sc,
                                                        int32_t *__restrict__ bucket_off, int32_t *__restrict__ q) {
    constexpr int kPerThread = 3 * kBuckets / 1024;
    __shared__ int32_t A[3 * kBuckets];
    __shared__ int32_t wtot[16];
    const int t = threadIdx.x;
    for (int i = t; i < 3 * kBuckets; i += 1024) A[i] = 0;
    __syncthreads();
    for (int b = t; b < kBuckets; b += 1024) A[queue_pos(sc, b)] = bucket_items[b];
    __syncthreads();
    int32_t v[kPerThread];
    int32_t sum = 0;
#pragma unroll
    for (int j = 0; j < kPerThread; ++j) { v[j] = A[kPerThread * t + j]; sum += v[j]; }
    const int32_t inc = wave_incl_scan(sum);
    if (lane_id() == kWave - 1) wtot[t / kWave] = inc;
    __syncthreads();
    int32_t run = inc - sum;
    for (int i = 0; i < t / kWave; ++i) run += wtot[i];
#pragma unroll
    for (int j = 0; j < kPerThread; ++j) { A[kPerThread * t + j] = run; run += v[j]; }
    if (t == 1023) q[3] = run;
    __syncthreads();
    for (int b = t; b < kBuckets; b += 1024) bucket_off[b] = A[queue_pos(sc, b)];
    if (t == 0) {
        q[2] = A[kBuckets];       // first wavefront item
        q[4] = A[2 * kBuckets];   // first lane item
    }
}

// ---------------------------------------------------------------- probes

// LDS hash table of 2-slot buckets.  A key's home bucket is a
// multiplicative hash of the id; a lookup reads the bucket (one 8-byte read)
// and walks on only while the bucket is full without the key.  The bucket
// width is a measured balance: 16-byte buckets saturate the LDS address unit
// (a wavefront's 64 random reads fall into 8 bank groups), while single
// slots send about one key in eight past its home slot at load 1/8 against
// about one in forty here.
// Tables loaded above 1/16 take two candidate buckets per key (balanced
// allocation): a key goes to the emptier of the two, and only when both are
// full to linear probing from the first.  A lookup reads both and walks only
// when both are full without the key: at load 1/4 one lookup in 800 instead
// of one in ten.  Every window of lookups pays the slowest lane's walks, so
// this trades a second read per key for the walks; below 1/16 the walks are
// rare enough that one read is cheaper.
// Tables are sized so at most half the slots are used (a quarter under the
// heuristic schedule, 1/32 where LDS allows).
struct HashTab {
    int32_t *tab;
    uint32_t mask;    // buckets - 1 (2 slots a bucket)
    int off, bits;    // home bucket: bits [off, off + bits) of the 24-bit product, bits = log2(buckets)
    int two;          // two candidate buckets per key
    uint32_t *cnt;    // per-vertex / per-edge counts: a hit counter per slot, else unused
};

constexpr int kTwoChoiceLoad = 16;   // two candidates above a load of 1 / kTwoChoiceLoad

// keys: how many keys the table will hold
__device__ __forceinline__ HashTab make_tab(int32_t *tab, int lg_slots, int32_t keys, uint32_t *cnt = nullptr) {
    HashTab t;
    t.tab = tab;
    t.cnt = cnt;
    t.mask = (1u << (lg_slots - 1)) - 1;
    t.bits = lg_slots - 1;
    t.off = 24 - t.bits;
    t.two = __builtin_amdgcn_readfirstlane((int64_t)keys * kTwoChoiceLoad > ((int64_t)1 << lg_slots) ? 1 : 0);
    return t;
}

// Fibonacci hashing on a 2^24 ring: the product
// (v * floor(2^24 / golden ratio)) mod 2^24; the home bucket is its top
// log2(buckets) bits, the second candidate its low ones.  The 24-bit
// multiply, the field extract and the mask all issue at full rate, where a
// 32-bit multiply takes four passes; ids of 2^24 and above share the hash of
// their low 24 bits, which only lengthens probe sequences.
__device__ __forceinline__ uint32_t hash_product(int32_t v) { return (uint32_t)__umul24((uint32_t)v, 0x9E3779u); }
__device__ __forceinline__ uint32_t home_of(const HashTab &t, uint32_t p) {
    return __builtin_amdgcn_ubfe(p, (uint32_t)t.off, (uint32_t)t.bits);
}
__device__ __forceinline__ uint32_t home_slot(const HashTab &t, int32_t v) { return home_of(t, hash_product(v)); }

__device__ __forceinline__ int bucket_used(const int32_t *tab, uint32_t b) {
    const uint64_t w = __hip_atomic_load(reinterpret_cast<const uint64_t *>(tab + 2 * b), __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_WORKGROUP);
    return ((int32_t)(uint32_t)w != kEmpty ? 1 : 0) + ((int32_t)(uint32_t)(w >> 32) != kEmpty ? 1 : 0);
}

// Slots of a bucket fill in order: a bucket whose second slot is empty ends
// every probe sequence through it.  With two candidates the emptier one is
// tried first (the counts are a hint: the compare-and-swaps decide), then
// the other; a key that finds both full probes on from the home bucket.
__device__ __forceinline__ void hash_insert(const HashTab &t, int32_t v) {
    const uint32_t p = hash_product(v);
    uint32_t b = home_of(t, p);
    if (t.two) {
        const uint32_t c = p & t.mask;
        const bool swap = bucket_used(t.tab, c) < bucket_used(t.tab, b);
        const uint32_t f = swap ? c : b, g = swap ? b : c;
        if (atomicCAS(&t.tab[2 * f], kEmpty, v) == kEmpty) return;
        if (atomicCAS(&t.tab[2 * f + 1], kEmpty, v) == kEmpty) return;
        if (atomicCAS(&t.tab[2 * g], kEmpty, v) == kEmpty) return;
        if (atomicCAS(&t.tab[2 * g + 1], kEmpty, v) == kEmpty) return;
    } else {
        if (atomicCAS(&t.tab[2 * b], kEmpty, v) == kEmpty) return;
        if (atomicCAS(&t.tab[2 * b + 1], kEmpty, v) == kEmpty) return;
    }
    for (;;) {
        b = (b + 1) & t.mask;
        if (atomicCAS(&t.tab[2 * b], kEmpty, v) == kEmpty) return;
        if (atomicCAS(&t.tab[2 * b + 1], kEmpty, v) == kEmpty) return;
    }
}

// Membership of up to kPer keys: ids >= 0, or kNoKey for window padding,
// which matches no slot (never kEmpty, which would match empty ones).  Every
// key's candidate buckets are read once, unconditionally and interleaved; a
// key whose candidates are all full without it (rare at the tables' load)
// then follows its probe sequence from the home bucket, one pending key at a
// time per lane.  Keeping the common case free of per-key predication is
// what bounds the instruction count: the slowest of a wavefront's keys no
// longer sets the work of all of them.
// With kMask the result is the mask of keys found (bit u for key u) instead
// of their number; with kSlots as well, slot[u] receives the slot of each key
// found (per-vertex / per-edge counts credit the slot's counter).
template <int kPer, bool kMask = false, bool kSlots = false>
__device__ __forceinline__ uint32_t hash_probe(const HashTab &t, const int32_t (&v)[kPer], int32_t *slot) {
    uint32_t hits = 0;
    uint32_t pend = 0;   // keys whose candidates are full (second slot used: keys are >= 0) without them
    if (t.two) {
        uint32_t b[kPer], c[kPer];
        int2 q[kPer], r[kPer];
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const uint32_t p = hash_product(v[u]);
            b[u] = home_of(t, p);
            c[u] = p & t.mask;
        }
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            q[u] = *reinterpret_cast<const int2 *>(&t.tab[2 * b[u]]);
            r[u] = *reinterpret_cast<const int2 *>(&t.tab[2 * c[u]]);
        }
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int32_t x = v[u];
            const bool m0 = q[u].x == x, m1 = q[u].y == x, m2 = r[u].x == x, m3 = r[u].y == x;
            const bool m = m0 | m1 | m2 | m3;
            if constexpr (kMask) hits |= m ? (1u << u) : 0u;
            else hits += m ? 1u : 0u;
            if constexpr (kSlots)
                slot[u] = (int32_t)((m0 | m1) ? 2 * b[u] + (m0 ? 0 : 1) : 2 * c[u] + (m2 ? 0 : 1));
            pend |= (!m & (q[u].y >= 0) & (r[u].y >= 0)) ? (1u << u) : 0u;
        }
    } else {
        uint32_t b[kPer];
        int2 q[kPer];
#pragma unroll
        for (int u = 0; u < kPer; ++u) b[u] = home_slot(t, v[u]);
#pragma unroll
        for (int u = 0; u < kPer; ++u) q[u] = *reinterpret_cast<const int2 *>(&t.tab[2 * b[u]]);
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int32_t x = v[u];
            const bool m0 = q[u].x == x, m1 = q[u].y == x;
            if constexpr (kMask) hits |= (m0 | m1) ? (1u << u) : 0u;
            else hits += (m0 | m1) ? 1u : 0u;
            if constexpr (kSlots) slot[u] = (int32_t)(2 * b[u] + (m0 ? 0 : 1));
            // padding keys walk on too, rarely, and never match
            pend |= (!(m0 | m1) & (q[u].y >= 0)) ? (1u << u) : 0u;
        }
    }
    if (__ballot(pend != 0) == 0) return hits;
    while (pend) {
        const int u = __builtin_ctz(pend);
        pend &= pend - 1;
        int32_t x = v[0];
#pragma unroll
        for (int j = 1; j < kPer; ++j) x = u == j ? v[j] : x;
        uint32_t bb = home_slot(t, x);   // recomputed: cheaper than a second select chain
        for (;;) {
            bb = (bb + 1) & t.mask;
            const int2 r = *reinterpret_cast<const int2 *>(&t.tab[2 * bb]);
            if (r.x == x || r.y == x) {
                if constexpr (kMask) hits |= 1u << u;
                else ++hits;
                if constexpr (kSlots) {
#pragma unroll
                    for (int j = 0; j < kPer; ++j)
                        if (j == u) slot[j] = (int32_t)(2 * bb + (r.x == x ? 0 : 1));
                }
                break;
            }
            if (r.y == kEmpty) break;
        }
    }
    return hits;
}

template <int kPer, bool kMask = false>
__device__ __forceinline__ uint32_t hash_count(const HashTab &t, const int32_t (&v)[kPer]) {
    return hash_probe<kPer, kMask, false>(t, v, nullptr);
}

template <int kPer>
__device__ __forceinline__ uint32_t hash_find(const HashTab &t, const int32_t (&v)[kPer], int32_t (&e)[kPer]) {
    return hash_probe<kPer, true, true>(t, v, e);
}

// Lookups of the kPer keys of a window in two interleaved groups of four
// (eight keys in flight would need twice the registers).
template <class Group>
__device__ __forceinline__ uint32_t in_fours(const int32_t (&v)[8], Group grp) {
    const int32_t a[4] = {v[0], v[1], v[2], v[3]};
    const int32_t b[4] = {v[4], v[5], v[6], v[7]};
    return grp(a) + grp(b);
}

// Membership of up to kPer keys in a sorted global list by branch-free binary
// search, the searches interleaved.  kMask as for hash_count.
template <int kPer, bool kMask = false>
__device__ __forceinline__ uint32_t search_count(const int32_t *a, int32_t len, const int32_t (&v)[kPer]) {
    int32_t base[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) base[u] = 0;
    int32_t n = len;
    while (n > 1) {
        const int32_t half = n >> 1;
#pragma unroll
        for (int u = 0; u < kPer; ++u) base[u] = a[base[u] + half] < v[u] ? base[u] + half : base[u];
        n -= half;
    }
    // base is now the last index whose element is below the key (or 0);
    // the lower bound is one further when that element is below the key
    uint32_t hits = 0;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        if (v[u] < 0 || len <= 0) continue;
        const int32_t lb = base[u] + (a[base[u]] < v[u] ? 1 : 0);
        if constexpr (kMask) hits |= (lb < len && a[lb] == v[u]) ? (1u << u) : 0u;
        else hits += (lb < len && a[lb] == v[u]) ? 1u : 0u;
    }
    return hits;
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

// Line samples of a list array: smp[j] = a[32 j + off], the first element of
// every 128-byte line (off: the first index at a line start).  A search in a
// list first narrows to one line through the samples (a small array that
// stays in cache), then searches that line: about one line of the list is
// read instead of one per halving step, and that line is the first one the
// stream then reads anyway.
constexpr int kSmpShift = 5;
__host__ __device__ constexpr int64_t samples_of(int64_t entries) { return (entries >> kSmpShift) + 2; }

// First index i in [b, b + len) with a[i] >= v, else b + len (a sorted there).
__device__ __forceinline__ int32_t sampled_lower(const int32_t *a, const int32_t *smp, int32_t off, int32_t b,
                                                 int32_t len, int32_t v) {
    const int32_t e = b + len;
    // samples whose positions 32 j + off lie in [b, e): j0 .. j1
    const int32_t j0 = b > off ? (b - off + 31) >> kSmpShift : 0;
    const int32_t j1 = e - 1 >= off ? (e - 1 - off) >> kSmpShift : -1;
    if (j0 > j1) return b + lower_idx(a + b, len, v);
    const int32_t j = j0 + lower_idx(smp + j0, j1 - j0 + 1, v);   // first sample >= v (j1 + 1: none)
    // the answer lies after the sample before j (or from b) and at most at
    // sample j's position (or the list's end)
    const int32_t ps = j == j0 ? b : ((j - 1) << kSmpShift) + off + 1;
    const int32_t pe = j <= j1 ? (j << kSmpShift) + off : e;
    return ps + lower_idx(a + ps, pe - ps, v);
}

// search_count that also returns, for each key found, its index in a.
template <int kPer>
__device__ __forceinline__ uint32_t search_find(const int32_t *a, int32_t len, const int32_t (&v)[kPer],
                                                int32_t (&e)[kPer]) {
    uint32_t mask = 0;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        e[u] = 0;
        if (v[u] < 0 || len <= 0) continue;
        const int32_t lb = lower_idx(a, len, v[u]);
        if (lb < len && a[lb] == v[u]) {
            mask |= 1u << u;
            e[u] = lb;
        }
    }
    return mask;
}

// Wave-parallel merge of sorted a (owner, length la) and b (partner, lb):
// lane l merges its 1/64 slice of a with the matching value range of b.
// `on(value, i, j)` sees every common value with its indices in a and b.
template <class OnHit>
__device__ __forceinline__ uint32_t merge_count(const int32_t *a, int32_t la, const int32_t *b, int32_t lb, OnHit on) {
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
        else { on(x, i, j); ++hits; ++i; ++j; }
    }
    return hits;
}

struct Graph {
    const int32_t *rp0, *c0, *up0, *rp1, *c1;
    const int4 *vrec;   // per vertex {rp0, |N0+|, rp1, |N1|}
    const int2 *prec0, *prec1;   // per c0 entry, kind 0 / 1: the partner's list {offset, size} if owned, else {0, 0}
    const int32_t *pos0, *pos1;   // per-edge counts: input entry of every c0 / c1 entry
    int wide;           // the list arrays reach 2^30 entries: element byte offsets need 64 bits
    const int32_t *s0, *s1;   // line samples of c0 / c1 (sliced searches; NULL when nothing is sliced)
    int32_t so0, so1;         // index of the first line start in c0 / c1
};

// Elements per lane per window step, and the per-wavefront LDS scratch used
// to flatten a batch of partner lists: 64 * kPer marker bytes (window offset
// o lives at byte (o % 64) * kPer + o / 64, so a lane reads its kPer window
// slots with one load) and 64 partner records {start in the batch, list
// offset}; with records (per-vertex and per-edge counts, the cover-edge
// count) 128 more ints hold a tag per record (the partner vertex, or the
// input entry of the edge owner-partner) and a hit counter per record.
constexpr int kPer = 8;
constexpr int kScratchInts = 16 * kPer + 128;
constexpr int kScratchIdsInts = kScratchInts + 128;

// What the intersection pass produces besides T0 and T1: per-graph counts of
// a batch, per-vertex triangle counts, or per-edge supports.  kModeCover is
// the cover-edge count (Algorithm 3) over the full-row view: every common
// neighbour w of a horizontal edge xy is tested by its level.
enum { kModePlain = 0, kModeBatch = 1, kModeVertex = 2, kModeEdge = 3, kModeCover = 4 };

// Every hit is one triangle {x, y, w}: owner x, partner y, common neighbour w
// (each triangle is found exactly once, through its one cover edge xy).
struct Sink {
    const int32_t *gid;            // batch: graph of every vertex
    unsigned long long *counts;    // batch: one counter per graph
    unsigned long long *tv;        // vertex: triangles through every vertex
    uint32_t *sup;                 // edge: triangles through every edge, added at one of its two entries
    const int32_t *lev;            // cover: the BFS levels
};

// Algorithm 3's test for a common neighbour w of the horizontal edge xy (x
// at level lx): a triangle is counted from this edge when w is on another
// level, or on the same level with the larger id of the three (so that a
// triangle with three horizontal edges is counted from the edge of its two
// smaller ids only).
__device__ __forceinline__ bool cover_counts(int32_t lw, int32_t lx, int32_t w, int32_t hi_xy) {
    return lw != lx || w > hi_xy;
}

// Partner information for the c0 position p of owner x: is the edge owned
// for this kind, where is the partner's list (both from the ownership pass's
// record, read coalesced), and which vertex is the partner (read only by the
// modes that use it).
__device__ __forceinline__ bool partner_at(const Graph &g, int kind, int32_t p, int32_t je, int32_t &sy,
                                           int32_t &yb, int32_t &y) {
    sy = 0;
    yb = 0;
    y = 0;
    if (p >= je) return false;
    y = g.c0[p];
    const int2 r = (kind == 0 ? g.prec0 : g.prec1)[p];
    yb = r.x;
    sy = r.y;
    return sy > 0;
}

// Partner lists at least this long stream through stream_long.
constexpr int32_t kLongList = kWave;

// Element `at` of a list array: with 32-bit byte offsets (arrays below 2^30
// entries) the load takes the array's scalar base plus one 32-bit offset, so
// the address costs one instruction; `wide` arrays use 64-bit offsets.
template <bool kWideIdx>
__device__ __forceinline__ int32_t list_elem(const int32_t *lists, int32_t at) {
    if constexpr (kWideIdx)
        return lists[at];
    else
        return *reinterpret_cast<const int32_t *>(reinterpret_cast<const char *>(lists) + ((uint32_t)at << 2));
}

// Streams lists of at least 64 elements, a row of 64 consecutive elements of
// one list at a time (lane l takes element 64 r + l of the list's row r), kPer
// rows per window, kPer loads in flight per lane.  A row never spans two
// lists, so its address is the row's scalar base plus the lane (clamped to
// the list's last element in a partial row, which is then masked before its
// lookups by a uniform branch).  The lists are taken in lane order of m;
// the cursor (next row's base, elements left in the list) is uniform and
// lives in scalar registers.  m: lanes holding a list; len / yb: the list's
// length (0 off m) and offset in `lists`.
template <bool kWideIdx, class Count>
__device__ __forceinline__ uint32_t stream_rows(const int32_t *lists, uint64_t m, int32_t len, int32_t yb,
                                                Count count) {
    const int l = lane_id();
    // rows of the batch: the loop runs until every row has been probed (a
    // scalar, so that the loop's branches stay uniform)
    int32_t left = __builtin_amdgcn_readfirstlane(wave_sum((len + kWave - 1) >> 6));
    uint64_t rest = m;
    const int first = (int)__builtin_ctzll(rest);
    rest &= rest - 1;
    int32_t s_off = __builtin_amdgcn_readlane(yb, first);
    int32_t s_rem = __builtin_amdgcn_readlane(len, first);
    const int32_t s_safe = s_off;   // rows past the last list re-read the first list's first row
    // the next row: its base and how many of its lanes hold elements (<= 0:
    // past the last list); a row that ends a list moves the cursor on
    auto gather = [&](int32_t (&v)[kPer], int32_t (&lim)[kPer]) {
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            if (s_rem <= 0 && rest) {
                const int nl = (int)__builtin_ctzll(rest);
                rest &= rest - 1;
                s_off = __builtin_amdgcn_readlane(yb, nl);
                s_rem = __builtin_amdgcn_readlane(len, nl);
            }
            lim[u] = s_rem;
            // lanes past a list's end re-read its last element (a line the
            // row fetches anyway); rows past the last list re-read the first
            const int32_t base = s_rem > 0 ? s_off : s_safe;
            const int32_t last = s_rem > 0 && s_rem < kWave ? s_rem - 1 : kWave - 1;
            v[u] = list_elem<kWideIdx>(lists, base + min(l, last));
            s_off += kWave;
            s_rem -= kWave;
        }
    };
    // the lanes of a partial or spent row become padding keys: a compare
    // and a select per key, unconditionally (testing first whether the row
    // is partial makes the compiler select between selects, twice the VALU)
    auto masked = [&](int32_t (&v)[kPer], const int32_t (&lim)[kPer]) {
#pragma unroll
        for (int u = 0; u < kPer; ++u) v[u] = lim[u] > l ? v[u] : kNoKey;
    };
    // software pipeline, two windows in ping-pong registers: the next
    // window's loads are issued (unconditionally, past the end at valid
    // addresses) before this window's lookups, so their latency overlaps the
    // LDS probes and every wait covers one window's loads
    uint32_t hits = 0;
    int32_t va[kPer], la[kPer], vb[kPer], lb[kPer];
    gather(va, la);
    for (;;) {
        gather(vb, lb);
        masked(va, la);
        hits += count(va);
        left -= kPer;
        if (left <= 0) break;
        gather(va, la);
        masked(vb, lb);
        hits += count(vb);
        left -= kPer;
        if (left <= 0) break;
    }
    return hits;
}

template <class Count>
__device__ __forceinline__ uint32_t stream_long(const int32_t *lists, uint64_t m, int32_t len, int32_t yb, bool wide,
                                                Count count) {
    if (wide) return stream_rows<true>(lists, m, len, yb, count);
    return stream_rows<false>(lists, m, len, yb, count);
}

// Streams the owned partner lists among the 64 c0 positions starting at p0
// through `count` (a functor over kPer keys).  The lists are concatenated
// into one virtual array that the wavefront consumes 64 * kPer elements per
// step (kPer loads in flight per lane); the list an element belongs to is
// found from a ballot of the marked list starts in the window and a
// popcount, O(1) per element.
// With `sliced`, only the part of each partner list with values in
// [lo, hi) is streamed (two binary searches per partner).  kRec selects what
// else travels with each element: nothing (`count(v)`), the index of its
// partner record (`count(v, rec)`), or that and the element's own index in
// the list array (`count(v, rec, idx)`).  Records hold a tag (kRecVertex:
// the partner vertex; kRecEdge: the input entry of the edge owner-partner)
// and a hit counter that the functor may bump in LDS; `count.finish(tag, c)`
// then sees every record with c > 0 once at the end of the chunk.
enum { kRecNone = 0, kRecVertex = 1, kRecEdge = 2 };
template <int kRec, class Count>
__device__ __forceinline__ uint32_t stream_chunk(const Graph &g, int kind, int32_t x, int32_t sx, int32_t p0,
                                                 int32_t je, int32_t *scr, Count count, bool sliced = false,
                                                 int32_t lo = 0, int32_t hi = 0) {
    static_assert(kPer == 8, "a lane reads its window markers as one 64-bit word");
    const int l = lane_id();
    int32_t sy, yb, yid;
    bool mine = partner_at(g, kind, p0 + l, je, sy, yb, yid);
    const int32_t *lists = kind == 0 ? g.c0 : g.c1;
    if (sliced && mine) {
        const int32_t *smp = kind == 0 ? g.s0 : g.s1;
        const int32_t so = kind == 0 ? g.so0 : g.so1;
        const int32_t b = sampled_lower(lists, smp, so, yb, sy, lo);
        const int32_t e = sampled_lower(lists, smp, so, b, yb + sy - b, hi);
        yb = b;
        sy = e - b;
        mine = sy > 0;   // two lists may not start at one window offset
    }
    uint32_t long_hits = 0;
    if constexpr (kRec == kRecNone) {   // long lists take the marker-free path
        const bool lng = mine && sy >= kLongList;
        const uint64_t ml = __ballot(lng);
        if (ml) long_hits = stream_long(lists, ml, lng ? sy : 0, yb, g.wide != 0, count);
        mine = mine && !lng;
    }
    const uint64_t m = __ballot(mine);
    if (m == 0) return long_hits;
    uint8_t *marker = reinterpret_cast<uint8_t *>(scr);
    int2 *pinfo = reinterpret_cast<int2 *>(scr + 16 * kPer);
    int32_t *ptag = scr + kScratchInts;                                     // kRec != kRecNone only
    uint32_t *pcnt = reinterpret_cast<uint32_t *>(scr + kScratchInts + 64);   // kept zero between chunks
    const int32_t len = mine ? sy : 0;
    const int32_t incl = wave_incl_scan(len);
    const int32_t start = incl - len;
    const int32_t total = __shfl(incl, kWave - 1, kWave);
    if (mine) {
        const int r = __popcll(m & ((1ull << l) - 1));
        pinfo[r] = make_int2(start, yb);
        if constexpr (kRec == kRecVertex) ptag[r] = yid;
        if constexpr (kRec == kRecEdge) ptag[r] = g.pos0[p0 + l];   // owned partners sit at c0[p0 + l]
    }
    const uint64_t le = (l == kWave - 1) ? ~0ull : ((2ull << l) - 1);
    int32_t before = 0;   // lists that start before the current window
    constexpr int32_t kStep = kPer * kWave;
    // loads of the window at `base`: lane l takes elements base + 64u + l;
    // slots past the end read element 0 of the list array and are masked
    // when consumed, so the loads need no branch and stay in flight
    auto gather = [&](int32_t base, int32_t (&v)[kPer], int32_t (&ys)[kPer], int32_t (&ix)[kPer]) {
        const int32_t o = start - base;
        const bool mark = mine && o >= 0 && o < kStep;
        const int mslot = (o & 63) * kPer + (o >> 6);
        if (mark) marker[mslot] = 1;
        wave_lds_sync();
        const uint64_t mk = *reinterpret_cast<const uint64_t *>(marker + l * kPer);
        wave_lds_sync();
        if (mark) marker[mslot] = 0;
        // a slot past the end belongs to the last list (no list starts
        // after it), so clamping its position to total - 1 keeps every
        // address valid without a branch; such slots are masked later
        int32_t k[kPer];
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const uint64_t mw = __ballot((mk >> (8 * u)) & 0xffu);
            k[u] = max(before + (int32_t)__popcll(mw & le) - 1, 0);   // int max: a mixed signed / unsigned max resolves to double
            before += __popcll(mw);
        }
        int2 pi[kPer];
#pragma unroll
        for (int u = 0; u < kPer; ++u) pi[u] = pinfo[k[u]];
        if constexpr (kRec != kRecNone) {
#pragma unroll
            for (int u = 0; u < kPer; ++u) ys[u] = k[u];
        }
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int32_t f = min(base + u * kWave + l, total - 1);
            const int32_t at = pi[u].y + f - pi[u].x;
            v[u] = lists[at];
            if constexpr (kRec == kRecEdge) ix[u] = at;
        }
    };
    auto masked = [&](int32_t base, int32_t (&v)[kPer]) {
#pragma unroll
        for (int u = 0; u < kPer; ++u) v[u] = base + u * kWave + l < total ? v[u] : kNoKey;
    };
    // software pipeline: the next window's loads are issued before this
    // window's lookups, so their latency overlaps the LDS probes.  The next
    // gather is unconditional (past the end it reads clamped, valid
    // addresses) so that every iteration has the same loads in flight and the
    // wait before the lookups covers only this window's loads.
    uint32_t hits = 0;
    int32_t va[kPer], ya[kPer], ia[kPer];
    gather(0, va, ya, ia);
    for (int32_t base = 0;; base += kStep) {
        int32_t vb[kPer], yb2[kPer], ib[kPer];
        gather(base + kStep, vb, yb2, ib);
        masked(base, va);
        if constexpr (kRec == kRecEdge) hits += count(va, ya, ia, ptag, pcnt);
        else if constexpr (kRec == kRecVertex) hits += count(va, ya, ptag, pcnt);
        else hits += count(va);
        if (base + kStep >= total) break;
#pragma unroll
        for (int u = 0; u < kPer; ++u) va[u] = vb[u];
        if constexpr (kRec != kRecNone) {
#pragma unroll
            for (int u = 0; u < kPer; ++u) ya[u] = yb2[u];
        }
        if constexpr (kRec == kRecEdge) {
#pragma unroll
            for (int u = 0; u < kPer; ++u) ia[u] = ib[u];
        }
    }
    if constexpr (kRec != kRecNone) {
        wave_lds_sync();   // every lane's counter updates are done
        if (l < __popcll(m)) {
            const uint32_t c = pcnt[l];
            if (c) {
                count.finish(ptag[l], c);
                pcnt[l] = 0;
            }
        }
    }
    wave_lds_sync();   // pinfo is rewritten by the next batch
    return hits + long_hits;
}

// Merge strategy for a small owner, one lane per item: the lane walks the
// item's partners and merges each owned partner list (never longer than the
// owner's) with the owner list.  Hits of this lane; in vertex mode every
// common neighbour w and the partner get their triangles (the owner's are
// added by the caller), in edge mode the three edges of every triangle.
// When only counts are needed, owners of at most kOw elements take the
// register form: the owner list sits in registers, and the partners are
// taken kB at a time: their records, then all their list elements (never
// more than the owner's), each with independent loads, then every element is
// compared with the whole owner list.  A batch of partners thus costs two
// load latencies, where a merge waits on every step.  The caller picks kOw
// for the largest owner of the wavefront's items (a uniform choice).
template <int kOw, int kB>
__device__ __forceinline__ uint32_t lane_reg_item(const Graph &g, int kind, int32_t sx, const int32_t *a, int32_t jb,
                                                  int32_t je) {
    const int32_t *lists = kind == 0 ? g.c0 : g.c1;
    int32_t ao[kOw];
#pragma unroll
    for (int k = 0; k < kOw; ++k) ao[k] = k < sx ? a[k] : -1;
    uint32_t hits = 0;
    for (int32_t p = jb; p < je; p += kB) {
        int32_t sy[kB], yb[kB];
#pragma unroll
        for (int q = 0; q < kB; ++q) {
            int32_t y;
            partner_at(g, kind, p + q, je, sy[q], yb[q], y);   // sy = 0 past je or where not owned
        }
        // a partner's elements in rounds of at most 8 (16 loads in flight
        // per lane keep the kernel within its registers)
        constexpr int kC = kOw < 8 ? kOw : 8;
#pragma unroll 1
        for (int c = 0; c < kOw; c += kC) {
            int32_t bv[kB][kC];
#pragma unroll
            for (int q = 0; q < kB; ++q)
#pragma unroll
                for (int k = 0; k < kC; ++k) bv[q][k] = c + k < sy[q] ? lists[yb[q] + c + k] : -2;
#pragma unroll
            for (int q = 0; q < kB; ++q)
#pragma unroll
                for (int i = 0; i < kOw; ++i)
#pragma unroll
                    for (int k = 0; k < kC; ++k) hits += ao[i] == bv[q][k] ? 1u : 0u;
        }
    }
    return hits;
}

template <int kMode>
__device__ __forceinline__ uint32_t lane_merge_item(const Graph &g, int kind, int32_t x, int32_t jb, int32_t je,
                                                    const Sink &sk) {
    const int32_t *a = list_ptr(kind, g.rp0, g.c0, g.rp1, g.c1, x);
    const int32_t sx = list_size(kind, g.up0, g.rp1, x);
    const int32_t *lists = kind == 0 ? g.c0 : g.c1;
    const int32_t *lpos = kind == 0 ? g.pos0 : g.pos1;   // edge mode only
    const int32_t xb = (int32_t)(a - lists);
    const int32_t lx = kMode == kModeCover ? sk.lev[x] : 0;
    uint32_t hits = 0;
    for (int32_t p = jb; p < je; ++p) {
        int32_t sy, yb, y;
        if (!partner_at(g, kind, p, je, sy, yb, y)) continue;   // owned: sx >= sy >= 1
        const int32_t *b = lists + yb;
        int32_t i = 0, j = 0, ai = a[0], bj = b[0];
        const uint32_t h0 = hits;
        const int32_t hi_xy = max(x, y);
        for (;;) {
            if (ai == bj) {
                if constexpr (kMode == kModeVertex) atomicAdd(&sk.tv[ai], 1ull);
                if constexpr (kMode == kModeEdge) {
                    atomicAdd(&sk.sup[lpos[xb + i]], 1u);
                    atomicAdd(&sk.sup[lpos[yb + j]], 1u);
                }
                if constexpr (kMode == kModeCover) hits += cover_counts(sk.lev[ai], lx, ai, hi_xy) ? 1u : 0u;
                else ++hits;
                if (++i >= sx || ++j >= sy) break;
                ai = a[i];
                bj = b[j];
            } else if (ai < bj) {
                if (++i >= sx) break;
                ai = a[i];
            } else {
                if (++j >= sy) break;
                bj = b[j];
            }
        }
        if constexpr (kMode == kModeVertex)
            if (hits != h0) atomicAdd(&sk.tv[y], (unsigned long long)(hits - h0));
        if constexpr (kMode == kModeEdge)
            if (hits != h0) atomicAdd(&sk.sup[g.pos0[p]], hits - h0);
    }
    return hits;
}

// Owners of up to kLdsOwner elements when only counts are needed and the
// wavefront's table region holds kLdsOwner ints per lane: each lane keeps
// its owner list in LDS, element k of lane l at tab[k * 64 + l] (a
// wavefront's reads of one step hit 64 distinct banks), padded with
// INT32_MAX, and looks every partner element up by a branch-free binary
// search there (five dependent LDS reads, no global ones).  Partners come
// kB at a time and their elements eight at a time, loaded independently,
// so a batch costs two load latencies as in the register form.
constexpr int kLdsOwner = 32;
template <int kB>
__device__ __forceinline__ uint32_t lane_lds_item(const Graph &g, int kind, int32_t sx, const int32_t *a, int32_t jb,
                                                  int32_t je, int32_t *tab) {
    static_assert(kLdsOwner == 32, "the search below takes five halving steps");
    const int l = lane_id();
    const int32_t *lists = kind == 0 ? g.c0 : g.c1;
#pragma unroll 1
    for (int c = 0; c < kLdsOwner; c += 8) {
        int32_t v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = c + k < sx ? a[c + k] : INT32_MAX;
#pragma unroll
        for (int k = 0; k < 8; ++k) tab[(c + k) * kWave + l] = v[k];
    }
    uint32_t hits = 0;
    for (int32_t p = jb; p < je; p += kB) {
        int32_t sy[kB], yb[kB];
#pragma unroll
        for (int q = 0; q < kB; ++q) {
            int32_t y;
            partner_at(g, kind, p + q, je, sy[q], yb[q], y);   // sy = 0 past je or where not owned
        }
#pragma unroll 1
        for (int c = 0; c < kLdsOwner; c += 8) {
            int32_t bv[kB][8];
#pragma unroll
            for (int q = 0; q < kB; ++q)
#pragma unroll
                for (int k = 0; k < 8; ++k) bv[q][k] = c + k < sy[q] ? lists[yb[q] + c + k] : -2;
#pragma unroll
            for (int q = 0; q < kB; ++q) {
                int32_t pos[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) pos[k] = 0;
#pragma unroll
                for (int step = 16; step > 0; step >>= 1)
#pragma unroll
                    for (int k = 0; k < 8; ++k) pos[k] += tab[(pos[k] + step - 1) * kWave + l] < bv[q][k] ? step : 0;
#pragma unroll
                for (int k = 0; k < 8; ++k) hits += tab[pos[k] * kWave + l] == bv[q][k] ? 1u : 0u;
            }
        }
    }
    return hits;
}

// The counting modes' lane items of one wavefront (a lane without an item
// has an empty partner range): the register form sized for the largest
// owner among them, the LDS form up to kLdsOwner elements where the
// wavefront's table region holds them, or the merge.
template <int kMode>
__device__ __forceinline__ uint32_t lane_count_item(const Graph &g, bool has, int kind, int32_t x, int32_t jb,
                                                    int32_t je, const Sink &sk, int32_t *tab, int wave_log2) {
    const int32_t *a = list_ptr(kind, g.rp0, g.c0, g.rp1, g.c1, x);
    const int32_t sx = has ? list_size(kind, g.up0, g.rp1, x) : 0;
    int32_t smax = sx;
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) smax = max(smax, __shfl_xor(smax, d, kWave));
    if (smax <= 2) return lane_reg_item<2, 4>(g, kind, sx, a, jb, je);
    if (smax <= 4) return lane_reg_item<4, 4>(g, kind, sx, a, jb, je);
    if (smax <= 8) return lane_reg_item<8, 2>(g, kind, sx, a, jb, je);
    if (smax <= 16) return lane_reg_item<16, 1>(g, kind, sx, a, jb, je);
    if (smax <= kLdsOwner && (kLdsOwner << 6) <= (1 << wave_log2)) return lane_lds_item<2>(g, kind, sx, a, jb, je, tab);
    return has ? lane_merge_item<kMode>(g, kind, x, jb, je, sk) : 0u;
}

// Merge strategy: partners one at a time, each merged against the owner list.
template <int kMode>
__device__ __forceinline__ uint32_t merge_chunk(const Graph &g, int kind, int32_t x, int32_t sx, const int32_t *a,
                                                int32_t p0, int32_t je, const Sink &sk) {
    int32_t sy, yb, yid;
    const bool mine = partner_at(g, kind, p0 + lane_id(), je, sy, yb, yid);
    uint64_t m = __ballot(mine);
    const int32_t *lists = kind == 0 ? g.c0 : g.c1;
    uint32_t hits = 0;
    while (m) {
        const int src = __ffsll((unsigned long long)m) - 1;
        m &= m - 1;
        if constexpr (kMode == kModeVertex) {
            const uint32_t h = merge_count(a, sx, lists + __shfl(yb, src, kWave), __shfl(sy, src, kWave),
                                           [&](int32_t w, int32_t, int32_t) { atomicAdd(&sk.tv[w], 1ull); });
            const int32_t y = __shfl(yid, src, kWave);
            if (h) atomicAdd(&sk.tv[y], (unsigned long long)h);
            hits += h;
        } else if constexpr (kMode == kModeEdge) {
            const int32_t *lpos = kind == 0 ? g.pos0 : g.pos1;
            const int32_t xb = (int32_t)(a - lists), ybs = __shfl(yb, src, kWave);
            const uint32_t h = merge_count(a, sx, lists + ybs, __shfl(sy, src, kWave), [&](int32_t, int32_t i, int32_t j) {
                atomicAdd(&sk.sup[lpos[xb + i]], 1u);
                atomicAdd(&sk.sup[lpos[ybs + j]], 1u);
            });
            if (h) atomicAdd(&sk.sup[g.pos0[p0 + src]], h);
            hits += h;
        } else if constexpr (kMode == kModeCover) {
            const int32_t hi_xy = max(x, __shfl(yid, src, kWave));
            const int32_t lx = sk.lev[x];
            uint32_t c = 0;
            merge_count(a, sx, lists + __shfl(yb, src, kWave), __shfl(sy, src, kWave),
                        [&](int32_t w, int32_t, int32_t) { c += cover_counts(sk.lev[w], lx, w, hi_xy) ? 1u : 0u; });
            hits += c;
        } else {
            hits += merge_count(a, sx, lists + __shfl(yb, src, kWave), __shfl(sy, src, kWave),
                                [](int32_t, int32_t, int32_t) {});
        }
    }
    return hits;
}

// The lookups of one window.  Plain modes count the keys found.  The other
// modes take the mask of keys found and, per key, where it was found: a hash
// table slot (kSlots: its LDS counter is bumped and flushed once per item by
// the caller) or an index in the owner list (credited at once).
struct HashProbe {
    static constexpr bool kSlots = true;
    static constexpr bool kWide = true;   // all kPer keys of a window in one group
    HashTab t;
    template <bool kMask> __device__ __forceinline__ uint32_t run(const int32_t (&q)[4]) const {
        return hash_count<4, kMask>(t, q);
    }
    template <bool kMask> __device__ __forceinline__ uint32_t run8(const int32_t (&q)[kPer]) const {
        return hash_count<kPer, kMask>(t, q);
    }
    __device__ __forceinline__ uint32_t find(const int32_t (&q)[4], int32_t (&e)[4]) const {
        return hash_find<4>(t, q, e);
    }
    __device__ __forceinline__ uint32_t find8(const int32_t (&q)[kPer], int32_t (&e)[kPer]) const {
        return hash_find<kPer>(t, q, e);
    }
};
struct SearchProbe {
    static constexpr bool kSlots = false;
    static constexpr bool kWide = false;
    const int32_t *a;
    int32_t len;
    template <bool kMask> __device__ __forceinline__ uint32_t run(const int32_t (&q)[4]) const {
        return search_count<4, kMask>(a, len, q);
    }
    __device__ __forceinline__ uint32_t find(const int32_t (&q)[4], int32_t (&e)[4]) const {
        return search_find<4>(a, len, q, e);
    }
};
template <class Probe> struct WindowCount {
    Probe p;
    __device__ __forceinline__ uint32_t operator()(const int32_t (&v)[kPer]) const {
        if constexpr (Probe::kWide) return p.template run8<false>(v);
        else return in_fours(v, [&](const int32_t(&q)[4]) { return p.template run<false>(q); });
    }
};

template <class Probe>
__device__ __forceinline__ uint32_t find8(const Probe &p, const int32_t (&v)[kPer], int32_t (&e)[kPer]) {
    if constexpr (Probe::kWide) return p.find8(v, e);
    const int32_t a[4] = {v[0], v[1], v[2], v[3]};
    const int32_t b[4] = {v[4], v[5], v[6], v[7]};
    int32_t ea[4], eb[4];
    const uint32_t mk = p.find(a, ea) | (p.find(b, eb) << 4);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        e[u] = ea[u];
        e[u + 4] = eb[u];
    }
    return mk;
}

// Per-vertex counts: the common neighbour w through the slot counter (hash)
// or at once (search), the partner through its record counter; the owner's
// share is added per item by the caller.
template <class Probe> struct WindowVertex {
    Probe p;
    unsigned long long *tv;
    __device__ __forceinline__ uint32_t operator()(const int32_t (&v)[kPer], const int32_t (&rec)[kPer],
                                                   const int32_t *, uint32_t *pcnt) const {
        int32_t e[kPer];
        const uint32_t mk = find8(p, v, e);
#pragma unroll
        for (int u = 0; u < kPer; ++u)
            if ((mk >> u) & 1u) {
                if constexpr (Probe::kSlots) atomicAdd(&p.t.cnt[e[u]], 1u);
                else atomicAdd(&tv[v[u]], 1ull);
                atomicAdd(&pcnt[rec[u]], 1u);
            }
        return (uint32_t)__popc(mk);
    }
    __device__ __forceinline__ void finish(int32_t y, uint32_t c) const { atomicAdd(&tv[y], (unsigned long long)c); }
};

// Per-edge counts: owner-w through the slot counter (hash) or at once
// (search), partner-w at once (a distinct edge per element), owner-partner
// through the record counter.
template <class Probe> struct WindowEdge {
    Probe p;
    uint32_t *sup;
    const int32_t *lpos;   // input entry of every element of the list array streamed
    const int32_t *apos;   // the same for the owner list (search only)
    __device__ __forceinline__ uint32_t operator()(const int32_t (&v)[kPer], const int32_t (&rec)[kPer],
                                                   const int32_t (&idx)[kPer], const int32_t *,
                                                   uint32_t *pcnt) const {
        int32_t e[kPer];
        const uint32_t mk = find8(p, v, e);
#pragma unroll
        for (int u = 0; u < kPer; ++u)
            if ((mk >> u) & 1u) {
                if constexpr (Probe::kSlots) atomicAdd(&p.t.cnt[e[u]], 1u);
                else atomicAdd(&sup[apos[e[u]]], 1u);
                atomicAdd(&sup[lpos[idx[u]]], 1u);
                atomicAdd(&pcnt[rec[u]], 1u);
            }
        return (uint32_t)__popc(mk);
    }
    __device__ __forceinline__ void finish(int32_t exy, uint32_t c) const { atomicAdd(&sup[exy], c); }
};

template <class Probe> struct WindowCover {
    Probe p;
    const int32_t *lev;
    int32_t x, lx;
    __device__ __forceinline__ uint32_t operator()(const int32_t (&v)[kPer], const int32_t (&rec)[kPer],
                                                   const int32_t *ptag, uint32_t *) const {
        uint32_t mk;
        if constexpr (Probe::kWide) {
            mk = p.template run8<true>(v);
        } else {
            const int32_t a[4] = {v[0], v[1], v[2], v[3]};
            const int32_t b[4] = {v[4], v[5], v[6], v[7]};
            mk = p.template run<true>(a) | (p.template run<true>(b) << 4);
        }
        uint32_t c = 0;
#pragma unroll
        for (int u = 0; u < kPer; ++u)
            if ((mk >> u) & 1u) c += cover_counts(lev[v[u]], lx, v[u], max(x, ptag[rec[u]])) ? 1u : 0u;
        return c;
    }
    __device__ __forceinline__ void finish(int32_t, uint32_t) const {}
};

// One chunk of owned partners through a lookup structure, in the kernel's mode.
template <int kMode, class Probe>
__device__ __forceinline__ uint32_t probe_chunk(const Graph &g, int kind, int32_t x, int32_t sx, int32_t p0,
                                                int32_t je, int32_t *scr, const Probe &pr, const Sink &sk,
                                                bool sliced = false, int32_t lo = 0, int32_t hi = 0) {
    if constexpr (kMode == kModeVertex)
        return stream_chunk<kRecVertex>(g, kind, x, sx, p0, je, scr, WindowVertex<Probe>{pr, sk.tv}, sliced, lo, hi);
    else if constexpr (kMode == kModeCover)
        return stream_chunk<kRecVertex>(g, kind, x, sx, p0, je, scr, WindowCover<Probe>{pr, sk.lev, x, sk.lev[x]},
                                        sliced, lo, hi);
    else if constexpr (kMode == kModeEdge)
        return stream_chunk<kRecEdge>(
            g, kind, x, sx, p0, je, scr,
            WindowEdge<Probe>{pr, sk.sup, kind == 0 ? g.pos0 : g.pos1,
                              kind == 0 ? g.pos0 + g.rp0[x] : g.pos1 + g.rp1[x]},
            sliced, lo, hi);
    else
        return stream_chunk<kRecNone>(g, kind, x, sx, p0, je, scr, WindowCount<Probe>{pr}, sliced, lo, hi);
}

// Table size for sx keys: load at most 1/32 where the space allows, never
// above max_log2 (the LDS region is reserved either way; only the clearing
// grows, and fewer probes leave their home bucket); feasibility guarantees
// load at most 1/2 at the cap.
__device__ __forceinline__ int table_log2(int32_t sx, int max_log2) {
    int lg = 6;   // at least 64 slots
    while (lg < max_log2 && (1 << lg) < 32 * sx) ++lg;
    return lg;
}

// kProf adds the profile: per (bucket, strategy) the wavefront-ticks of the
// items (elapsed constant-clock ticks times the wavefronts an item occupies)
// and the item count, accumulated into prof[(b * 4 + s) * 3 + {0, 2}].
// kMode: kModeBatch adds each item's hits to the counter of the owner's
// graph; kModeVertex adds every triangle to its three vertices (the owner's
// share once per item); kModeEdge adds every triangle to its three edges,
// each at one of the edge's two input entries.  These two modes keep a hit
// counter beside every hash table slot (a second LDS region as large as the
// tables), flushed to the common neighbour's count once per item, so a hub
// that is a common neighbour of many pairs sees one global atomic per owner
// list instead of one per triangle.
template <bool kProf, int kMode>
__global__ __launch_bounds__(kIsectThreads) void k_isect(Graph g, const Item *__restrict__ items,
                                                          int32_t *__restrict__ q, int wg_log2, int wave_log2,
                                                          int wg_cap_log2,
                                                          int table_ints, unsigned long long *__restrict__ tri,
                                                          unsigned long long *__restrict__ prof, Sink sk) {
    extern __shared__ int32_t lds[];
    __shared__ int32_t s_item, s_chunk;
    const int32_t n_wg = q[2], n_all = q[3];
    constexpr bool kBatch = kMode == kModeBatch;
    constexpr bool kEdge = kMode == kModeEdge;
    constexpr bool kOwnerSink = kMode == kModeBatch || kMode == kModeVertex;
    constexpr bool kSlotCnt = kMode == kModeVertex || kEdge;   // counters beside the table slots
    constexpr int kScr = kMode == kModeVertex || kMode == kModeCover || kEdge ? kScratchIdsInts : kScratchInts;
    const int w = threadIdx.x / kWave;
    const int l = lane_id();
    int32_t *scr = lds + (kSlotCnt ? 2 : 1) * table_ints + w * kScr;
    uint32_t *slot_cnt = reinterpret_cast<uint32_t *>(lds + table_ints);   // kSlotCnt only
    reinterpret_cast<uint64_t *>(scr)[l] = 0ull;   // markers start clear
    if (kScr == kScratchIdsInts) scr[kScratchInts + 64 + l] = 0;   // record counters start clear
    if constexpr (kSlotCnt)   // slot counters start clear (the first item's barrier orders this)
        for (int i = threadIdx.x; i < table_ints; i += kIsectThreads) slot_cnt[i] = 0;
    // a flush of the slot counters after an item's lookups: the hits of each
    // owner-list key go to its vertex / to the input entry of the edge
    // owner-key (found by binary search in the owner list)
    auto flush_slots = [&](const HashTab &ht, int nslots, int first, int step, const int32_t *a, int32_t sx,
                           int kind, int32_t x) {
        for (int i = first; i < nslots; i += step) {
            const uint32_t c = ht.cnt[i];
            if (c == 0) continue;
            ht.cnt[i] = 0;
            const int32_t key = ht.tab[i];
            if constexpr (kMode == kModeVertex) {
                atomicAdd(&sk.tv[key], (unsigned long long)c);
            } else if constexpr (kEdge) {
                const int32_t *apos = kind == 0 ? g.pos0 + g.rp0[x] : g.pos1 + g.rp1[x];
                atomicAdd(&sk.sup[apos[lower_idx(a, sx, key)]], c);
            }
        }
    };
    uint64_t acc0 = 0, acc1 = 0;

    // ---- workgroup items, claimed by blocks from a counter (they are few):
    // one shared table, wavefronts claim 64-position chunks through LDS
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(&q[0], 1);
        __syncthreads();
        const int32_t it = s_item;
        if (it >= n_wg) break;
        const uint64_t t_beg = kProf ? wall_clock64() : 0;
        const Item item = items[it];
        const int kind = item.code & 1;
        const int32_t x = item.owner;
        const int32_t *a = list_ptr(kind, g.rp0, g.c0, g.rp1, g.c1, x);
        const int32_t sx = list_size(kind, g.up0, g.rp1, x);
        // the owner slice of this item: positions [a_lo, a_hi), values [lo, hi)
        const int32_t nsl = owner_slices(sx, wg_cap_log2 - (((uint32_t)item.code >> kHalfShift) & 1));
        const int32_t si = (int32_t)((uint32_t)item.code >> kSliceShift);
        const int32_t a_lo = (int32_t)((int64_t)sx * si / nsl), a_hi = (int32_t)((int64_t)sx * (si + 1) / nsl);
        const bool sliced = nsl > 1;
        const int32_t lo = sliced ? a[a_lo] : 0;
        const int32_t hi = sliced && a_hi < sx ? a[a_hi] : INT32_MAX;
        const int lg = table_log2(a_hi - a_lo, wg_log2);
        const HashTab ht = make_tab(lds, lg, a_hi - a_lo, kSlotCnt ? slot_cnt : nullptr);
        if (threadIdx.x == 0) s_chunk = 0;
        for (int i = threadIdx.x; i < (1 << lg) / 4; i += kIsectThreads)
            reinterpret_cast<int4 *>(lds)[i] = make_int4(kEmpty, kEmpty, kEmpty, kEmpty);
        __syncthreads();   // (slot counters are zero: the kernel starts them so and every flush clears them)
        for (int i = a_lo + (int)threadIdx.x; i < a_hi; i += kIsectThreads) hash_insert(ht, a[i]);
        __syncthreads();
        uint32_t h = 0;
        for (;;) {
            int32_t c = 0;
            if (l == 0) c = atomicAdd(&s_chunk, 1);
            const int32_t p0 = item.jb + __shfl(c, 0, kWave) * kWave;
            if (p0 >= item.je) break;
            h += probe_chunk<kMode>(g, kind, x, sx, p0, item.je, scr, HashProbe{ht}, sk, sliced, lo, hi);
        }
        if constexpr (kSlotCnt) {
            __syncthreads();   // every wavefront's lookups are done
            flush_slots(ht, 1 << lg, (int)threadIdx.x, kIsectThreads, a, sx, kind, x);
        }
        if (kind == 0) acc0 += h; else acc1 += h;
        if (kOwnerSink) {
            const unsigned long long hs = wave_sum((unsigned long long)h);
            if (l == 0 && hs) atomicAdd(kBatch ? &sk.counts[sk.gid[x]] : &sk.tv[x], hs);
        }
        __syncthreads();   // the table, s_item and s_chunk are reused by the next item
        if (kProf && threadIdx.x == 0) {
            unsigned long long *pr = prof + (((item.code >> 3) & (kBuckets - 1)) * TC_NUM_STRATEGIES + TC_STRAT_WG_HASH) * 3;
            atomicAdd(&pr[0], (unsigned long long)(wall_clock64() - t_beg) * kIsectWaves);
            atomicAdd(&pr[2], 1ull);
        }
    }

    // ---- wavefront items in queue order (heavy first), claimed one at a
    // time so that wavefronts finish together: a static round-robin left up
    // to a fifth of the pass to the slowest wavefronts.  One counter would
    // serialise the claims, so the items are dealt to kClaimStreams
    // interleaved streams, one per XCD (blocks are placed on XCDs
    // round-robin), each with its own counter in its own cache line.  A
    // claim is issued before the claimed item is needed, hiding the
    // atomic's latency.
    int32_t *tab = lds + (w << wave_log2);
    const int32_t n_lane0 = q[4];
    // (fewer streams when the grid has fewer blocks: every stream needs one)
    const int32_t n_streams = min((int32_t)gridDim.x, kClaimStreams);
    const int32_t stream = (int32_t)blockIdx.x % n_streams;
    int32_t *ctr_wave = q + kQueueInts + kClaimStride * stream;
    int32_t *ctr_lane = ctr_wave + 1;
    auto claim = [&](int32_t *ctr) {
        int32_t c = 0;
        if (l == 0) c = atomicAdd(ctr, 1);
        return c;
    };
    int32_t c_next = __shfl(claim(ctr_wave), 0, kWave);
    for (;;) {
        const int32_t it = n_wg + stream + n_streams * c_next;
        if (it >= n_lane0) break;
        const int32_t c_pend = claim(ctr_wave);
        const uint64_t t_beg = kProf ? wall_clock64() : 0;
        const Item item = items[it];
        const int kind = item.code & 1;
        const int strat = (item.code >> 1) & 3;
        const int32_t x = item.owner;
        const int32_t *a = list_ptr(kind, g.rp0, g.c0, g.rp1, g.c1, x);
        const int32_t sx = list_size(kind, g.up0, g.rp1, x);
        uint32_t h = 0;
        if (strat == TC_STRAT_WAVE_HASH) {
            const int lg = table_log2(sx, wave_log2);
            const HashTab ht = make_tab(tab, lg, sx, kSlotCnt ? reinterpret_cast<uint32_t *>(tab + table_ints) : nullptr);
            for (int i = l; i < (1 << lg) / 4; i += kWave)
                reinterpret_cast<int4 *>(tab)[i] = make_int4(kEmpty, kEmpty, kEmpty, kEmpty);
            wave_lds_sync();
            for (int i = l; i < sx; i += kWave) hash_insert(ht, a[i]);
            wave_lds_sync();
            for (int32_t p0 = item.jb; p0 < item.je; p0 += kWave)
                h += probe_chunk<kMode>(g, kind, x, sx, p0, item.je, scr, HashProbe{ht}, sk);
            wave_lds_sync();   // lookups done before the next item clears the table
            if constexpr (kSlotCnt) {
                flush_slots(ht, 1 << lg, l, kWave, a, sx, kind, x);
                wave_lds_sync();
            }
        } else if (strat == TC_STRAT_MERGE) {
            for (int32_t p0 = item.jb; p0 < item.je; p0 += kWave) h += merge_chunk<kMode>(g, kind, x, sx, a, p0, item.je, sk);
        } else {
            for (int32_t p0 = item.jb; p0 < item.je; p0 += kWave)
                h += probe_chunk<kMode>(g, kind, x, sx, p0, item.je, scr,
                                        SearchProbe{a, sx}, sk);
        }
        if (kind == 0) acc0 += h; else acc1 += h;
        if (kOwnerSink) {
            const unsigned long long hs = wave_sum((unsigned long long)h);
            if (l == 0 && hs) atomicAdd(kBatch ? &sk.counts[sk.gid[x]] : &sk.tv[x], hs);
        }
        if (kProf && l == 0) {
            unsigned long long *pr = prof + (((item.code >> 3) & (kBuckets - 1)) * TC_NUM_STRATEGIES + strat) * 3;
            atomicAdd(&pr[0], (unsigned long long)(wall_clock64() - t_beg));
            atomicAdd(&pr[2], 1ull);
        }
        c_next = __shfl(c_pend, 0, kWave);
    }

    // ---- lane items: groups of 64 consecutive items, one per lane, claimed
    // like the wavefront items
    int32_t g_next = __shfl(claim(ctr_lane), 0, kWave);
    for (;;) {
        const int32_t g0 = n_lane0 + (stream + n_streams * g_next) * kWave;
        if (g0 >= n_all) break;
        const int32_t g_pend = claim(ctr_lane);
        const uint64_t t_beg = kProf ? wall_clock64() : 0;
        const int32_t it = g0 + l;
        int32_t code = 0;
        if constexpr (kMode == kModePlain || kMode == kModeBatch) {
            const bool has = it < n_all;
            const Item item = has ? items[it] : Item{0, 0, 0, 0};
            const int kind = item.code & 1;
            code = item.code;
            const uint32_t h = lane_count_item<kMode>(g, has, kind, item.owner, item.jb, item.je, sk, tab, wave_log2);
            if (kind == 0) acc0 += h; else acc1 += h;
            if (kOwnerSink && h)
                atomicAdd(kBatch ? &sk.counts[sk.gid[item.owner]] : &sk.tv[item.owner], (unsigned long long)h);
        } else if (it < n_all) {
            const Item item = items[it];
            const int kind = item.code & 1;
            code = item.code;
            const uint32_t h = lane_merge_item<kMode>(g, kind, item.owner, item.jb, item.je, sk);
            if (kind == 0) acc0 += h; else acc1 += h;
            if (kOwnerSink && h)
                atomicAdd(kBatch ? &sk.counts[sk.gid[item.owner]] : &sk.tv[item.owner], (unsigned long long)h);
        }
        if (kProf) {   // the group holds the wavefront until its slowest lane ends: 1/64 of that per item
            const uint64_t t_group = wall_clock64() - t_beg;
            if (it < n_all) {
                unsigned long long *pr =
                    prof + (((code >> 3) & (kBuckets - 1)) * TC_NUM_STRATEGIES + TC_STRAT_MERGE) * 3;
                atomicAdd(&pr[0], (unsigned long long)(t_group + kWave - 1) / kWave);
                atomicAdd(&pr[2], 1ull);
            }
        }
        g_next = __shfl(g_pend, 0, kWave);
    }

    const uint64_t t0 = wave_sum(acc0);
    const uint64_t t1 = wave_sum(acc1);
    if (l == 0) {
        if (t0) atomicAdd(&tri[0], (unsigned long long)t0);
        if (t1) atomicAdd(&tri[1], (unsigned long long)t1);
    }
}

// {T, T0, T1, |E0|} from the pass's sums, into a caller's device buffer.
__global__ void k_result(const unsigned long long *__restrict__ stats, const int64_t *__restrict__ e0x2,
                         unsigned long long *__restrict__ out) {
    if (threadIdx.x == 0) {
        out[0] = stats[8] + stats[9];
        out[1] = stats[8];
        out[2] = stats[9];
        out[3] = (unsigned long long)(*e0x2 / 2);
    }
}

// Per-edge counts land at either of an edge's two input entries; this pass
// adds the two and writes the sum to both.  The entry (u, v) with u < v finds
// its reverse (v, u) by binary search in row v, so each edge is handled by
// exactly one thread.
__global__ __launch_bounds__(kThreads) void k_edge_mirror(int32_t n, int64_t nnz, const int32_t *__restrict__ rp,
                                                          const int32_t *__restrict__ col, uint32_t *__restrict__ sup) {
    __shared__ int64_t rows[2];
    constexpr int64_t kTile = (int64_t)kThreads * kRun;
    for (int64_t t0 = (int64_t)blockIdx.x * kTile; t0 < nnz; t0 += (int64_t)gridDim.x * kTile) {
        tile_rows(rp, n, t0, t0 + kTile < nnz ? t0 + kTile : nnz, rows);
        const int64_t e0 = t0 + (int64_t)threadIdx.x * kRun;
        if (e0 < nnz) {
            const int64_t e1 = e0 + kRun < nnz ? e0 + kRun : nnz;
            int64_t u = row_of(rp, rows[0], rows[1], e0);
            int64_t ue = rp[u + 1];
            for (int64_t e = e0; e < e1; ++e) {
                while (e >= ue) { ++u; ue = rp[u + 1]; }
                const int32_t v = col[e];
                if (v <= u) continue;
                const int32_t b = rp[v], len = rp[v + 1] - b;
                const int32_t r = b + lower_idx(col + b, len, (int32_t)u);
                if (r < b + len && col[r] == (int32_t)u) {
                    const uint32_t t = sup[e] + sup[r];
                    sup[e] = t;
                    sup[r] = t;
                }
            }
        }
        __syncthreads();   // rows is rewritten by the next tile
    }
}

// Full-row view of a partition for the cover-edge count: no N0+ lists (so no
// kind-0 units) and kind-1 lists that are the whole input rows; the partner
// rows stay the N0 rows, so every horizontal edge is still offered to the
// endpoint with the longer list.
__global__ void k_cover_view(int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ rp0,
                             int32_t *__restrict__ up0, int4 *__restrict__ vrec) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        up0[v] = 0;
        vrec[v] = make_int4(rp0[v], 0, rp[v], rp[v + 1] - rp[v]);
    }
}

unsigned grid_for(int64_t work, int threads, int64_t cap) {
    int64_t g = (work + threads - 1) / threads;
    if (g > cap) g = cap;
    if (g < 1) g = 1;
    return (unsigned)g;
}

struct CountLayout {
    int2 *prec0, *prec1;   // per c0 entry and kind: owned partner's list (k_own)
    int32_t *tlo, *thi;   // tile table of the N0 lists (k_own)
    int32_t *cnt;
    unsigned long long *work;
    int32_t *bucket_items, *bucket_off, *bucket_cur, *q;
    Item *items;
    unsigned long long *stats;   // [0..6] unit stats, [8..9] T0/T1
    int32_t *s0, *s1;            // line samples of the c0 / c1 lists (sliced searches)
};

static_assert(lane_partners(kLaneMergeOb) >= kMinPartnersPerItem, "lane items must respect the item capacity");

}  // namespace

// Larger items cost fewer claims and partner lookups per element, but on a
// small input they leave too few items per wavefront to balance the pass:
// measured on Kronecker graphs, 65536 is about 3 % faster than 16384 from
// scale 20 (2^25 entries) up, and 1.6x slower at scale 16.
int default_chunk_work(int64_t nnz) {
    int mult = 1;
    for (int64_t f = nnz >> 22; f >= 2 && mult < 4; f >>= 1) mult <<= 1;
    return 16384 * mult;
}

namespace {

int64_t item_capacity(int32_t n, int64_t nnz) {
    // per unit: at most ceil(|N0(x)| / kMinPartnersPerItem) items
    return 2 * ((int64_t)n + nnz / kMinPartnersPerItem) + 64;
}

// Line samples of a list array (see sampled_lower).  Valid entries: the
// c0 array holds *e0x2 of them, the c1 array nnz - *e0x2, the input rows
// (cover-edge view) nnz.
enum { kSmpC0 = 0, kSmpC1 = 1, kSmpAll = 2 };
__global__ void k_samples(const int32_t *__restrict__ a, int32_t off, const int64_t *__restrict__ e0x2p, int mode,
                          int64_t nnz, int32_t *__restrict__ smp) {
    const int64_t lim = mode == kSmpC0 ? *e0x2p : mode == kSmpC1 ? nnz - *e0x2p : nnz;
    const int64_t cnt = lim > off ? (lim - off + 31) >> kSmpShift : 0;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < cnt; j += (int64_t)gridDim.x * blockDim.x)
        smp[j] = a[(j << kSmpShift) + off];
}

// index of the first element of a that starts a 128-byte line
int32_t line_start(const int32_t *a) {
    return (int32_t)(((128 - (reinterpret_cast<uintptr_t>(a) & 127)) & 127) >> 2);
}

CountLayout carve_count(Carver &c, int32_t n, int64_t nnz) {
    CountLayout L;
    const int64_t nn = n > 0 ? n : 1;
    L.prec0 = c.take<int2>(nnz > 0 ? nnz : 1);
    L.prec1 = c.take<int2>(nnz > 0 ? nnz : 1);
    L.tlo = c.take<int32_t>(tiles_of(nnz));
    L.thi = c.take<int32_t>(tiles_of(nnz));
    L.cnt = c.take<int32_t>(2 * nn);
    L.work = c.take<unsigned long long>(2 * nn);
    L.bucket_items = c.take<int32_t>(kBuckets + 1);
    L.bucket_off = c.take<int32_t>(kBuckets + 1);
    L.bucket_cur = c.take<int32_t>(kBuckets);
    L.q = c.take<int32_t>(kQueueBlockInts);
    L.items = c.take<Item>(item_capacity(n, nnz));
    L.stats = c.take<unsigned long long>(16);
    L.s0 = c.take<int32_t>(samples_of(nnz));
    L.s1 = c.take<int32_t>(samples_of(nnz));
    return L;
}

}  // namespace

int cover_view_run(int32_t n, const int32_t *rp, const int32_t *col, PartBufs *pb, hipStream_t s) {
    if (n > 0) {
        hipLaunchKernelGGL(k_cover_view, dim3(grid_for(n, 256, 65536)), dim3(256), 0, s, n, rp, pb->rp0, pb->up0,
                           pb->vrec);
        TC_HIP_TRY(hipGetLastError());
    }
    pb->rp1 = const_cast<int32_t *>(rp);    // read only from here on
    pb->c1 = const_cast<int32_t *>(col);
    return TC_OK;
}

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

static SchedCfg sched_cfg(int32_t n, int64_t nnz, const CountCfg &cfg) {
    const int wave_log2 = ilog2_host(cfg.wave_slots);
    const int wg_log2 = ilog2_host(cfg.wg_slots);
    SchedCfg sc;
    sc.table = cfg.table;
    sc.force = cfg.force;
    sc.wave_ob_max = wave_log2 - 2;
    sc.wg_cap_log2 = cfg.wg_slice_max > 0 ? ilog2_host(cfg.wg_slice_max) : wg_log2 - kWgCapShift;
    sc.wg_ob_max = sc.wg_cap_log2 - 1;
    {   // slicing needs at most 2^17 slices per owner list (list length <= min(n - 1, nnz)),
        // also with half-size slices
        const int64_t longest = (int64_t)n - 1 < nnz ? (int64_t)n - 1 : nnz;
        sc.wg_slicing = longest <= ((int64_t)1 << (kMaxSlicesLog2 + sc.wg_cap_log2 - 1)) ? 1 : 0;
    }
    // heuristic default: wavefront tables up to a quarter full (linear
    // probing lengthens quickly above that; the feasibility limit is half)
    sc.heur_wave_ob = cfg.wave_max_owner > 0 ? ilog2_host(cfg.wave_max_owner) : wave_log2 - 3;
    // lane items by default for owners up to 31 when only counts are needed
    // and the wavefront tables hold the LDS form (32 ints per lane), else up
    // to 15 (the per-vertex, per-edge and cover counts merge)
    const bool lds_form = !cfg.tv && !cfg.sup && !cfg.cover_lev && wave_log2 >= 11;
    sc.lane_batched = lds_form ? 1 : 0;
    sc.heur_merge_ob =
        cfg.merge_max_owner < 0 ? -1 : ilog2_host(cfg.merge_max_owner > 0 ? cfg.merge_max_owner : lds_form ? 31 : 15);
    if (sc.heur_merge_ob > kLaneMergeOb) sc.heur_merge_ob = kLaneMergeOb;
    sc.chunk_work = cfg.chunk_work > 0 ? cfg.chunk_work : default_chunk_work(nnz);
    return sc;
}

static __global__ void k_schedule_table(SchedCfg sc, int32_t *__restrict__ out) {
    const int b = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (b < kBuckets) {
        const int st = strategy_for(sc, b);
        out[b] = st | (tile_half(sc, b, st) ? kTileHalf : 0);
    }
}

int schedule_table_run(int32_t n, int64_t nnz, const CountCfg &cfg, int32_t *table, hipStream_t s) {
    hipLaunchKernelGGL(k_schedule_table, dim3(kBuckets / 256), dim3(256), 0, s, sched_cfg(n, nnz, cfg), table);
    TC_HIP_TRY(hipGetLastError());
    return TC_OK;
}

namespace {

// The largest dynamic LDS request and the blocks per CU of each
// intersection kernel variant, per device: the attribute call and the
// occupancy query run once per (device, kernel, LDS size), outside the
// timed region of any call.
struct LaunchCache {
    int dev;
    const void *kern;
    size_t lds;
    int per_cu;
};
std::mutex g_launch_mu;
LaunchCache g_launch[64];
int g_launch_n = 0;

int isect_blocks_per_cu(const void *kern, size_t lds, int *per_cu) {
    int dev = 0;
    TC_HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_launch_mu);
    for (int i = 0; i < g_launch_n; ++i)
        if (g_launch[i].dev == dev && g_launch[i].kern == kern && g_launch[i].lds == lds) {
            *per_cu = g_launch[i].per_cu;
            return TC_OK;
        }
    TC_HIP_TRY(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int pc = 1;
    TC_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&pc, kern, kIsectThreads, lds));
    if (pc < 1) pc = 1;
    if (g_launch_n < 64) g_launch[g_launch_n++] = LaunchCache{dev, kern, lds, pc};
    *per_cu = pc;
    return TC_OK;
}

// The intersection kernel variant, its table size and LDS bytes for cfg
// (kern is NULL for an invalid mix of modes).
struct IsectShape {
    const void *kern = nullptr;
    int table_ints = 0;
    size_t lds_bytes = 0;
};

IsectShape isect_shape(const CountCfg &cfg) {
    IsectShape sh;
    const int wave_log2 = ilog2_host(cfg.wave_slots);
    const int wg_log2 = ilog2_host(cfg.wg_slots);
    const bool batch = cfg.gid != nullptr;
    const bool vertex = cfg.tv != nullptr;
    const bool edge = cfg.sup != nullptr;
    const bool cover = cfg.cover_lev != nullptr;
    if ((vertex || edge || cover) && (batch || cfg.prof)) return sh;
    if ((int)vertex + (int)edge + (int)cover > 1) return sh;
    sh.table_ints = 1 << wg_log2;
    if ((kIsectWaves << wave_log2) > sh.table_ints) sh.table_ints = kIsectWaves << wave_log2;
    sh.lds_bytes = (size_t)((edge || vertex ? 2 : 1) * sh.table_ints +
                            kIsectWaves * (vertex || edge || cover ? kScratchIdsInts : kScratchInts)) *
                   sizeof(int32_t);
    sh.kern = cfg.prof ? (batch ? (const void *)k_isect<true, kModeBatch> : (const void *)k_isect<true, kModePlain>)
              : vertex ? (const void *)k_isect<false, kModeVertex>
              : edge   ? (const void *)k_isect<false, kModeEdge>
              : cover  ? (const void *)k_isect<false, kModeCover>
              : batch  ? (const void *)k_isect<false, kModeBatch>
                       : (const void *)k_isect<false, kModePlain>;
    return sh;
}

}  // namespace

int count_prepare(int32_t n, int64_t nnz, const CountCfg &cfg) {
    (void)nnz;
    const IsectShape sh = isect_shape(cfg);
    if (!sh.kern) return TC_ERR_ARG;
    int per_cu = 1;
    if (n > 0) TC_TRY(isect_blocks_per_cu(sh.kern, sh.lds_bytes, &per_cu));
    return TC_OK;
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
    const SchedCfg sc = sched_cfg(n, nnz, cfg);

    // mode checks and the launch shape come first: nothing below is timed
    // that is not device work
    const bool batch = cfg.gid != nullptr;
    const bool vertex = cfg.tv != nullptr;
    const bool edge = cfg.sup != nullptr;
    const bool cover = cfg.cover_lev != nullptr;
    if (edge && (!pb.pos0 || !pb.pos1 || !cfg.rp || !cfg.col)) return TC_ERR_ARG;
    const IsectShape sh = isect_shape(cfg);
    if (!sh.kern) return TC_ERR_ARG;
    const int table_ints = sh.table_ints;
    const size_t lds_bytes = sh.lds_bytes;
    int per_cu = 1;
    if (n > 0) TC_TRY(isect_blocks_per_cu(sh.kern, lds_bytes, &per_cu));
    if (getenv("TC_LOG")) fprintf(stderr, "libtc: k_isect %d blocks/CU, %zu B LDS\n", per_cu, lds_bytes);

    EventSet ev;
    if (cfg.timing) {
        TC_TRY(ev.create(3));
        TC_HIP_TRY(hipEventRecord(ev.e[0], s));
    }
    const int64_t nn = n > 0 ? n : 1;
    // zeroed by fill kernels (a captured graph records no memset nodes)
    TC_TRY(fill_u32(L.cnt, 0, 2 * nn, s));
    TC_TRY(fill_u32(L.work, 0, 4 * nn, s));
    TC_TRY(fill_u32(L.bucket_items, 0, kBuckets + 1, s));
    TC_TRY(fill_u32(L.bucket_cur, 0, kBuckets, s));
    TC_TRY(fill_u32(L.q, 0, kQueueBlockInts, s));
    TC_TRY(fill_u32(L.stats, 0, 32, s));
    if (cfg.tv && n > 0) TC_TRY(fill_u32(cfg.tv, 0, 2 * (int64_t)n, s));
    if (cfg.sup && nnz > 0) TC_TRY(fill_u32(cfg.sup, 0, nnz, s));
    const unsigned gp = (unsigned)di.cus * 8;
    // owner lists are sliced only when longer than a workgroup slice, and no
    // list is longer than nnz: below that, no search runs and no samples
    const bool sliced_lists = sc.wg_slicing && nnz > ((int64_t)1 << sc.wg_cap_log2);
    if (n > 0) {
        TC_TRY(tile_table_run(n, pb.rp0, L.tlo, L.thi, s));
        hipLaunchKernelGGL(k_own, dim3(gp), dim3(kThreads), 0, s, n, pb.e0x2, pb.rp0, pb.c0, pb.up0, pb.rp1, pb.vrec, L.cnt,
                           L.work, L.prec0, L.prec1, L.tlo, L.thi);
        TC_HIP_TRY(hipGetLastError());
        const unsigned gu = grid_for(2 * (int64_t)n, kItemThreads * kUnitsPerThread, (int64_t)1 << 30);
        hipLaunchKernelGGL((k_items<0>), dim3(gu), dim3(kItemThreads), 0, s, n, pb.rp0, pb.up0, pb.rp1, L.cnt,
                           L.work, sc, L.bucket_items, L.bucket_off, L.bucket_cur, L.items, L.stats, cfg.prof);
        TC_HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_bucket_order, dim3(1), dim3(1024), 0, s, L.bucket_items, sc, L.bucket_off, L.q);
        TC_HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL((k_items<1>), dim3(gu), dim3(kItemThreads), 0, s, n, pb.rp0, pb.up0, pb.rp1, L.cnt,
                           L.work, sc, L.bucket_items, L.bucket_off, L.bucket_cur, L.items, L.stats, nullptr);
        TC_HIP_TRY(hipGetLastError());
        if (sliced_lists) {
            const unsigned gs = grid_for(samples_of(nnz), 256, (int64_t)1 << 16);
            hipLaunchKernelGGL(k_samples, dim3(gs), dim3(256), 0, s, pb.c0, line_start(pb.c0), pb.e0x2, (int)kSmpC0,
                               nnz, L.s0);
            hipLaunchKernelGGL(k_samples, dim3(gs), dim3(256), 0, s, pb.c1, line_start(pb.c1), pb.e0x2,
                               cover ? (int)kSmpAll : (int)kSmpC1, nnz, L.s1);
            TC_HIP_TRY(hipGetLastError());
        }
    }
    if (cfg.timing) TC_HIP_TRY(hipEventRecord(ev.e[1], s));
    if (n > 0) {
        const unsigned gi = cfg.grid_blocks > 0 ? (unsigned)cfg.grid_blocks : (unsigned)(di.cus * per_cu);
        // byte offsets of list elements fit 32 bits below 2^30 entries (with
        // the padding)
        const int wide = nnz + 2 * kListPad + 1024 >= (int64_t(1) << 30) ? 1 : 0;
        Graph g{pb.rp0,       pb.c0,  pb.up0, pb.rp1, pb.c1, pb.vrec, L.prec0, L.prec1, pb.pos0, pb.pos1, wide,
                sliced_lists ? L.s0 : nullptr, sliced_lists ? L.s1 : nullptr, line_start(pb.c0), line_start(pb.c1)};
        const Sink sk{cfg.gid, cfg.batch_counts, cfg.tv, cfg.sup, cfg.cover_lev};
        if (cfg.prof && batch)
            hipLaunchKernelGGL((k_isect<true, kModeBatch>), dim3(gi), dim3(kIsectThreads), lds_bytes, s, g, L.items,
                               L.q, wg_log2, wave_log2, sc.wg_cap_log2, table_ints, L.stats + 8, cfg.prof, sk);
        else if (cfg.prof)
            hipLaunchKernelGGL((k_isect<true, kModePlain>), dim3(gi), dim3(kIsectThreads), lds_bytes, s, g, L.items,
                               L.q, wg_log2, wave_log2, sc.wg_cap_log2, table_ints, L.stats + 8, cfg.prof, sk);
        else if (vertex)
            hipLaunchKernelGGL((k_isect<false, kModeVertex>), dim3(gi), dim3(kIsectThreads), lds_bytes, s, g,
                               L.items, L.q, wg_log2, wave_log2, sc.wg_cap_log2, table_ints, L.stats + 8, nullptr, sk);
        else if (edge)
            hipLaunchKernelGGL((k_isect<false, kModeEdge>), dim3(gi), dim3(kIsectThreads), lds_bytes, s, g,
                               L.items, L.q, wg_log2, wave_log2, sc.wg_cap_log2, table_ints, L.stats + 8, nullptr, sk);
        else if (cover)
            hipLaunchKernelGGL((k_isect<false, kModeCover>), dim3(gi), dim3(kIsectThreads), lds_bytes, s, g,
                               L.items, L.q, wg_log2, wave_log2, sc.wg_cap_log2, table_ints, L.stats + 8, nullptr, sk);
        else if (batch)
            hipLaunchKernelGGL((k_isect<false, kModeBatch>), dim3(gi), dim3(kIsectThreads), lds_bytes, s, g,
                               L.items, L.q, wg_log2, wave_log2, sc.wg_cap_log2, table_ints, L.stats + 8, nullptr, sk);
        else
            hipLaunchKernelGGL((k_isect<false, kModePlain>), dim3(gi), dim3(kIsectThreads), lds_bytes, s, g,
                               L.items, L.q, wg_log2, wave_log2, sc.wg_cap_log2, table_ints, L.stats + 8, nullptr, sk);
        TC_HIP_TRY(hipGetLastError());
    }
    if (cfg.sup && nnz > 0) {
        hipLaunchKernelGGL(k_edge_mirror, dim3(gp), dim3(kThreads), 0, s, n, nnz, cfg.rp, cfg.col, cfg.sup);
        TC_HIP_TRY(hipGetLastError());
    }
    if (cfg.timing) TC_HIP_TRY(hipEventRecord(ev.e[2], s));
    if (cfg.result) {
        hipLaunchKernelGGL(k_result, dim3(1), dim3(64), 0, s, L.stats, pb.e0x2, cfg.result);
        TC_HIP_TRY(hipGetLastError());
    }
    if (!cfg.sync) return TC_OK;   // results stay on the device (captured pipelines)
    Mailbox mb;
    TC_TRY(mailbox(&mb));
    TC_TRY(mail_u64(reinterpret_cast<const uint64_t *>(L.stats), mb.dev, 16, s));
    TC_TRY(mail_u64(reinterpret_cast<const uint64_t *>(pb.e0x2), mb.dev + 16, 1, s));
    TC_HIP_TRY(hipStreamSynchronize(s));
    const uint64_t *h = mb.host;
    if (out) {
        out->e0x2 = (int64_t)h[16];
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
            TC_HIP_TRY(hipEventElapsedTime(&out->ms_bucket, ev.e[0], ev.e[1]));
            TC_HIP_TRY(hipEventElapsedTime(&out->ms_isect, ev.e[1], ev.e[2]));
        }
    }
    return TC_OK;
}

}  // namespace tc
