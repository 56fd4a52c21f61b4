// Partition of the edge set (Algorithm 4, partition loop) into horizontal
// edges E0 (equal levels) and the rest E1, compacted into two CSRs whose rows
// keep the input order:
//   N0(x) = [ neighbours y with L(y)=L(x) and rank(y) > rank(x) | the rest of
//             the equal-level neighbours ],   rank(y) = (deg(y), y);
//   N1(x) = neighbours y with L(y) != L(x).
// The rank-above part N0+(x) is the forward algorithm's oriented list
// (Algorithm 2 with degree ordering); with the id orientation rank(y) = y,
// Algorithm 2's own u < v.
//
// Two coalesced passes over the CSR entries.  Pass 1 marks each entry
// (horizontal, rank-above) into a byte, counts per row with atomics and per
// 2048-entry block.  Pass 2 turns block offsets plus an in-block scan into the
// number of horizontal / rank-above entries before every entry, which fixes
// its destination without any per-row cursor:
//   N1 entry at e     -> c1[e - H(e)]
//   N0+ entry at e    -> c0[rp0[x] + U(e) - rpu[x]]
//   other N0 entry    -> c0[H(e) - U(e) + rpu[x+1]]
// where H(e), U(e) count horizontal and rank-above entries before e and rpu is
// the prefix sum of |N0+|.
#include "tc_internal.hpp"

namespace tc {
namespace {

constexpr int kThreads = 256;
constexpr int kRun = 8;
constexpr int kBlockEntries = kThreads * kRun;
static_assert(kBlockEntries == kTileEntries, "a block is one tile of the tile table");
static_assert(kRun == 8, "runs are loaded by load_run8");
constexpr int kWaves = kThreads / kWave;
constexpr int kTileRowsMax = 1024;   // rows a tile may span and still count in LDS

// rank(y) > rank(x) with rank = (degree, id)
__device__ __forceinline__ bool rank_above(int32_t dy, int32_t y, int32_t x, int32_t dx) {
    return dy > dx || (dy == dx && y > x);
}

// {level, degree} of every vertex in one byte, so the marking pass gathers
// one byte per neighbour from an array of n bytes (a quarter of the levels'
// size, so more of it stays in L2): degree code << 2 | (level mod 4).
// Levels of adjacent vertices differ by at most one (BFS levels do;
// caller-given levels must), so two neighbours share a level exactly when
// their levels agree mod 4.  The degree code is monotone: the degree itself
// below 32, then 32 + floor(log2 d) - 5 (at most 57); when two codes differ
// they order the degrees, when they are equal below 32 the degrees are
// equal, and equal codes above that take the exact degree from the row
// pointers.
constexpr uint32_t kExactCodes = 32;
__device__ __forceinline__ uint32_t deg_code(int32_t d) {
    return d < (int32_t)kExactCodes ? (uint32_t)d : kExactCodes + (31u - __clz(d)) - 5u;
}
// The level parities also go into a bitmap of n bits (bit v of word v / 64),
// small enough to stay in every L2: the marking pass tests a neighbour's
// parity there first and gathers its byte record only for an equal-level
// neighbour under the degree rank, which needs its degree code.
__global__ void k_part_vld(int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ lev,
                           uint8_t *__restrict__ vld, uint64_t *__restrict__ par) {
    for (int64_t vb = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~(kWave - 1)); vb < n;
         vb += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = vb + lane_id();
        uint32_t l = 0;
        if (v < n) {
            l = (uint32_t)lev[v];
            vld[v] = (uint8_t)(deg_code(rp[v + 1] - rp[v]) << 2 | (l & 3u));
        }
        const uint64_t word = __ballot((l & 1u) != 0);
        if (lane_id() == 0) par[vb >> 6] = word;
    }
}

// rank_above with y's degree code cy from its record and x's exact degree dx.
__device__ __forceinline__ bool rank_above_rec(uint32_t cy, int32_t y, int32_t x, int32_t dx,
                                               const int32_t *__restrict__ rp) {
    const uint32_t cx = deg_code(dx);
    if (cy != cx) return cy > cx;
    if (cx < kExactCodes) return y > x;   // equal degrees
    return rank_above(rp[y + 1] - rp[y], y, x, dx);
}

__global__ __launch_bounds__(kThreads) void k_part_mark(int32_t n, int64_t nnz, const int32_t *__restrict__ rp,
                                                         const int32_t *__restrict__ col,
                                                         const uint8_t *__restrict__ vld,
                                                         const uint64_t *__restrict__ par,
                                                         const int32_t *__restrict__ tlo,
                                                         const int32_t *__restrict__ thi,
                                                         uint8_t *__restrict__ flags, int32_t *__restrict__ d0,
                                                         int32_t *__restrict__ up0, int32_t *__restrict__ bh,
                                                         int32_t *__restrict__ bu, int by_id) {
    __shared__ int32_t sh[kWaves], su[kWaves];
    __shared__ int32_t acc_h[kTileRowsMax], acc_u[kTileRowsMax];
    __shared__ int32_t s_rp[kTileRowsMax + 1];
    __shared__ uint8_t s_lv[kTileRowsMax];
    const int64_t t0 = (int64_t)blockIdx.x * kBlockEntries;
    const int64_t r_lo = tlo[blockIdx.x], r_hi = thi[blockIdx.x];
    const int64_t nr = r_hi - r_lo + 1;
    // rows of the tile are counted in LDS; only the two boundary rows can be
    // shared with other tiles.  Their row pointers and levels are staged in
    // LDS too: a thread's walk across row boundaries then waits on LDS, not
    // on one dependent global load per boundary.
    const bool local = nr <= kTileRowsMax;
    if (local) {
        for (int64_t i = threadIdx.x; i < nr; i += kThreads) {
            acc_h[i] = 0;
            acc_u[i] = 0;
            s_rp[i] = rp[r_lo + i];
            s_lv[i] = (uint8_t)(vld[r_lo + i] & 3u);
        }
        if (threadIdx.x == 0) s_rp[nr] = rp[r_hi + 1];
    }
    __syncthreads();
    auto rpx = [&](int64_t r) -> int64_t { return local ? (int64_t)s_rp[r - r_lo] : (int64_t)rp[r]; };
    auto lvx = [&](int64_t r) -> uint32_t { return local ? (uint32_t)s_lv[r - r_lo] : vld[r] & 3u; };
    const int64_t e0 = t0 + (int64_t)threadIdx.x * kRun;
    int32_t th = 0, tu = 0;
    if (e0 < nnz) {
        const int64_t e1 = e0 + kRun < nnz ? e0 + kRun : nnz;
        int64_t x = local ? r_lo + row_of(s_rp, 0, nr - 1, e0) : row_of(rp, r_lo, r_hi, e0);
        int64_t xe = rpx(x + 1);
        uint32_t lx = lvx(x);
        int32_t dx = (int32_t)(xe - rpx(x));
        int32_t ch = 0, cu = 0;
        auto flush = [&]() {
            if (local) {
                if (ch) atomicAdd(&acc_h[x - r_lo], ch);
                if (cu) atomicAdd(&acc_u[x - r_lo], cu);
            } else {
                if (ch) atomicAdd(&d0[x], ch);
                if (cu) atomicAdd(&up0[x], cu);
            }
            ch = cu = 0;
        };
        // the run's neighbour ids, their level parities, then the records
        // of the equal-parity ones, all issued before the row walk: three
        // memory latencies per thread instead of three per entry.  The
        // parity of row x decides which records are needed: the run's rows
        // all lie in [x, row of e1 - 1], and a row change only matters for
        // entries past it, whose records are then gathered in the walk.
        int32_t y[kRun];
        uint32_t py[kRun], iy[kRun];
        load_run8(col, e0, e1, y);
#pragma unroll
        for (int k = 0; k < kRun; ++k)
            py[k] = e0 + k < e1 ? (uint32_t)(par[(uint32_t)y[k] >> 6] >> (y[k] & 63)) & 1u : 2u;
#pragma unroll
        for (int k = 0; k < kRun; ++k) iy[k] = 0u;
        if (!by_id) {
#pragma unroll
            for (int k = 0; k < kRun; ++k)
                if (py[k] == (lx & 1u)) iy[k] = (uint32_t)vld[y[k]];
        }
        uint8_t f[kRun];
#pragma unroll
        for (int k = 0; k < kRun; ++k) f[k] = 0;
#pragma unroll
        for (int k = 0; k < kRun; ++k) {
            const int64_t e = e0 + k;
            if (e < e1) {
                while (e >= xe) {
                    flush();
                    ++x;
                    const int64_t xb = xe;
                    xe = rpx(x + 1);
                    lx = lvx(x);
                    dx = (int32_t)(xe - xb);
                }
                const bool hor = py[k] == (lx & 1u);
                bool up = false;
                if (hor) {
                    if (by_id) {
                        up = y[k] > (int32_t)x;
                    } else {
                        // not prefetched (the row changed parity since):
                        // gather now; a neighbour's record is never 0, its
                        // degree being at least one
                        if (iy[k] == 0u) iy[k] = (uint32_t)vld[y[k]];
                        up = rank_above_rec(iy[k] >> 2, y[k], (int32_t)x, dx, rp);
                    }
                }
                f[k] = (uint8_t)(hor | (up << 1));
                ch += hor;
                cu += up;
            }
        }
        flush();
        uint64_t word = 0;
#pragma unroll
        for (int k = 0; k < kRun; ++k) {
            word |= (uint64_t)f[k] << (8 * k);
            th += f[k] & 1;
            tu += f[k] >> 1;
        }
        if (e1 - e0 == kRun) {
            *reinterpret_cast<uint64_t *>(flags + e0) = word;   // e0 is a multiple of 8
        } else {
#pragma unroll
            for (int k = 0; k < kRun; ++k)
                if (e0 + k < e1) flags[e0 + k] = f[k];
        }
    }
    th = wave_sum(th);
    tu = wave_sum(tu);
    if (lane_id() == 0) { sh[threadIdx.x / kWave] = th; su[threadIdx.x / kWave] = tu; }
    __syncthreads();
    if (local) {
        for (int64_t i = threadIdx.x; i < nr; i += kThreads) {
            const int64_t r = r_lo + i;
            const int32_t h = acc_h[i], u = acc_u[i];
            if (r == r_lo || r == r_hi) {
                if (h) atomicAdd(&d0[r], h);
                if (u) atomicAdd(&up0[r], u);
            } else {
                d0[r] = h;
                up0[r] = u;
            }
        }
    }
    if (threadIdx.x == 0) {
        int32_t a = 0, b = 0;
        for (int i = 0; i < kWaves; ++i) { a += sh[i]; b += su[i]; }
        bh[blockIdx.x] = a;
        bu[blockIdx.x] = b;
    }
}

// Per-vertex record of the partition {rp0, |N0+|, rp1, |N1|}: the counting
// kernels read one 16-byte record per partner instead of three words.
__global__ void k_part_vrec(int32_t n, const int32_t *__restrict__ rp0, const int32_t *__restrict__ up0,
                            const int32_t *__restrict__ rp1, int4 *__restrict__ vrec) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x)
        vrec[x] = make_int4(rp0[x], up0[x], rp1[x], rp1[x + 1] - rp1[x]);
}

__global__ void k_part_rp1(int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ rp0,
                           int32_t *__restrict__ rp1, int64_t *__restrict__ e0x2) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x <= n; x += (int64_t)gridDim.x * blockDim.x)
        rp1[x] = rp[x] - rp0[x];
    if (e0x2 && blockIdx.x == 0 && threadIdx.x == 0) *e0x2 = rp0[n];
}

// kPos also records, for every c0 / c1 entry, the input entry it came from
// (per-edge counts add to input entries).  The block's N1 entries fill one
// run of c1 (entry e goes to e - H(e)): they are gathered in LDS and leave
// in consecutive stores instead of one 4-byte store per entry spread over
// the wavefront's 2 KB of input.
template <bool kPos>
__global__ __launch_bounds__(kThreads) void k_part_scatter(int32_t n, int64_t nnz, const int32_t *__restrict__ rp,
                                                            const int32_t *__restrict__ col,
                                                            const int32_t *__restrict__ tlo,
                                                            const int32_t *__restrict__ thi,
                                                            const uint8_t *__restrict__ flags,
                                                            const int32_t *__restrict__ bh_off,
                                                            const int32_t *__restrict__ bu_off,
                                                            const int32_t *__restrict__ rp0,
                                                            const int32_t *__restrict__ rpu,
                                                            int32_t *__restrict__ c0, int32_t *__restrict__ c1,
                                                            int32_t *__restrict__ pos0, int32_t *__restrict__ pos1) {
    __shared__ int64_t wsum[kWaves];
    __shared__ int32_t s_rp[kTileRowsMax + 1], s_ub[kTileRowsMax], s_lb[kTileRowsMax];
    __shared__ int32_t s_c1[kBlockEntries], s_p1[kPos ? kBlockEntries : 1];
    const int64_t t0 = (int64_t)blockIdx.x * kBlockEntries;
    // the tile's row pointers and per-row targets staged in LDS (made
    // visible by the scan's barrier below): the walk across row boundaries
    // then waits on LDS, not on dependent global loads
    const int64_t r_lo = tlo[blockIdx.x], r_hi = thi[blockIdx.x];
    const int64_t nr = r_hi - r_lo + 1;
    const bool local = nr <= kTileRowsMax;
    if (local) {
        for (int64_t i = threadIdx.x; i < nr; i += kThreads) {
            const int64_t r = r_lo + i;
            s_rp[i] = rp[r];
            s_ub[i] = rp0[r] - rpu[r];
            s_lb[i] = rpu[r + 1];
        }
        if (threadIdx.x == 0) s_rp[nr] = rp[r_hi + 1];
    }
    const int64_t e0 = t0 + (int64_t)threadIdx.x * kRun;
    const int64_t e1 = e0 < nnz ? (e0 + kRun < nnz ? e0 + kRun : nnz) : e0;
    uint8_t f[kRun];
    int64_t packed = 0;   // horizontal count << 32 | rank-above count
    uint64_t word = 0;
    if (e1 - e0 == kRun) {
        word = *reinterpret_cast<const uint64_t *>(flags + e0);
    } else {
#pragma unroll
        for (int k = 0; k < kRun; ++k)
            if (e0 + k < e1) word |= (uint64_t)flags[e0 + k] << (8 * k);
    }
#pragma unroll
    for (int k = 0; k < kRun; ++k) {
        f[k] = (uint8_t)(word >> (8 * k));
        packed += ((int64_t)(f[k] & 1) << 32) | (int64_t)(f[k] >> 1);
    }
    // block exclusive scan of the packed counts
    int64_t inc = wave_incl_scan(packed);
    const int w = threadIdx.x / kWave;
    if (lane_id() == kWave - 1) wsum[w] = inc;
    __syncthreads();
    int64_t before = inc - packed;
    int64_t blk = 0;   // the block's horizontal entries
    for (int i = 0; i < kWaves; ++i) {
        if (i < w) before += wsum[i];
        blk += wsum[i] >> 32;
    }
    const int64_t hb = bh_off[blockIdx.x];   // horizontal entries before the block
    const int64_t nblk = (t0 + kBlockEntries < nnz ? t0 + kBlockEntries : nnz) - t0;
    if (e0 < e1) {
        int64_t H = hb + (before >> 32);
        int64_t U = (int64_t)bu_off[blockIdx.x] + (before & 0xffffffffll);
        int32_t y[kRun];   // issued before the row walk
        load_run8(col, e0, e1, y);
        auto rpx = [&](int64_t r) -> int64_t { return local ? (int64_t)s_rp[r - r_lo] : (int64_t)rp[r]; };
        // N0+ entries of row x go to rp0[x] + (U - rpu[x]), the rest of its
        // horizontal entries to H - U + rpu[x + 1]: two per-row terms
        auto upb = [&](int64_t r) -> int64_t { return local ? (int64_t)s_ub[r - r_lo] : (int64_t)rp0[r] - rpu[r]; };
        auto lob = [&](int64_t r) -> int64_t { return local ? (int64_t)s_lb[r - r_lo] : (int64_t)rpu[r + 1]; };
        int64_t x = local ? r_lo + row_of(s_rp, 0, nr - 1, e0) : row_of(rp, r_lo, r_hi, e0);
        int64_t xe = rpx(x + 1);
        int64_t up_base = upb(x), lo_base = lob(x);
#pragma unroll
        for (int k = 0; k < kRun; ++k) {
            const int64_t e = e0 + k;
            if (e < e1) {
                if (e >= xe) {
                    do { ++x; xe = rpx(x + 1); } while (e >= xe);
                    up_base = upb(x);
                    lo_base = lob(x);
                }
                const uint8_t fe = f[k];
                if (fe & 1) {
                    const int64_t d = (fe & 2) ? up_base + U : H - U + lo_base;
                    c0[d] = y[k];
                    if (kPos) pos0[d] = (int32_t)e;
                } else {
                    const int64_t i = (e - t0) - (H - hb);   // place in the block's run of c1
                    s_c1[i] = y[k];
                    if (kPos) s_p1[i] = (int32_t)e;
                }
                H += fe & 1;
                U += fe >> 1;
            }
        }
    }
    __syncthreads();
    const int64_t n1 = nblk - blk, d1 = t0 - hb;   // the run: c1[d1, d1 + n1)
    for (int64_t i = threadIdx.x; i < n1; i += kThreads) {
        c1[d1 + i] = s_c1[i];
        if (kPos) pos1[d1 + i] = s_p1[i];
    }
}

struct PartLayout {
    int32_t *tlo, *thi;   // tile table of the input CSR
    uint8_t *vld;
    uint64_t *par;        // level parity, one bit per vertex
    uint8_t *flags;
    int32_t *bh, *bu;
    void *scan;
};

PartLayout carve_part(Carver &c, int32_t n, int64_t nnz) {
    PartLayout L;
    const int64_t nblk = (nnz + kBlockEntries - 1) / kBlockEntries;
    L.tlo = c.take<int32_t>(tiles_of(nnz));
    L.thi = c.take<int32_t>(tiles_of(nnz));
    L.vld = c.take<uint8_t>(n > 0 ? n : 1);
    L.par = c.take<uint64_t>(n > 0 ? ((int64_t)n + 63) / 64 : 1);
    L.flags = c.take<uint8_t>(nnz > 0 ? nnz : 1);
    L.bh = c.take<int32_t>(nblk + 1);
    L.bu = c.take<int32_t>(nblk + 1);
    int64_t big = (int64_t)n + 1 > nblk ? (int64_t)n + 1 : nblk;
    L.scan = c.take<char>(scan_ws_bytes(big));
    return L;
}

unsigned grid_for(int64_t work, int threads) {
    int64_t g = (work + threads - 1) / threads;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (unsigned)g;
}

}  // namespace

size_t partition_ws_bytes(int32_t n, int64_t nnz) {
    Carver c(nullptr, 0);
    carve_part(c, n, nnz);
    return c.used();
}

int partition_run(int32_t n, int64_t nnz, const int32_t *rp, const int32_t *col, const int32_t *lev,
                  const PartBufs &pb, void *ws, size_t ws_bytes, hipStream_t s) {
    Carver c(ws, ws_bytes);
    PartLayout L = carve_part(c, n, nnz);
    if (!c.fits()) return TC_ERR_WORKSPACE;
    TC_TRY(fill_u32(pb.d0, 0, n > 0 ? n : 1, s));
    TC_TRY(fill_u32(pb.up0, 0, n > 0 ? n : 1, s));
    const int64_t nblk = (nnz + kBlockEntries - 1) / kBlockEntries;
    if (nnz > 0) {
        TC_TRY(tile_table_run(n, rp, L.tlo, L.thi, s));
        hipLaunchKernelGGL(k_part_vld, dim3(grid_for(n, 256)), dim3(256), 0, s, n, rp, lev, L.vld, L.par);
        hipLaunchKernelGGL(k_part_mark, dim3((unsigned)nblk), dim3(kThreads), 0, s, n, nnz, rp, col, L.vld, L.par, L.tlo,
                           L.thi, L.flags, pb.d0, pb.up0, L.bh, L.bu, pb.by_id);
        TC_HIP_TRY(hipGetLastError());
    }
    TC_TRY(scan_exclusive_i32_to_i32(pb.d0, pb.rp0, n, L.scan, s));
    TC_TRY(scan_exclusive_i32_to_i32(pb.up0, pb.rpu, n, L.scan, s));
    hipLaunchKernelGGL(k_part_rp1, dim3(grid_for((int64_t)n + 1, 256)), dim3(256), 0, s, n, rp, pb.rp0, pb.rp1,
                       pb.e0x2);
    TC_HIP_TRY(hipGetLastError());
    if (pb.vrec) {
        hipLaunchKernelGGL(k_part_vrec, dim3(grid_for(n, 256)), dim3(256), 0, s, n, pb.rp0, pb.up0, pb.rp1, pb.vrec);
        TC_HIP_TRY(hipGetLastError());
    }
    if (nnz > 0) {
        TC_TRY(scan_exclusive_i32_to_i32(L.bh, L.bh, nblk, L.scan, s));
        TC_TRY(scan_exclusive_i32_to_i32(L.bu, L.bu, nblk, L.scan, s));
        if (pb.pos0)
            hipLaunchKernelGGL(k_part_scatter<true>, dim3((unsigned)nblk), dim3(kThreads), 0, s, n, nnz, rp, col,
                               L.tlo, L.thi, L.flags, L.bh, L.bu, pb.rp0, pb.rpu, pb.c0, pb.c1, pb.pos0, pb.pos1);
        else
            hipLaunchKernelGGL(k_part_scatter<false>, dim3((unsigned)nblk), dim3(kThreads), 0, s, n, nnz, rp, col,
                               L.tlo, L.thi, L.flags, L.bh, L.bu, pb.rp0, pb.rpu, pb.c0, pb.c1, nullptr, nullptr);
        TC_HIP_TRY(hipGetLastError());
    }
    return TC_OK;
}

}  // namespace tc
