// Degree relabel: the degree ordering that the paper applies before its
// counting variants (Section III, last paragraph: vertices re-ordered by
// decreasing degree in Theta(n log n) time; BaderD and CED in the
// experiments).  New id i goes to the vertex of i-th largest degree, ties by
// increasing old id; the relabelled CSR has sorted rows.
//
// Two sorts with the library's radix sort: n vertex keys (n-1-deg, id), then
// the nnz entry keys (new row, new column).  Entries of new row i then sit
// exactly at [rp'[i], rp'[i+1]) since row i keeps its degree, so no
// duplicate removal or row counting is needed.
#include "tc_internal.hpp"

namespace tc {
namespace {

constexpr int kThreads = 256;
constexpr int kRun = 8;

unsigned grid_for(int64_t work, int threads) {
    int64_t g = (work + threads - 1) / threads;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (unsigned)g;
}

// key = (n-1-deg(v)) << bv | v: ascending keys list vertices by decreasing
// degree, ties by increasing id
__global__ void k_rl_vkeys(int32_t n, const int32_t *__restrict__ rp, int bv, uint64_t *__restrict__ keys) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int64_t deg = (int64_t)rp[v + 1] - rp[v];
        keys[v] = ((uint64_t)(n - 1 - deg) << bv) | (uint64_t)v;
    }
}

__global__ void k_rl_perm(int32_t n, const uint64_t *__restrict__ sorted, int bv, const int32_t *__restrict__ rp,
                          int32_t *__restrict__ perm, int32_t *__restrict__ inv, int32_t *__restrict__ ndeg) {
    const uint64_t vmask = (1ull << bv) - 1;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = (int32_t)(sorted[i] & vmask);
        perm[i] = v;
        inv[v] = (int32_t)i;
        ndeg[i] = rp[v + 1] - rp[v];
    }
}

// entry keys (inv[u] << bv | inv[v]); rows found per tile as in the other
// row passes
__global__ __launch_bounds__(kThreads) void k_rl_ekeys(int32_t n, int64_t nnz, const int32_t *__restrict__ rp,
                                                        const int32_t *__restrict__ col,
                                                        const int32_t *__restrict__ inv, int bv,
                                                        uint64_t *__restrict__ keys) {
    __shared__ int64_t rows[2];
    constexpr int64_t kTile = (int64_t)kThreads * kRun;
    for (int64_t t0 = (int64_t)blockIdx.x * kTile; t0 < nnz; t0 += (int64_t)gridDim.x * kTile) {
        tile_rows(rp, n, t0, t0 + kTile < nnz ? t0 + kTile : nnz, rows);
        const int64_t e0 = t0 + (int64_t)threadIdx.x * kRun;
        if (e0 < nnz) {
            const int64_t e1 = e0 + kRun < nnz ? e0 + kRun : nnz;
            int64_t u = row_of(rp, rows[0], rows[1], e0);
            int64_t ue = rp[u + 1];
            uint64_t nu = (uint64_t)inv[u] << bv;
            for (int64_t e = e0; e < e1; ++e) {
                while (e >= ue) {
                    ++u;
                    ue = rp[u + 1];
                    nu = (uint64_t)inv[u] << bv;
                }
                keys[e] = nu | (uint64_t)inv[col[e]];
            }
        }
        __syncthreads();   // rows is rewritten by the next tile
    }
}

__global__ void k_rl_col(int64_t nnz, const uint64_t *__restrict__ sorted, int bv, int32_t *__restrict__ out) {
    const uint64_t vmask = (1ull << bv) - 1;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nnz; j += (int64_t)gridDim.x * blockDim.x)
        out[j] = (int32_t)(sorted[j] & vmask);
}

struct RelabelLayout {
    uint64_t *ka, *kb;
    int32_t *inv, *ndeg;
    void *sort;
    size_t sort_bytes;
};

RelabelLayout carve_relabel(Carver &c, int32_t n, int64_t nnz) {
    RelabelLayout L;
    const int64_t nk = nnz > (int64_t)n ? nnz : (int64_t)n;
    L.ka = c.take<uint64_t>(nk > 0 ? nk : 1);
    L.kb = c.take<uint64_t>(nk > 0 ? nk : 1);
    L.inv = c.take<int32_t>(n > 0 ? n : 1);
    L.ndeg = c.take<int32_t>((int64_t)n + 1);
    L.sort_bytes = radix_sort_ws_bytes(nk + 1);
    L.sort = c.take<char>(L.sort_bytes);
    return L;
}

}  // namespace

size_t relabel_ws_bytes(int32_t n, int64_t nnz) {
    Carver c(nullptr, 0);
    carve_relabel(c, n, nnz);
    return c.used();
}

int relabel_run(int32_t n, int64_t nnz, const int32_t *rp, const int32_t *col, int32_t *out_rp, int32_t *out_col,
                int32_t *perm, void *ws, size_t ws_bytes, hipStream_t s) {
    Carver c(ws, ws_bytes);
    RelabelLayout L = carve_relabel(c, n, nnz);
    if (!c.fits()) return TC_ERR_WORKSPACE;
    if (n == 0) {
        TC_HIP_TRY(hipMemsetAsync(out_rp, 0, sizeof(int32_t), s));
        return TC_OK;
    }
    const int bv = bits_for_ids(n);
    hipLaunchKernelGGL(k_rl_vkeys, dim3(grid_for(n, 256)), dim3(256), 0, s, n, rp, bv, L.ka);
    TC_HIP_TRY(hipGetLastError());
    uint64_t *vs = nullptr;
    TC_TRY(radix_sort_u64(L.ka, L.kb, n, bv + bits_for_ids(n), L.sort, L.sort_bytes, s, &vs));
    hipLaunchKernelGGL(k_rl_perm, dim3(grid_for(n, 256)), dim3(256), 0, s, n, vs, bv, rp, perm, L.inv, L.ndeg);
    TC_HIP_TRY(hipGetLastError());
    TC_TRY(scan_exclusive_i32_to_i32(L.ndeg, out_rp, n, L.sort, s));
    if (nnz > 0) {
        const int64_t tiles = (nnz + (int64_t)kThreads * kRun - 1) / ((int64_t)kThreads * kRun);
        hipLaunchKernelGGL(k_rl_ekeys, dim3((unsigned)(tiles < 65536 ? tiles : 65536)), dim3(kThreads), 0, s, n, nnz,
                           rp, col, L.inv, bv, L.ka);
        TC_HIP_TRY(hipGetLastError());
        uint64_t *es = nullptr;
        TC_TRY(radix_sort_u64(L.ka, L.kb, nnz, 2 * bv, L.sort, L.sort_bytes, s, &es));
        hipLaunchKernelGGL(k_rl_col, dim3(grid_for(nnz, 256)), dim3(256), 0, s, nnz, es, bv, out_col);
        TC_HIP_TRY(hipGetLastError());
    }
    return TC_OK;
}

}  // namespace tc
