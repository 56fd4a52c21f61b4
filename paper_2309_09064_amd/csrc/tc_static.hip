// tc_count_noalloc: tc_count for callers that cannot allocate (code under
// graph capture, tight serving loops).  Its scratch is one file-scope device
// array per GPU instead of a caller workspace, and it runs with no host read:
// levels from the one-workgroup BFS kernel, then the partition, bucketing
// and intersection kernels of tc_count, the result written to the caller's
// device buffer by a kernel.
#include <mutex>

#include "tc_internal.hpp"

namespace tc {
namespace {

constexpr size_t kScratchBytes = size_t(256) << 20;

// The scratch of every call on this GPU.  Host code never passes this name
// to a kernel (on the host it is only a stand-in for the symbol): it uses
// the device address that hipGetSymbolAddress returns for it.
__device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// The scratch array's device address on the current device (looked up once
// per device, with that device current).
int scratch_ptr(void **out) {
    int dev = 0;
    TC_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return TC_ERR_NO_DEVICE;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        TC_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return TC_ERR_HIP;
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return TC_OK;
}

// Bytes the call needs: tc_count's buffers with its own levels (the BFS
// scratch shares the phases' scratch region: the BFS ends before the
// partition starts on the same stream).
size_t noalloc_bytes(int32_t n, int64_t nnz) {
    Carver c(nullptr, 0);
    carve_count_plan(c, n, nnz, true, false);
    return c.used();
}

int fail(int code) {
    set_error(code);
    return code;
}

}  // namespace
}  // namespace tc

using namespace tc;

extern "C" {

int tc_count_noalloc(int32_t n, int64_t nnz, const int32_t *d_row_ptr, const int32_t *d_col_idx,
                     const int32_t *d_levels, const tc_options *opt, uint64_t *d_result, void *stream) {
    if (n < 0 || nnz < 0 || !d_result) return fail(TC_ERR_ARG);
    if (nnz >= (int64_t(1) << 31)) return fail(TC_ERR_OVERFLOW);
    if ((n > 0 && !d_row_ptr) || (nnz > 0 && !d_col_idx) || (n == 0 && nnz > 0)) return fail(TC_ERR_ARG);
    CountCfg cfg;
    int flags = 0;
    int rc = options_cfg(opt, &cfg, &flags);
    if (rc != TC_OK) return fail(rc);
    if (flags & (TC_TIMING | TC_VALIDATE)) return fail(TC_ERR_ARG);   // both read results on the host
    if (cfg.schedule == TC_SCHED_TABLE && !cfg.table) return fail(TC_ERR_ARG);
    if (noalloc_bytes(n, nnz) > kScratchBytes) return fail(TC_ERR_TOO_LARGE);
    DeviceInfo di;
    rc = device_info(&di);
    if (rc != TC_OK) return fail(rc);
    void *base = nullptr;
    rc = scratch_ptr(&base);
    if (rc != TC_OK) return fail(rc);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (n == 0) return fail(fill_u32(d_result, 0, 8, s));
    Carver c(base, kScratchBytes);
    CountPlanBufs P = carve_count_plan(c, n, nnz, true, false);
    if (!c.fits() || P.scratch_bytes < bfs_single_ws_bytes(n)) return fail(TC_ERR_TOO_LARGE);
    const int32_t *lev = d_levels;
    if (!lev) {
        rc = bfs_single_run(n, d_row_ptr, d_col_idx, P.levels, P.scratch, P.scratch_bytes, s);
        if (rc != TC_OK) return fail(rc);
        lev = P.levels;
    }
    P.pb.by_id = cfg.orientation == TC_ORIENT_ID ? 1 : 0;
    rc = partition_run(n, nnz, d_row_ptr, d_col_idx, lev, P.pb, P.scratch, P.scratch_bytes, s);
    if (rc != TC_OK) return fail(rc);
    cfg.sync = false;
    cfg.result = reinterpret_cast<unsigned long long *>(d_result);
    return fail(count_run(n, nnz, P.pb, cfg, nullptr, P.scratch, P.scratch_bytes, s));
}

}  // extern "C"
