// Cost network of the learned schedule: initialisation, forward pass,
// gradient, Adam and the per-bucket strategy choice.
//
// Not part of the paper's method: the network only decides which exact
// intersection kernel counts a bucket of work, so it never changes a count.
//
//   a1 = relu(W1 x + b1),  a2 = relu(W2 a1 + b2),  y = W3 a2 + b3
//
// Parameters are float32, row-major, W1[H][3] b1[H] W2[H][H] b2[H] W3[K][H]
// b3[K].  The data sets are small (one row per profiled bucket and strategy,
// a few thousand rows), so the kernels favour simplicity and determinism:
// one thread per row for the per-row passes, one thread per parameter for
// the sums over rows, which run in a fixed order in float64.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "tc_internal.hpp"

namespace tc {
namespace {

constexpr int kMaxK = 8;
constexpr int kIn = TC_MLP_IN;
constexpr int kRowThreads = 256;

struct Net {
    int H, K;
    int64_t oW1, ob1, oW2, ob2, oW3, ob3, P;
};

Net net_of(int H, int K) {
    Net n;
    n.H = H;
    n.K = K;
    n.oW1 = 0;
    n.ob1 = n.oW1 + (int64_t)H * kIn;
    n.oW2 = n.ob1 + H;
    n.ob2 = n.oW2 + (int64_t)H * H;
    n.oW3 = n.ob2 + H;
    n.ob3 = n.oW3 + (int64_t)K * H;
    n.P = n.ob3 + K;
    return n;
}

bool valid_hk(int H, int K) { return (H == 8 || H == 16 || H == 32 || H == 64) && K >= 1 && K <= kMaxK; }

// Copies the parameters into LDS (every thread of the block then reads the
// same addresses: broadcasts).
__device__ __forceinline__ void load_params(float *sp, const float *__restrict__ params, int64_t P) {
    for (int64_t i = threadIdx.x; i < P; i += blockDim.x) sp[i] = params[i];
    __syncthreads();
}

// Forward pass of one row.  relu'(z) = [z > 0] = [a > 0], so backward needs
// only the activations.
template <int H>
__device__ __forceinline__ void forward_row(const float *sp, const Net &n, const float (&x)[kIn], float (&a1)[H],
                                            float (&a2)[H], float (&y)[kMaxK]) {
    const float *W1 = sp + n.oW1, *b1 = sp + n.ob1, *W2 = sp + n.oW2, *b2 = sp + n.ob2;
    const float *W3 = sp + n.oW3, *b3 = sp + n.ob3;
#pragma unroll
    for (int j = 0; j < H; ++j) {
        float z = b1[j];
#pragma unroll
        for (int q = 0; q < kIn; ++q) z += W1[j * kIn + q] * x[q];
        a1[j] = z > 0.f ? z : 0.f;
    }
#pragma unroll
    for (int i = 0; i < H; ++i) {
        float z = b2[i];
#pragma unroll
        for (int j = 0; j < H; ++j) z += W2[i * H + j] * a1[j];
        a2[i] = z > 0.f ? z : 0.f;
    }
#pragma unroll
    for (int k = 0; k < kMaxK; ++k) {
        float v = 0.f;
        if (k < n.K) {
            v = b3[k];
#pragma unroll
            for (int i = 0; i < H; ++i) v += W3[k * H + i] * a2[i];
        }
        y[k] = v;
    }
}

// ---------------------------------------------------------------- init

__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t index) {
    // the (index + 1)-th output of SplitMix64 started at `seed`
    uint64_t z = seed + (index + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void k_mlp_init(float *__restrict__ params, Net n, uint64_t seed, float s1, float s2, float s3) {
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n.P) return;
    float scale = 0.f;
    if (i < n.ob1) scale = s1;
    else if (i >= n.oW2 && i < n.ob2) scale = s2;
    else if (i >= n.oW3 && i < n.ob3) scale = s3;
    float w = 0.f;
    if (scale != 0.f) {
        const float u = (float)(splitmix64_at(seed, (uint64_t)i) >> 40) * 0x1.0p-24f;   // exact
        const float d = 2.f * u - 1.f;                                                  // exact
        w = d * scale;                                                                  // one rounding
    }
    params[i] = w;
}

// ---------------------------------------------------------------- forward

template <int H>
__global__ __launch_bounds__(kRowThreads) void k_mlp_forward(const float *__restrict__ params, Net n,
                                                               const float *__restrict__ X, int32_t rows,
                                                               float *__restrict__ Y) {
    extern __shared__ float sp[];
    load_params(sp, params, n.P);
    const int32_t r = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (r >= rows) return;
    const float x[kIn] = {X[3 * (int64_t)r], X[3 * (int64_t)r + 1], X[3 * (int64_t)r + 2]};
    float a1[H], a2[H], y[kMaxK];
    forward_row<H>(sp, n, x, a1, a2, y);
#pragma unroll
    for (int k = 0; k < kMaxK; ++k)
        if (k < n.K) Y[(int64_t)r * n.K + k] = y[k];
}

// ---------------------------------------------------------------- gradient

// Per row: a1, a2, dz1, dz2 (H each), dy at the measured output, the row's
// loss term, all before the division by the total weight W (applied to the
// sums).  Row stride 4H + 2 floats.
template <int H>
__global__ __launch_bounds__(kRowThreads) void k_mlp_rows(const float *__restrict__ params, Net n,
                                                            const float *__restrict__ X,
                                                            const int32_t *__restrict__ C,
                                                            const float *__restrict__ Tgt,
                                                            const float *__restrict__ Wt, int32_t rows,
                                                            float *__restrict__ rowbuf) {
    extern __shared__ float sp[];
    load_params(sp, params, n.P);
    const int32_t r = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (r >= rows) return;
    const float x[kIn] = {X[3 * (int64_t)r], X[3 * (int64_t)r + 1], X[3 * (int64_t)r + 2]};
    float a1[H], a2[H], y[kMaxK];
    forward_row<H>(sp, n, x, a1, a2, y);
    // a row whose strategy index lies outside [0, K) contributes nothing
    const int c0 = C[r];
    const bool live = c0 >= 0 && c0 < n.K;
    const int c = live ? c0 : 0;
    float yc = 0.f;
#pragma unroll
    for (int k = 0; k < kMaxK; ++k) yc = k == c ? y[k] : yc;
    const float res = live ? yc - Tgt[r] : 0.f;
    const float w = Wt ? Wt[r] : 1.f;
    const float dyc = w * res;
    const float *W2 = sp + n.oW2, *W3 = sp + n.oW3;
    float dz2[H];
#pragma unroll
    for (int i = 0; i < H; ++i) dz2[i] = a2[i] > 0.f ? W3[c * H + i] * dyc : 0.f;
    float *o = rowbuf + (int64_t)r * (4 * H + 2);
#pragma unroll
    for (int j = 0; j < H; ++j) {
        float da = 0.f;
#pragma unroll
        for (int i = 0; i < H; ++i) da += W2[i * H + j] * dz2[i];
        o[2 * H + j] = a1[j] > 0.f ? da : 0.f;   // dz1
    }
#pragma unroll
    for (int j = 0; j < H; ++j) {
        o[j] = a1[j];
        o[H + j] = a2[j];
        o[3 * H + j] = dz2[j];
    }
    o[4 * H] = dyc;
    o[4 * H + 1] = 0.5f * w * res * res;
}

// One thread per parameter (plus one for the loss): its sum over all rows,
// in row order, in float64, divided by the total weight W (the row count
// when there are no weights).
__global__ __launch_bounds__(kRowThreads) void k_mlp_sums(Net n, const float *__restrict__ X,
                                                            const int32_t *__restrict__ C,
                                                            const float *__restrict__ Wt, int32_t rows,
                                                            const float *__restrict__ rowbuf,
                                                            float *__restrict__ grad, float *__restrict__ loss) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p > n.P) return;
    const int H = n.H;
    const int64_t S = 4 * H + 2;
    double wsum = rows;
    if (Wt) {
        wsum = 0.0;
        for (int32_t r = 0; r < rows; ++r) wsum += Wt[r];
    }
    double acc = 0.0;
    if (p == n.P) {
        for (int32_t r = 0; r < rows; ++r) acc += (double)rowbuf[r * S + 4 * H + 1];
        if (loss) loss[0] = (float)(acc / wsum);
        return;
    }
    if (p < n.ob1) {                       // W1[j][q] = sum dz1[j] x[q]
        const int j = (int)(p / kIn), q = (int)(p % kIn);
        for (int32_t r = 0; r < rows; ++r) acc += (double)rowbuf[r * S + 2 * H + j] * X[3 * (int64_t)r + q];
    } else if (p < n.oW2) {                // b1[j] = sum dz1[j]
        const int j = (int)(p - n.ob1);
        for (int32_t r = 0; r < rows; ++r) acc += rowbuf[r * S + 2 * H + j];
    } else if (p < n.ob2) {                // W2[i][j] = sum dz2[i] a1[j]
        const int i = (int)((p - n.oW2) / H), j = (int)((p - n.oW2) % H);
        for (int32_t r = 0; r < rows; ++r) acc += (double)rowbuf[r * S + 3 * H + i] * rowbuf[r * S + j];
    } else if (p < n.oW3) {                // b2[i] = sum dz2[i]
        const int i = (int)(p - n.ob2);
        for (int32_t r = 0; r < rows; ++r) acc += rowbuf[r * S + 3 * H + i];
    } else if (p < n.ob3) {                // W3[k][i] = sum over rows measuring k of dy a2[i]
        const int k = (int)((p - n.oW3) / H), i = (int)((p - n.oW3) % H);
        for (int32_t r = 0; r < rows; ++r)
            if (C[r] == k) acc += (double)rowbuf[r * S + 4 * H] * rowbuf[r * S + H + i];
    } else {                               // b3[k] = sum over rows measuring k of dy
        const int k = (int)(p - n.ob3);
        for (int32_t r = 0; r < rows; ++r)
            if (C[r] == k) acc += rowbuf[r * S + 4 * H];
    }
    grad[p] = (float)(acc / wsum);
}

// ---------------------------------------------------------------- Adam

__global__ void k_mlp_adam(float *__restrict__ params, const float *__restrict__ grad, float *__restrict__ m,
                           float *__restrict__ v, int64_t count, float lr, float beta1, float beta2, float eps,
                           float inv_bc1, float inv_bc2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float g = grad[i];
    const float mi = beta1 * m[i] + (1.f - beta1) * g;
    const float vi = beta2 * v[i] + (1.f - beta2) * g * g;
    m[i] = mi;
    v[i] = vi;
    params[i] -= lr * (mi * inv_bc1) / (sqrtf(vi * inv_bc2) + eps);
}

// ---------------------------------------------------------------- schedule

template <int H>
__global__ __launch_bounds__(kRowThreads) void k_mlp_schedule(const float *__restrict__ params, Net n,
                                                                int wave_ob_max, int32_t *__restrict__ table,
                                                                float *__restrict__ cost) {
    extern __shared__ float sp[];
    load_params(sp, params, n.P);
    const int b = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (b >= TC_NUM_BUCKETS) return;
    const int kind = b >> 10, ob = (b >> 5) & 31, pb = b & 31;
    const float x[kIn] = {(float)ob, (float)pb, (float)kind};
    float a1[H], a2[H], y[kMaxK];
    forward_row<H>(sp, n, x, a1, a2, y);
    int best = TC_STRAT_BSEARCH;
    float best_y = y[TC_STRAT_BSEARCH];
#pragma unroll
    for (int k = 0; k < TC_NUM_STRATEGIES; ++k) {
        const bool feasible = k == TC_STRAT_WAVE_HASH ? ob <= wave_ob_max : true;
        if (feasible && (y[k] < best_y || (y[k] == best_y && k < best))) {
            best = k;
            best_y = y[k];
        }
    }
    table[b] = best;
    if (cost) {
#pragma unroll
        for (int k = 0; k < kMaxK; ++k)
            if (k < n.K) cost[(int64_t)b * n.K + k] = y[k];
    }
}

int ilog2i(int v) {
    int k = 0;
    while ((1 << (k + 1)) <= v) ++k;
    return k;
}

template <template <int> class Launch, class... A>
int by_hidden(int H, A... a) {
    switch (H) {
        case 8: return Launch<8>::run(a...);
        case 16: return Launch<16>::run(a...);
        case 32: return Launch<32>::run(a...);
        default: return Launch<64>::run(a...);
    }
}

template <int H>
struct LaunchForward {
    static int run(const float *params, Net n, const float *X, int32_t rows, float *Y, hipStream_t s) {
        const unsigned g = (unsigned)((rows + kRowThreads - 1) / kRowThreads);
        hipLaunchKernelGGL(k_mlp_forward<H>, dim3(g), dim3(kRowThreads), n.P * sizeof(float), s, params, n, X, rows,
                           Y);
        TC_HIP_TRY(hipGetLastError());
        return TC_OK;
    }
};

template <int H>
struct LaunchRows {
    static int run(const float *params, Net n, const float *X, const int32_t *C, const float *T, const float *W,
                   int32_t rows, float *rowbuf, hipStream_t s) {
        const unsigned g = (unsigned)((rows + kRowThreads - 1) / kRowThreads);
        hipLaunchKernelGGL(k_mlp_rows<H>, dim3(g), dim3(kRowThreads), n.P * sizeof(float), s, params, n, X, C, T,
                           W, rows, rowbuf);
        TC_HIP_TRY(hipGetLastError());
        return TC_OK;
    }
};

template <int H>
struct LaunchSchedule {
    static int run(const float *params, Net n, int wave_ob_max, int32_t *table, float *cost, hipStream_t s) {
        const unsigned g = (unsigned)((TC_NUM_BUCKETS + kRowThreads - 1) / kRowThreads);
        hipLaunchKernelGGL(k_mlp_schedule<H>, dim3(g), dim3(kRowThreads), n.P * sizeof(float), s, params, n,
                           wave_ob_max, table, cost);
        TC_HIP_TRY(hipGetLastError());
        return TC_OK;
    }
};

size_t rowbuf_bytes(int H, int32_t rows) { return (size_t)rows * (4 * H + 2) * sizeof(float); }

int grad_run(const float *params, Net n, const float *X, const int32_t *C, const float *T, const float *W,
             int32_t rows, float *grad, float *loss, float *rowbuf, hipStream_t s) {
    TC_TRY(by_hidden<LaunchRows>(n.H, params, n, X, C, T, W, rows, rowbuf, s));
    const unsigned g = (unsigned)((n.P + 1 + kRowThreads - 1) / kRowThreads);
    hipLaunchKernelGGL(k_mlp_sums, dim3(g), dim3(kRowThreads), 0, s, n, X, C, W, rows, rowbuf, grad, loss);
    TC_HIP_TRY(hipGetLastError());
    return TC_OK;
}

int adam_run(float *params, const float *grad, float *m, float *v, int64_t count, int32_t step, float lr,
             float beta1, float beta2, float eps, hipStream_t s) {
    // bias corrections in float64 on the host, applied as reciprocals
    const float inv_bc1 = (float)(1.0 / (1.0 - pow((double)beta1, (double)step)));
    const float inv_bc2 = (float)(1.0 / (1.0 - pow((double)beta2, (double)step)));
    const unsigned g = (unsigned)((count + 255) / 256);
    hipLaunchKernelGGL(k_mlp_adam, dim3(g), dim3(256), 0, s, params, grad, m, v, count, lr, beta1, beta2, eps,
                       inv_bc1, inv_bc2);
    TC_HIP_TRY(hipGetLastError());
    return TC_OK;
}

bool adam_args_ok(int32_t step, float lr, float beta1, float beta2, float eps) {
    return step >= 1 && lr > 0.f && beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps >= 0.f;
}

int ret(int code) {
    set_error(code);
    return code;
}

}  // namespace
}  // namespace tc

using namespace tc;

extern "C" {

int tc_mlp_param_count(int32_t hidden, int32_t k, int64_t *h_count) {
    if (!h_count || !valid_hk(hidden, k)) return ret(TC_ERR_ARG);
    *h_count = net_of(hidden, k).P;
    return ret(TC_OK);
}

int tc_mlp_init(float *d_params, int32_t hidden, int32_t k, uint64_t seed, void *stream) {
    if (!d_params || !valid_hk(hidden, k)) return ret(TC_ERR_ARG);
    DeviceInfo di;
    int rc = device_info(&di);
    if (rc != TC_OK) return ret(rc);
    const Net n = net_of(hidden, k);
    const float s1 = (float)sqrt(6.0 / kIn), s2 = (float)sqrt(6.0 / hidden), s3 = s2;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_mlp_init, dim3((unsigned)((n.P + 255) / 256)), dim3(256), 0, s, d_params, n, seed, s1, s2,
                       s3);
    if (hipGetLastError() != hipSuccess) return ret(TC_ERR_HIP);
    return ret(TC_OK);
}

int tc_mlp_forward(const float *d_params, int32_t hidden, int32_t k, const float *d_x, int32_t rows, float *d_y,
                   void *stream) {
    if (!valid_hk(hidden, k) || rows < 0) return ret(TC_ERR_ARG);
    if (rows == 0) return ret(TC_OK);
    if (!d_params || !d_x || !d_y) return ret(TC_ERR_ARG);
    DeviceInfo di;
    int rc = device_info(&di);
    if (rc != TC_OK) return ret(rc);
    return ret(by_hidden<LaunchForward>(hidden, d_params, net_of(hidden, k), d_x, rows, d_y,
                                        static_cast<hipStream_t>(stream)));
}

int tc_mlp_grad_ws(int32_t hidden, int32_t k, int32_t rows, size_t *h_ws_bytes) {
    if (!h_ws_bytes || !valid_hk(hidden, k) || rows < 1) return ret(TC_ERR_ARG);
    Carver c(nullptr, 0);
    c.take<char>(rowbuf_bytes(hidden, rows));
    *h_ws_bytes = c.used();
    return ret(TC_OK);
}

int tc_mlp_grad(const float *d_params, int32_t hidden, int32_t k, const float *d_x, const int32_t *d_c,
                const float *d_t, const float *d_w, int32_t rows, float *d_grad, float *d_loss, void *ws,
                size_t ws_bytes, void *stream) {
    if (!valid_hk(hidden, k) || rows < 1) return ret(TC_ERR_ARG);
    if (!d_params || !d_x || !d_c || !d_t || !d_grad) return ret(TC_ERR_ARG);
    Carver c(ws, ws_bytes);
    float *rowbuf = c.take<float>(rowbuf_bytes(hidden, rows) / sizeof(float));
    if (!ws || !c.fits() || ((uintptr_t)ws & 255) != 0) return ret(TC_ERR_WORKSPACE);
    DeviceInfo di;
    int rc = device_info(&di);
    if (rc != TC_OK) return ret(rc);
    return ret(grad_run(d_params, net_of(hidden, k), d_x, d_c, d_t, d_w, rows, d_grad, d_loss, rowbuf,
                        static_cast<hipStream_t>(stream)));
}

int tc_mlp_adam(float *d_params, const float *d_grad, float *d_m, float *d_v, int64_t count, int32_t step, float lr,
                float beta1, float beta2, float eps, void *stream) {
    if (count < 0 || !adam_args_ok(step, lr, beta1, beta2, eps)) return ret(TC_ERR_ARG);
    if (count == 0) return ret(TC_OK);
    if (!d_params || !d_grad || !d_m || !d_v) return ret(TC_ERR_ARG);
    DeviceInfo di;
    int rc = device_info(&di);
    if (rc != TC_OK) return ret(rc);
    return ret(adam_run(d_params, d_grad, d_m, d_v, count, step, lr, beta1, beta2, eps,
                        static_cast<hipStream_t>(stream)));
}

int tc_mlp_train_ws(int32_t hidden, int32_t k, int32_t rows, size_t *h_ws_bytes) {
    if (!h_ws_bytes || !valid_hk(hidden, k) || rows < 1) return ret(TC_ERR_ARG);
    Carver c(nullptr, 0);
    c.take<char>(rowbuf_bytes(hidden, rows));
    c.take<float>((size_t)net_of(hidden, k).P);
    *h_ws_bytes = c.used();
    return ret(TC_OK);
}

int tc_mlp_train(float *d_params, float *d_m, float *d_v, int32_t hidden, int32_t k, const float *d_x,
                 const int32_t *d_c, const float *d_t, const float *d_w, int32_t rows, int32_t first_step,
                 int32_t steps, float lr,
                 float beta1, float beta2, float eps, float *d_loss, void *ws, size_t ws_bytes, void *stream) {
    if (!valid_hk(hidden, k) || rows < 1 || steps < 0) return ret(TC_ERR_ARG);
    if (!adam_args_ok(first_step, lr, beta1, beta2, eps)) return ret(TC_ERR_ARG);
    if ((int64_t)first_step + steps > INT32_MAX) return ret(TC_ERR_ARG);
    if (!d_params || !d_m || !d_v || !d_x || !d_c || !d_t) return ret(TC_ERR_ARG);
    const Net n = net_of(hidden, k);
    Carver c(ws, ws_bytes);
    float *rowbuf = c.take<float>(rowbuf_bytes(hidden, rows) / sizeof(float));
    float *grad = c.take<float>((size_t)n.P);
    if (!ws || !c.fits() || ((uintptr_t)ws & 255) != 0) return ret(TC_ERR_WORKSPACE);
    DeviceInfo di;
    int rc = device_info(&di);
    if (rc != TC_OK) return ret(rc);
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int32_t i = 0; i < steps; ++i) {
        rc = grad_run(d_params, n, d_x, d_c, d_t, d_w, rows, grad, d_loss ? d_loss + i : nullptr, rowbuf, s);
        if (rc != TC_OK) return ret(rc);
        rc = adam_run(d_params, grad, d_m, d_v, n.P, first_step + i, lr, beta1, beta2, eps, s);
        if (rc != TC_OK) return ret(rc);
    }
    return ret(TC_OK);
}

int tc_mlp_schedule(const float *d_params, int32_t hidden, int32_t k, const tc_options *opt, int32_t *d_table,
                    float *d_cost, void *stream) {
    if (!valid_hk(hidden, k) || k != TC_NUM_STRATEGIES || !d_params || !d_table) return ret(TC_ERR_ARG);
    CountCfg cfg;
    int flags;
    int rc = options_cfg(opt, &cfg, &flags);
    if (rc != TC_OK) return ret(rc);
    DeviceInfo di;
    rc = device_info(&di);
    if (rc != TC_OK) return ret(rc);
    const int wave_ob_max = ilog2i(cfg.wave_slots) - 2;
    return ret(by_hidden<LaunchSchedule>(hidden, d_params, net_of(hidden, k), wave_ob_max, d_table, d_cost,
                                         static_cast<hipStream_t>(stream)));
}

}  // extern "C"
