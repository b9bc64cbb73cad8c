// Training side of the process-rate surrogate: float32 forward, backward
// (masked mean squared error) and Adam for the 12-128-128-128-12 SiLU
// network, normalisation statistics, parameter I/O and checkpoints.
//
// All reductions run in a fixed order (split-K partial sums reduced in
// split order, tree reductions in fixed shape), so a training run is
// bitwise reproducible for a given seed and batch order.
#include <math.h>
#include <string.h>

#include <vector>

#include "casim_internal.h"
#include "casim_mlp_internal.h"

namespace casim {

// ---- tiled float32 GEMM ------------------------------------------------------
// C[M x N] = op(A)[M x K] * op(B)[K x N], row-major; op transposes when TA/TB.
// Epilogues: store, bias + SiLU (z and a = silu(z) stored), bias only,
// multiply by silu'(Z) (backward through an activation), split-K partials.
enum Epi { EPI_STORE = 0, EPI_BIAS_SILU = 1, EPI_BIAS = 2, EPI_DSILU = 3 };

constexpr int GBM = 64, GBN = 64, GBK = 16;

__device__ __forceinline__ float sigm(float z) { return 1.0f / (1.0f + expf(-z)); }

template <bool TA, bool TB>
__global__ __launch_bounds__(256) void gemm_kernel(const float *__restrict__ A, int lda,
                                                   const float *__restrict__ B, int ldb,
                                                   float *__restrict__ C, int ldc, int M, int N, int K,
                                                   int epi, const float *__restrict__ bias,
                                                   float *__restrict__ C2, const float *__restrict__ Z,
                                                   int ksplit) {
    __shared__ float As[GBK][GBM + 4];
    __shared__ float Bs[GBK][GBN + 4];
    const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
    const int m0 = blockIdx.y * GBM, n0 = blockIdx.x * GBN;
    // split-K range of this block
    const int kper = (K + ksplit - 1) / ksplit;
    const int kb = blockIdx.z * kper, ke = min(K, kb + kper);
    float acc[4][4] = {};
    for (int k0 = kb; k0 < ke; k0 += GBK) {
        for (int e = tid; e < GBM * GBK; e += 256) {
            int mm, kk;
            if (TA) { mm = e % GBM; kk = e / GBM; } else { kk = e % GBK; mm = e / GBK; }
            const int gm = m0 + mm, gk = k0 + kk;
            float v = 0.0f;
            if (gm < M && gk < ke) v = TA ? A[(size_t)gk * lda + gm] : A[(size_t)gm * lda + gk];
            As[kk][mm] = v;
        }
        for (int e = tid; e < GBN * GBK; e += 256) {
            int nn, kk;
            if (TB) { kk = e % GBK; nn = e / GBK; } else { nn = e % GBN; kk = e / GBN; }
            const int gn = n0 + nn, gk = k0 + kk;
            float v = 0.0f;
            if (gn < N && gk < ke) v = TB ? B[(size_t)gn * ldb + gk] : B[(size_t)gk * ldb + gn];
            Bs[kk][nn] = v;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < GBK; ++kk) {
            float a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[kk][ty * 4 + i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx * 4 + j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
    float *Cz = C + (size_t)blockIdx.z * M * ldc;   // split-K partial slab (ksplit > 1)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int gm = m0 + ty * 4 + i;
        if (gm >= M) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int gn = n0 + tx * 4 + j;
            if (gn >= N) continue;
            float v = acc[i][j];
            const size_t o = (size_t)gm * ldc + gn;
            if (epi == EPI_BIAS_SILU) {
                v += bias[gn];
                C[o] = v;
                C2[o] = v * sigm(v);
            } else if (epi == EPI_BIAS) {
                C[o] = v + bias[gn];
            } else if (epi == EPI_DSILU) {
                const float z = Z[o], s = sigm(z);
                C[o] = v * (s * (1.0f + z * (1.0f - s)));
            } else {
                Cz[o] = v;
            }
        }
    }
}

// out[i] = sum over s of part[s][i], in split order.
__global__ void reduce_splits(const float *part, int nsplit, int64_t n, float *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = 0.0f;
    for (int k = 0; k < nsplit; ++k) s += part[(size_t)k * n + i];
    out[i] = s;
}

// Column sums of X (rows x cols) in a fixed order: one block per column.
__global__ __launch_bounds__(256) void colsum_kernel(const float *X, int rows, int cols, float *out) {
    __shared__ float red[256];
    const int c = blockIdx.x;
    float s = 0.0f;
    for (int r = threadIdx.x; r < rows; r += 256) s += X[(size_t)r * cols + c];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = red[0];
}

// Gather batch rows: xb[b] = x[idx[b]] (idx NULL: row b).
__global__ void gather_rows(const float *x, const float *y, const float *m, const int32_t *idx, int batch,
                            float *xb, float *yb, float *mb) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= batch * 12) return;
    const int b = i / 12, j = i % 12;
    const int64_t r = idx ? (int64_t)idx[b] : b;
    xb[i] = x[r * 12 + j];
    yb[i] = y[r * 12 + j];
    mb[i] = m[r * 12 + j];
}

// dY = 2 m (yhat - y) / max(1, sum m); per-block partial losses.  Single
// block per call, fixed order (batch <= CASIM_MLP_MAX_BATCH).
__global__ __launch_bounds__(256) void loss_kernel(const float *yh, const float *y, const float *m, int n,
                                                   float *dy, float *loss_out) {
    __shared__ float red[256];
    __shared__ float msum_s;
    float s = 0.0f;
    for (int i = threadIdx.x; i < n; i += 256) s += m[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) msum_s = fmaxf(1.0f, red[0]);
    __syncthreads();
    const float inv = 1.0f / msum_s;
    float l = 0.0f;
    for (int i = threadIdx.x; i < n; i += 256) {
        const float d = yh[i] - y[i];
        dy[i] = 2.0f * m[i] * d * inv;
        l += m[i] * d * d;
    }
    __syncthreads();
    red[threadIdx.x] = l;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0 && loss_out) loss_out[0] = red[0] * inv;
}

__global__ void adam_kernel(float *theta, float *mo, float *ve, const float *g, int n, float lr, float bc1,
                            float bc2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float gi = g[i];
    const float m = b1 * mo[i] + (1.0f - b1) * gi;
    const float v = b2 * ve[i] + (1.0f - b2) * gi * gi;
    mo[i] = m;
    ve[i] = v;
    theta[i] -= lr * (m / bc1) / (sqrtf(v / bc2) + eps);
}

__global__ void init_params_kernel(float *theta, uint64_t seed) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kMlpParams) return;
    // fan-in / fan-out of the layer this index belongs to; biases start at 0
    int fi = 0, fo = 0;
    bool bias = false;
    if (i < kOB1) { fi = 12; fo = 128; }
    else if (i < kOW2) bias = true;
    else if (i < kOB2) { fi = 128; fo = 128; }
    else if (i < kOW3) bias = true;
    else if (i < kOB3) { fi = 128; fo = 128; }
    else if (i < kOW4) bias = true;
    else if (i < kOB4) { fi = 128; fo = 12; }
    else bias = true;
    if (bias) { theta[i] = 0.0f; return; }
    const double lim = sqrt(6.0 / (fi + fo));
    theta[i] = (float)((2.0 * hash_uniform(seed, (uint64_t)i) - 1.0) * lim);
}

// ---- statistics ---------------------------------------------------------------
// Per-feature sum, sum of squares, min and max: one block per feature, fixed
// reduction order.  out[j*4 + 0..3].
__global__ __launch_bounds__(256) void stats_features(const float *feat, int64_t n, double *out) {
    __shared__ double r0[256], r1[256], r2[256], r3[256];
    const int c = blockIdx.x;
    double s = 0, ss = 0, mn = 1e300, mx = -1e300;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        const double v = feat[i * 12 + c];
        s += v; ss += v * v; mn = fmin(mn, v); mx = fmax(mx, v);
    }
    r0[threadIdx.x] = s; r1[threadIdx.x] = ss; r2[threadIdx.x] = mn; r3[threadIdx.x] = mx;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            r0[threadIdx.x] += r0[threadIdx.x + w];
            r1[threadIdx.x] += r1[threadIdx.x + w];
            r2[threadIdx.x] = fmin(r2[threadIdx.x], r2[threadIdx.x + w]);
            r3[threadIdx.x] = fmax(r3[threadIdx.x], r3[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[c * 4 + 0] = r0[0]; out[c * 4 + 1] = r1[0]; out[c * 4 + 2] = r2[0]; out[c * 4 + 3] = r3[0];
    }
}

// Scaled training target of rate j: asinh(rate / scale), of the magnitude for
// the two deposition rates (DEPI, DEPS), whose sign the gate word carries
// (bit 12: supersaturated over ice) and inference restores.
__device__ __forceinline__ double scaled_target(double rate, int j) {
    return asinh((j == 3 || j == 4 ? fabs(rate) : rate) * kRateScaleInv);
}

// Per-target count, sum and sum of squares of the scaled target over the
// samples whose gate is open: one block per target.  out[j*4 + 0..2].
__global__ __launch_bounds__(256) void stats_targets(const float *rates, const uint16_t *gates, int64_t n,
                                                     double *out) {
    __shared__ double r0[256], r1[256], r2[256];
    const int j = blockIdx.x;
    double cnt = 0, s = 0, ss = 0;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        if (!((gates[i] >> j) & 1u)) continue;
        const double v = scaled_target((double)rates[i * 12 + j], j);
        cnt += 1.0; s += v; ss += v * v;
    }
    r0[threadIdx.x] = cnt; r1[threadIdx.x] = s; r2[threadIdx.x] = ss;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            r0[threadIdx.x] += r0[threadIdx.x + w];
            r1[threadIdx.x] += r1[threadIdx.x + w];
            r2[threadIdx.x] += r2[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) { out[j * 4 + 0] = r0[0]; out[j * 4 + 1] = r1[0]; out[j * 4 + 2] = r2[0]; }
}

// Covariance of standardised features: one block per (a, b) pair, a <= b.
__global__ __launch_bounds__(256) void stats_cov(const float *feat, int64_t n, const float *mean,
                                                 const float *sd, double *cov) {
    __shared__ double red[256];
    int a = 0, b = blockIdx.x;
    while (b >= 12 - a) { b -= 12 - a; ++a; }
    b += a;
    double s = 0;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        const double za = (feat[i * 12 + a] - mean[a]) / sd[a];
        const double zb = (feat[i * 12 + b] - mean[b]) / sd[b];
        s += za * zb;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double v = red[0] / (double)(n > 1 ? n - 1 : 1);
        cov[a * 12 + b] = v;
        cov[b * 12 + a] = v;
    }
}

// Histogram of log10 of the squared Mahalanobis distance |W z|^2 (4096 bins
// over [-6, 6)), integer counts, for the 99.9th percentile.
__global__ __launch_bounds__(256) void stats_maha_hist(const float *feat, int64_t n, const float *mean,
                                                       const float *sd, const float *whiten,
                                                       unsigned long long *hist) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float z[12];
#pragma unroll
    for (int j = 0; j < 12; ++j) z[j] = (feat[i * 12 + j] - mean[j]) / sd[j];
    float d2 = 0.0f;
#pragma unroll
    for (int a = 0; a < 12; ++a) {
        float t = 0.0f;
#pragma unroll
        for (int b = 0; b <= a; ++b) t = fmaf(whiten[a * 12 + b], z[b], t);
        d2 = fmaf(t, t, d2);
    }
    const double l = log10(fmax((double)d2, 1e-6));
    int bin = (int)floor((l + 6.0) / 12.0 * 4096.0);
    bin = bin < 0 ? 0 : (bin > 4095 ? 4095 : bin);
    atomicAdd(&hist[bin], 1ull);
}

__global__ void prepare_kernel(const float *feat, const float *rates, const uint16_t *gates, int64_t n,
                               const float *st /* casim_mlp_stats */, float *x, float *y, float *m) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * 12) return;
    const int64_t p = i / 12;
    const int j = (int)(i % 12);
    const casim_mlp_stats *S = reinterpret_cast<const casim_mlp_stats *>(st);
    x[i] = (feat[i] - S->x_mean[j]) / S->x_std[j];
    const bool open = (gates[p] >> j) & 1u;
    m[i] = open ? 1.0f : 0.0f;
    y[i] = open ? ((float)scaled_target((double)rates[i], j) - S->y_mean[j]) / S->y_std[j] : 0.0f;
}

// ---- host side -------------------------------------------------------------------
namespace {

struct MlpCtx {
    bool have_params = false, have_stats = false;
    int device = -1;
    float *theta = nullptr, *mo = nullptr, *ve = nullptr, *grad = nullptr, *loss = nullptr;
    float *stats_dev = nullptr;
    int64_t step = 0;
    casim_mlp_stats stats{};
    // training scratch (CASIM_MLP_MAX_BATCH rows)
    float *xb = nullptr, *yb = nullptr, *mb = nullptr, *z1, *a1, *z2, *a2, *z3, *a3, *yh, *dy, *d1, *d2;
    float *part = nullptr;
};
MlpCtx M;

hipError_t ensure_alloc() {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (M.theta && M.device == dev) return hipSuccess;
    const size_t np = kMlpParams * sizeof(float);
    const size_t B = CASIM_MLP_MAX_BATCH;
    float **bufs[] = {&M.theta, &M.mo, &M.ve, &M.grad};
    for (float **b : bufs)
        if ((e = hipMalloc(b, np)) != hipSuccess) return e;
    if ((e = hipMalloc(&M.loss, 64)) != hipSuccess) return e;
    if ((e = hipMalloc(&M.stats_dev, sizeof(casim_mlp_stats))) != hipSuccess) return e;
    float **small[] = {&M.xb, &M.yb, &M.mb, &M.yh, &M.dy};
    for (float **b : small)
        if ((e = hipMalloc(b, B * 12 * sizeof(float))) != hipSuccess) return e;
    float **big[] = {&M.z1, &M.a1, &M.z2, &M.a2, &M.z3, &M.a3, &M.d1, &M.d2};
    for (float **b : big)
        if ((e = hipMalloc(b, B * 128 * sizeof(float))) != hipSuccess) return e;
    if ((e = hipMalloc(&M.part, (size_t)kMaxSplit * 128 * 128 * sizeof(float))) != hipSuccess) return e;
    M.device = dev;
    return hipSuccess;
}

template <bool TA, bool TB>
hipError_t gemm(const float *A, int lda, const float *B, int ldb, float *C, int ldc, int Mr, int N, int K,
                int epi, const float *bias, float *C2, const float *Z, hipStream_t s, int ksplit = 1) {
    dim3 grid((N + GBN - 1) / GBN, (Mr + GBM - 1) / GBM, ksplit);
    hipLaunchKernelGGL((gemm_kernel<TA, TB>), grid, dim3(256), 0, s, A, lda, B, ldb, C, ldc, Mr, N, K, epi,
                       bias, C2, Z, ksplit);
    return hipGetLastError();
}

// Weight gradient dW (K_in x N) = Aᵀ (B x K_in)ᵀ dZ (B x N), split over the
// batch, partials reduced in split order.
hipError_t weight_grad(const float *Ain, int kin, const float *dZ, int n, int batch, float *out, hipStream_t s) {
    int split = (batch + 63) / 64;
    split = split < 1 ? 1 : (split > kMaxSplit ? kMaxSplit : split);
    hipError_t e = gemm<true, false>(Ain, kin, dZ, n, M.part, n, kin, n, batch, EPI_STORE, nullptr, nullptr,
                                     nullptr, s, split);
    if (e != hipSuccess) return e;
    const int64_t tot = (int64_t)kin * n;
    hipLaunchKernelGGL(reduce_splits, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, M.part, split, tot, out);
    return hipGetLastError();
}

// Forward pass on rows xb (batch x 12); activations kept for backward.
hipError_t forward(const float *x, int batch, float *yout, hipStream_t s) {
    const float *T = M.theta;
    hipError_t e;
    if ((e = gemm<false, false>(x, 12, T + kOW1, 128, M.z1, 128, batch, 128, 12, EPI_BIAS_SILU, T + kOB1, M.a1, nullptr, s))) return e;
    if ((e = gemm<false, false>(M.a1, 128, T + kOW2, 128, M.z2, 128, batch, 128, 128, EPI_BIAS_SILU, T + kOB2, M.a2, nullptr, s))) return e;
    if ((e = gemm<false, false>(M.a2, 128, T + kOW3, 128, M.z3, 128, batch, 128, 128, EPI_BIAS_SILU, T + kOB3, M.a3, nullptr, s))) return e;
    return gemm<false, false>(M.a3, 128, T + kOW4, 12, yout, 12, batch, 12, 128, EPI_BIAS, T + kOB4, nullptr, nullptr, s);
}

hipError_t backward(int batch, float *g, hipStream_t s) {
    const float *T = M.theta;
    hipError_t e;
    // output layer
    if ((e = weight_grad(M.a3, 128, M.dy, 12, batch, g + kOW4, s))) return e;
    hipLaunchKernelGGL(colsum_kernel, dim3(12), dim3(256), 0, s, M.dy, batch, 12, g + kOB4);
    // dZ3 = (dY W4ᵀ) * silu'(Z3)
    if ((e = gemm<false, true>(M.dy, 12, T + kOW4, 12, M.d1, 128, batch, 128, 12, EPI_DSILU, nullptr, nullptr, M.z3, s))) return e;
    if ((e = weight_grad(M.a2, 128, M.d1, 128, batch, g + kOW3, s))) return e;
    hipLaunchKernelGGL(colsum_kernel, dim3(128), dim3(256), 0, s, M.d1, batch, 128, g + kOB3);
    if ((e = gemm<false, true>(M.d1, 128, T + kOW3, 128, M.d2, 128, batch, 128, 128, EPI_DSILU, nullptr, nullptr, M.z2, s))) return e;
    if ((e = weight_grad(M.a1, 128, M.d2, 128, batch, g + kOW2, s))) return e;
    hipLaunchKernelGGL(colsum_kernel, dim3(128), dim3(256), 0, s, M.d2, batch, 128, g + kOB2);
    if ((e = gemm<false, true>(M.d2, 128, T + kOW2, 128, M.d1, 128, batch, 128, 128, EPI_DSILU, nullptr, nullptr, M.z1, s))) return e;
    if ((e = weight_grad(M.xb, 12, M.d1, 128, batch, g + kOW1, s))) return e;
    hipLaunchKernelGGL(colsum_kernel, dim3(128), dim3(256), 0, s, M.d1, batch, 128, g + kOB1);
    return hipGetLastError();
}

hipError_t loss_and_grad(const float *x, const float *y, const float *m, const int32_t *idx, int batch,
                         float *g, float *loss, hipStream_t s) {
    hipLaunchKernelGGL(gather_rows, dim3((batch * 12 + 255) / 256), dim3(256), 0, s, x, y, m, idx, batch,
                       M.xb, M.yb, M.mb);
    hipError_t e = forward(M.xb, batch, M.yh, s);
    if (e) return e;
    hipLaunchKernelGGL(loss_kernel, dim3(1), dim3(256), 0, s, M.yh, M.yb, M.mb, batch * 12, M.dy, loss);
    return backward(batch, g, s);
}

}  // namespace

const float *mlp_params_device() { return M.have_params ? M.theta : nullptr; }
const casim_mlp_stats *mlp_stats_host() { return M.have_stats ? &M.stats : nullptr; }

}  // namespace casim

using namespace casim;

namespace {
int fail(hipError_t e) { return casim_record_hip_error((int)e, hipGetErrorString(e)); }
}
#define MLP_TRY(x)                               \
    do {                                         \
        hipError_t e_ = (x);                     \
        if (e_ != hipSuccess) return fail(e_);   \
    } while (0)

extern "C" {

int casim_mlp_init(uint64_t seed) {
    MLP_TRY(ensure_alloc());
    hipLaunchKernelGGL(init_params_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, 0, M.theta, seed);
    MLP_TRY(hipGetLastError());
    MLP_TRY(hipMemset(M.mo, 0, kMlpParams * sizeof(float)));
    MLP_TRY(hipMemset(M.ve, 0, kMlpParams * sizeof(float)));
    MLP_TRY(hipDeviceSynchronize());
    M.step = 0;
    M.have_params = true;
    return CASIM_OK;
}

int casim_mlp_get_params(float *host_params) {
    if (!host_params) return CASIM_EINVAL;
    if (!M.have_params) return CASIM_ENOSURROGATE;
    MLP_TRY(hipDeviceSynchronize());
    MLP_TRY(hipMemcpy(host_params, M.theta, kMlpParams * sizeof(float), hipMemcpyDeviceToHost));
    return CASIM_OK;
}

int casim_mlp_set_params(const float *host_params) {
    if (!host_params) return CASIM_EINVAL;
    MLP_TRY(ensure_alloc());
    MLP_TRY(hipDeviceSynchronize());
    MLP_TRY(hipMemcpy(M.theta, host_params, kMlpParams * sizeof(float), hipMemcpyHostToDevice));
    MLP_TRY(hipMemset(M.mo, 0, kMlpParams * sizeof(float)));
    MLP_TRY(hipMemset(M.ve, 0, kMlpParams * sizeof(float)));
    M.step = 0;
    M.have_params = true;
    return CASIM_OK;
}

int casim_mlp_grad(const float *x, const float *y, const float *m, const int32_t *idx, int32_t batch,
                   float *grad, float *loss, void *stream) {
    if (!x || !y || !m || !grad || !loss || batch < 1 || batch > CASIM_MLP_MAX_BATCH) return CASIM_EINVAL;
    if (!M.have_params) return CASIM_ENOSURROGATE;
    MLP_TRY(loss_and_grad(x, y, m, idx, batch, grad, loss, (hipStream_t)stream));
    return CASIM_OK;
}

int casim_mlp_train_step(const float *x, const float *y, const float *m, const int32_t *idx, int32_t batch,
                         float lr, float *loss, void *stream) {
    if (!x || !y || !m || batch < 1 || batch > CASIM_MLP_MAX_BATCH || !(lr > 0.0f) || !isfinite(lr))
        return CASIM_EINVAL;
    if (!M.have_params) return CASIM_ENOSURROGATE;
    hipStream_t s = (hipStream_t)stream;
    MLP_TRY(loss_and_grad(x, y, m, idx, batch, M.grad, loss ? loss : M.loss, s));
    M.step += 1;
    const float bc1 = (float)(1.0 - pow(0.9, (double)M.step));
    const float bc2 = (float)(1.0 - pow(0.999, (double)M.step));
    hipLaunchKernelGGL(adam_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, M.theta, M.mo, M.ve,
                       M.grad, kMlpParams, lr, bc1, bc2);
    MLP_TRY(hipGetLastError());
    return CASIM_OK;
}

int casim_mlp_forward(const float *x, int64_t n, float *y, void *stream) {
    if (!x || !y || n < 0) return CASIM_EINVAL;
    if (!M.have_params) return CASIM_ENOSURROGATE;
    hipStream_t s = (hipStream_t)stream;
    for (int64_t o = 0; o < n; o += CASIM_MLP_MAX_BATCH) {
        const int b = (int)((n - o) < CASIM_MLP_MAX_BATCH ? (n - o) : CASIM_MLP_MAX_BATCH);
        MLP_TRY(forward(x + o * 12, b, y + o * 12, s));
    }
    return CASIM_OK;
}

int casim_mlp_set_stats(const casim_mlp_stats *st) {
    if (!st) return CASIM_EINVAL;
    for (int j = 0; j < 12; ++j)
        if (!(st->x_std[j] > 0.0f) || !(st->y_std[j] > 0.0f)) return CASIM_EINVAL;
    for (int i = 0; i < 12; ++i)            // the whitening factor is lower triangular
        for (int j = i + 1; j < 12; ++j)
            if (st->whiten[i * 12 + j] != 0.0f) return CASIM_EINVAL;
    MLP_TRY(ensure_alloc());
    MLP_TRY(hipDeviceSynchronize());
    M.stats = *st;
    MLP_TRY(hipMemcpy(M.stats_dev, &M.stats, sizeof M.stats, hipMemcpyHostToDevice));
    M.have_stats = true;
    return CASIM_OK;
}

int casim_mlp_fit_stats(const float *feat, const float *rates, const uint16_t *gates, int64_t n,
                        casim_mlp_stats *out, void *stream) {
    if (!feat || !rates || !gates || !out || n < 2) return CASIM_EINVAL;
    MLP_TRY(ensure_alloc());
    hipStream_t s = (hipStream_t)stream;
    double *d_mom = nullptr, *d_cov = nullptr;
    float *d_mean = nullptr, *d_sd = nullptr, *d_cinv = nullptr;
    unsigned long long *d_hist = nullptr;
    MLP_TRY(hipMalloc(&d_mom, 24 * 4 * sizeof(double)));
    MLP_TRY(hipMalloc(&d_cov, 144 * sizeof(double)));
    MLP_TRY(hipMalloc(&d_mean, 3 * 144 * sizeof(float)));
    d_sd = d_mean + 144;
    d_cinv = d_sd + 144;
    MLP_TRY(hipMalloc(&d_hist, 4096 * sizeof(unsigned long long)));
    hipLaunchKernelGGL(stats_features, dim3(12), dim3(256), 0, s, feat, n, d_mom);
    hipLaunchKernelGGL(stats_targets, dim3(12), dim3(256), 0, s, rates, gates, n, d_mom + 48);
    double mom[96];
    MLP_TRY(hipMemcpyAsync(mom, d_mom, sizeof mom, hipMemcpyDeviceToHost, s));
    MLP_TRY(hipStreamSynchronize(s));
    casim_mlp_stats st{};
    for (int j = 0; j < 12; ++j) {
        const double mean = mom[j * 4 + 0] / n;
        const double var = fmax(mom[j * 4 + 1] / n - mean * mean, 0.0);
        st.x_mean[j] = (float)mean;
        st.x_std[j] = (float)fmax(sqrt(var), 1e-6);
        st.x_min[j] = (float)mom[j * 4 + 2];
        st.x_max[j] = (float)mom[j * 4 + 3];
        const double cnt = mom[48 + j * 4 + 0];
        const double ym = cnt > 0 ? mom[48 + j * 4 + 1] / cnt : 0.0;
        const double yv = cnt > 0 ? fmax(mom[48 + j * 4 + 2] / cnt - ym * ym, 0.0) : 1.0;
        st.y_mean[j] = (float)ym;
        st.y_std[j] = (float)fmax(sqrt(yv), 1e-3);
    }
    MLP_TRY(hipMemcpyAsync(d_mean, st.x_mean, 12 * sizeof(float), hipMemcpyHostToDevice, s));
    MLP_TRY(hipMemcpyAsync(d_sd, st.x_std, 12 * sizeof(float), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(stats_cov, dim3(78), dim3(256), 0, s, feat, n, d_mean, d_sd, d_cov);
    double cov[144];
    MLP_TRY(hipMemcpyAsync(cov, d_cov, sizeof cov, hipMemcpyDeviceToHost, s));
    MLP_TRY(hipStreamSynchronize(s));
    // Cholesky factor L of C + 1e-9 I and W = L^-1 (12 x 12, host, binary64)
    double L[12][12] = {}, Wd[12][12] = {};
    for (int i = 0; i < 12; ++i)
        for (int j = 0; j <= i; ++j) {
            double v = cov[i * 12 + j] + (i == j ? 1e-9 : 0.0);
            for (int k = 0; k < j; ++k) v -= L[i][k] * L[j][k];
            if (i == j) {
                if (!(v > 0.0)) return CASIM_EINVAL;
                L[i][i] = sqrt(v);
            } else {
                L[i][j] = v / L[j][j];
            }
        }
    for (int j = 0; j < 12; ++j) {          // forward substitution, column j of L^-1
        for (int i = j; i < 12; ++i) {
            double v = i == j ? 1.0 : 0.0;
            for (int k = j; k < i; ++k) v -= L[i][k] * Wd[k][j];
            Wd[i][j] = v / L[i][i];
        }
    }
    for (int i = 0; i < 12; ++i)
        for (int j = 0; j < 12; ++j) st.whiten[i * 12 + j] = (float)Wd[i][j];
    MLP_TRY(hipMemcpyAsync(d_cinv, st.whiten, sizeof st.whiten, hipMemcpyHostToDevice, s));
    MLP_TRY(hipMemsetAsync(d_hist, 0, 4096 * sizeof(unsigned long long), s));
    hipLaunchKernelGGL(stats_maha_hist, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, feat, n, d_mean, d_sd,
                       d_cinv, d_hist);
    std::vector<unsigned long long> hist(4096);
    MLP_TRY(hipMemcpyAsync(hist.data(), d_hist, 4096 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    MLP_TRY(hipStreamSynchronize(s));
    unsigned long long acc = 0, need = (unsigned long long)ceil(0.999 * (double)n);
    int bin = 4095;
    for (int b = 0; b < 4096; ++b) {
        acc += hist[b];
        if (acc >= need) { bin = b; break; }
    }
    st.maha_q999 = (float)pow(10.0, (bin + 1) / 4096.0 * 12.0 - 6.0);
    hipFree(d_mom); hipFree(d_cov); hipFree(d_mean); hipFree(d_hist);
    *out = st;
    return casim_mlp_set_stats(&st);
}

int casim_mlp_prepare(const float *feat, const float *rates, const uint16_t *gates, int64_t n, float *x,
                      float *y, float *m, void *stream) {
    if (!feat || !rates || !gates || !x || !y || !m || n < 0) return CASIM_EINVAL;
    if (!M.have_stats) return CASIM_ENOSURROGATE;
    if (n == 0) return CASIM_OK;
    hipLaunchKernelGGL(prepare_kernel, dim3((unsigned)((n * 12 + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       feat, rates, gates, n, M.stats_dev, x, y, m);
    MLP_TRY(hipGetLastError());
    return CASIM_OK;
}

// Checkpoint blob: 8-byte tag, int64 step, stats, params, Adam m, Adam v.
static const char kTag[8] = {'C', 'A', 'S', 'M', 'L', 'P', '0', '1'};

int casim_mlp_save(void *blob, size_t *bytes) {
    if (!bytes) return CASIM_EINVAL;
    const size_t np = kMlpParams * sizeof(float);
    const size_t need = 8 + sizeof(int64_t) + sizeof(casim_mlp_stats) + 3 * np;
    if (!blob) { *bytes = need; return CASIM_OK; }
    if (*bytes < need) { *bytes = need; return CASIM_ECAPACITY; }
    if (!M.have_params) return CASIM_ENOSURROGATE;
    MLP_TRY(hipDeviceSynchronize());
    char *p = (char *)blob;
    memcpy(p, kTag, 8); p += 8;
    memcpy(p, &M.step, sizeof(int64_t)); p += sizeof(int64_t);
    casim_mlp_stats st{};                     // all zero when no statistics are installed
    if (M.have_stats) st = M.stats;
    memcpy(p, &st, sizeof st); p += sizeof st;
    MLP_TRY(hipMemcpy(p, M.theta, np, hipMemcpyDeviceToHost)); p += np;
    MLP_TRY(hipMemcpy(p, M.mo, np, hipMemcpyDeviceToHost)); p += np;
    MLP_TRY(hipMemcpy(p, M.ve, np, hipMemcpyDeviceToHost));
    *bytes = need;
    return CASIM_OK;
}

int casim_mlp_load(const void *blob, size_t bytes) {
    const size_t np = kMlpParams * sizeof(float);
    const size_t need = 8 + sizeof(int64_t) + sizeof(casim_mlp_stats) + 3 * np;
    if (!blob || bytes < need || memcmp(blob, kTag, 8) != 0) return CASIM_EINVAL;
    const char *p = (const char *)blob + 8;
    int64_t step;
    memcpy(&step, p, sizeof step); p += sizeof step;
    casim_mlp_stats st;
    memcpy(&st, p, sizeof st); p += sizeof st;
    if (st.x_std[0] > 0.0f) {
        const int rc = casim_mlp_set_stats(&st);
        if (rc) return rc;
    }
    MLP_TRY(ensure_alloc());
    MLP_TRY(hipMemcpy(M.theta, p, np, hipMemcpyHostToDevice)); p += np;
    MLP_TRY(hipMemcpy(M.mo, p, np, hipMemcpyHostToDevice)); p += np;
    MLP_TRY(hipMemcpy(M.ve, p, np, hipMemcpyHostToDevice));
    M.step = step;
    M.have_params = true;
    return CASIM_OK;
}

}  // extern "C"
