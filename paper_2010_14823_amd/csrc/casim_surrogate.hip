// Inference of the process-rate surrogate on the matrix cores (gfx950).
//
// Each wavefront evaluates the 12-128-128-128-12 SiLU network for 64 points
// with v_mfma_f32_16x16x32_bf16: bfloat16 weights and activations, float32
// accumulation.  Operand layout of that instruction (checked on the device by
// a probe before this kernel was written): lane l supplies A[row l%16][k =
// 8*(l/16) .. +8) and B[k = 8*(l/16) .. +8)[col l%16]; it receives
// C[rows 4*(l/16) .. +4)[col l%16].
//
// The transposed weights (W^T, one row per output unit, 8 bfloat16 of padding
// per row against bank conflicts) stay in LDS for the whole block; a wave's
// activations go through its own 64 x 136 LDS tile between layers, because
// the accumulator layout is the transpose of the operand layout.  Biases
// initialise the accumulators.  Per point the kernel also standardises the
// features, checks them against the training range and computes the squared
// Mahalanobis distance, and after the last layer undoes the target scaling
// (rate = 1e-12 sinh(y)), applies the gates and the sign/positivity rules.
#include <math.h>
#include <string.h>

#include <vector>

#include "casim_internal.h"
#include "casim_mlp_internal.h"

namespace casim {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kK1 = 32;                 // layer-1 K (12 features padded)
constexpr int kRow1 = kK1 + 8;          // LDS row length of W1^T
constexpr int kRowH = 128 + 8;          // LDS row length of W2^T, W3^T, W4^T and of activations
constexpr int kW1 = 0;                                  // offsets in bfloat16 elements
constexpr int kW2 = kW1 + 128 * kRow1;
constexpr int kW3 = kW2 + 128 * kRowH;
constexpr int kW4 = kW3 + 128 * kRowH;
constexpr int kWElems = kW4 + 16 * kRowH;               // 42,112 bfloat16 = 84,224 bytes
constexpr int kBias = 128 * 3 + 16;
constexpr int kWavesPerBlock = 4;
constexpr int kActElems = 64 * kRowH;
constexpr size_t kInferLds = (size_t)kWElems * 2 + (size_t)kWavesPerBlock * kActElems * 2;

__device__ __forceinline__ float fast_silu(float z) {
    // z * sigma(z), sigma via the hardware base-2 exponential and reciprocal
    return z * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-1.44269504088896341f * z));
}

// acc[mt][nt] += A(64 x K from act) * W^T(nt) for one layer, NT output tiles.
template <int NT, int KSTEPS>
__device__ __forceinline__ void layer_mfma(const __bf16 *act, int act_row, const __bf16 *wt, int w_row,
                                           f32x4 (&acc)[4][8], int lane) {
    const int r16 = lane % 16, kq = (lane / 16) * 8;
#pragma unroll
    for (int kk = 0; kk < KSTEPS; ++kk) {
        bf16x8 a[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
            a[mt] = *reinterpret_cast<const bf16x8 *>(act + (mt * 16 + r16) * act_row + kk * 32 + kq);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const bf16x8 b = *reinterpret_cast<const bf16x8 *>(wt + (nt * 16 + r16) * w_row + kk * 32 + kq);
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
                acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt], b, acc[mt][nt], 0, 0, 0);
        }
    }
}

// SiLU of the accumulators, written back as the next layer's bfloat16 input.
__device__ __forceinline__ void store_silu(__bf16 *act, const f32x4 (&acc)[4][8], int lane) {
    const int c16 = lane % 16, r4 = (lane / 16) * 4;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < 8; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                act[(mt * 16 + r4 + i) * kRowH + nt * 16 + c16] = (__bf16)fast_silu(acc[mt][nt][i]);
}

__device__ __forceinline__ void init_acc(f32x4 (&acc)[4][8], const float *bias, int nt_count, int lane) {
#pragma unroll
    for (int nt = 0; nt < 8; ++nt) {
        const float b = nt < nt_count ? bias[nt * 16 + lane % 16] : 0.0f;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) acc[mt][nt] = f32x4{b, b, b, b};
    }
}

// Rows of region r: [r * rcap, r * rcap + count), the count from the slot
// counters of a step, else the part of [0, n_all) the region covers.
__device__ __forceinline__ int64_t region_rows(const unsigned long long *counters, int64_t rcap, int64_t n_all,
                                               int64_t r) {
    if (counters) {
        const unsigned long long c = counters[r * kCounterStride];
        return (int64_t)(c < (unsigned long long)rcap ? c : (unsigned long long)rcap);
    }
    const int64_t cnt = n_all - r * rcap;
    return cnt < 0 ? 0 : (cnt > rcap ? rcap : cnt);
}

__global__ __launch_bounds__(256) void surrogate_infer_kernel(const uint16_t *__restrict__ wglob,
                                                              const float *__restrict__ bias,
                                                              const float *__restrict__ stats_raw,
                                                              float range_margin, float maha_max_arg,
                                                              const float *__restrict__ feat,
                                                              const uint16_t *__restrict__ gates, int64_t n_all,
                                                              const unsigned long long *__restrict__ counters,
                                                              int64_t rcap, int64_t nreg,
                                                              float *__restrict__ rates, uint8_t *__restrict__ fallback) {
    extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
    __bf16 *W = reinterpret_cast<__bf16 *>(lds_raw);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __bf16 *act = W + kWElems + wv * kActElems;
    const casim_mlp_stats *S = reinterpret_cast<const casim_mlp_stats *>(stats_raw);

    // weights -> LDS, 16 bytes per load
    {
        const uint4 *src = reinterpret_cast<const uint4 *>(wglob);
        uint4 *dst = reinterpret_cast<uint4 *>(lds_raw);
        for (int i = threadIdx.x; i < kWElems / 8; i += blockDim.x) dst[i] = src[i];
    }
    __syncthreads();
    const float maha_max = maha_max_arg > 0.0f ? maha_max_arg : S->maha_q999;

    for (int64_t r = blockIdx.x; r < nreg; r += gridDim.x)
    for (int64_t t = (int64_t)wv * 64, cnt = region_rows(counters, rcap, n_all, r); t < cnt;
         t += kWavesPerBlock * 64) {
        const int64_t p = r * rcap + t + lane;
        const bool valid = t + lane < cnt;
        // ---- inputs: standardise, range check, Mahalanobis distance --------
        float z[12];
        bool out_of_range = false;
#pragma unroll
        for (int j = 0; j < 12; ++j) {
            const float x = valid ? feat[p * 12 + j] : S->x_mean[j];
            const float span = S->x_max[j] - S->x_min[j];
            out_of_range |= (x < S->x_min[j] - range_margin * span) | (x > S->x_max[j] + range_margin * span);
            z[j] = (x - S->x_mean[j]) / S->x_std[j];
        }
        float d2 = 0.0f;
#pragma unroll
        for (int a = 0; a < 12; ++a) {
            float t = 0.0f;
#pragma unroll
            for (int b = 0; b < 12; ++b) t = fmaf(S->cov_inv[a * 12 + b], z[b], t);
            d2 = fmaf(z[a], t, d2);
        }
        const bool fb = out_of_range || !(d2 <= maha_max);
#pragma unroll
        for (int j = 0; j < kK1; ++j) act[lane * kRowH + j] = (__bf16)(j < 12 ? z[j] : 0.0f);

        // ---- three hidden layers and the output layer ----------------------
        f32x4 acc[4][8];
        init_acc(acc, bias, 8, lane);
        layer_mfma<8, 1>(act, kRowH, W + kW1, kRow1, acc, lane);
        store_silu(act, acc, lane);
        init_acc(acc, bias + 128, 8, lane);
        layer_mfma<8, 4>(act, kRowH, W + kW2, kRowH, acc, lane);
        store_silu(act, acc, lane);
        init_acc(acc, bias + 256, 8, lane);
        layer_mfma<8, 4>(act, kRowH, W + kW3, kRowH, acc, lane);
        store_silu(act, acc, lane);
        init_acc(acc, bias + 384, 1, lane);
        layer_mfma<1, 4>(act, kRowH, W + kW4, kRowH, acc, lane);
        // output tile: lane holds y[rows 4*(l/16)..+4][col l%16] of each 16-row tile
        float *yst = reinterpret_cast<float *>(act);     // 64 x 16 floats, reusing the tile
        {
            const int c16 = lane % 16, r4 = (lane / 16) * 4;
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int i = 0; i < 4; ++i) yst[(mt * 16 + r4 + i) * 16 + c16] = acc[mt][0][i];
        }
        // ---- per point: undo the scaling, gates, signs ----------------------
        if (valid) {
            const unsigned gw = gates[p];
            const bool supersat_ice = gw & CASIM_GATE_SUPERSAT_ICE;
#pragma unroll
            for (int j = 0; j < 12; ++j) {
                const float y = yst[lane * 16 + j] * S->y_std[j] + S->y_mean[j];
                float r = (float)kRateScale * sinhf(y);
                if (j == 3 || j == 4) {      // DEPI, DEPS: sign of the ice supersaturation
                    r = supersat_ice ? fabsf(r) : -fabsf(r);
                } else {
                    r = fmaxf(r, 0.0f);
                }
                rates[p * 12 + j] = ((gw >> j) & 1u) ? r : 0.0f;
            }
            fallback[p] = fb ? 1 : 0;
        }
    }
}

// ---- host side -------------------------------------------------------------
namespace {
struct SurCtx {
    bool ready = false;
    int device = -1;
    uint16_t *w = nullptr;
    float *bias = nullptr, *stats = nullptr;
    bool attr_set = false;
};
SurCtx SC;

uint16_t to_bf16(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);   // quiet NaN
    const uint32_t lsb = (u >> 16) & 1u;
    return (uint16_t)((u + 0x7fffu + lsb) >> 16);                            // round to nearest even
}
}  // namespace

bool surrogate_ready() { return SC.ready; }

SurrogateDev surrogate_dev(float range_margin, float maha_max) {
    return SurrogateDev{SC.w, SC.bias, SC.stats, range_margin, maha_max};
}

hipError_t launch_surrogate_infer(const SurrogateDev &S, const float *feat, const uint16_t *gates, int64_t n,
                                  const unsigned long long *counters, int64_t rcap, float *rates,
                                  uint8_t *fallback, hipStream_t stream) {
    if (!SC.attr_set) {
        hipError_t e = hipFuncSetAttribute((const void *)surrogate_infer_kernel,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)kInferLds);
        if (e != hipSuccess) return e;
        SC.attr_set = true;
    }
    int64_t nreg = kSlotRegions;
    if (!counters) {       // plain rows: 1024 equal regions of whole 64-row tiles
        rcap = ((n + kSlotRegions - 1) / kSlotRegions + 63) / 64 * 64;
        nreg = (n + rcap - 1) / rcap;
    }
    const int64_t blocks = nreg < 1 ? 1 : nreg;
    hipLaunchKernelGGL(surrogate_infer_kernel, dim3((unsigned)blocks), dim3(kWavesPerBlock * 64), kInferLds, stream,
                       S.w, S.bias, S.stats, S.range_margin, S.maha_max, feat, gates, n, counters, rcap, nreg, rates,
                       fallback);
    return hipGetLastError();
}

}  // namespace casim

using namespace casim;

extern "C" {

int casim_surrogate_load(void) {
    const float *theta_dev = mlp_params_device();
    const casim_mlp_stats *st = mlp_stats_host();
    if (!theta_dev || !st) return CASIM_ENOSURROGATE;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return casim_record_hip_error((int)e, hipGetErrorString(e));
    if (!SC.w || SC.device != dev) {
        if ((e = hipMalloc(&SC.w, (size_t)kWElems * 2)) != hipSuccess ||
            (e = hipMalloc(&SC.bias, kBias * sizeof(float))) != hipSuccess ||
            (e = hipMalloc(&SC.stats, sizeof(casim_mlp_stats))) != hipSuccess)
            return casim_record_hip_error((int)e, hipGetErrorString(e));
        SC.device = dev;
        SC.attr_set = false;
    }
    std::vector<float> th(kMlpParams);
    if ((e = hipDeviceSynchronize()) != hipSuccess ||
        (e = hipMemcpy(th.data(), theta_dev, kMlpParams * sizeof(float), hipMemcpyDeviceToHost)) != hipSuccess)
        return casim_record_hip_error((int)e, hipGetErrorString(e));
    std::vector<uint16_t> w(kWElems, 0);
    std::vector<float> b(kBias, 0.0f);
    for (int n = 0; n < 128; ++n)
        for (int k = 0; k < 12; ++k) w[kW1 + n * kRow1 + k] = to_bf16(th[kOW1 + k * 128 + n]);
    for (int n = 0; n < 128; ++n)
        for (int k = 0; k < 128; ++k) {
            w[kW2 + n * kRowH + k] = to_bf16(th[kOW2 + k * 128 + n]);
            w[kW3 + n * kRowH + k] = to_bf16(th[kOW3 + k * 128 + n]);
        }
    for (int n = 0; n < 12; ++n)
        for (int k = 0; k < 128; ++k) w[kW4 + n * kRowH + k] = to_bf16(th[kOW4 + k * 12 + n]);
    for (int j = 0; j < 128; ++j) {
        b[j] = th[kOB1 + j];
        b[128 + j] = th[kOB2 + j];
        b[256 + j] = th[kOB3 + j];
    }
    for (int j = 0; j < 12; ++j) b[384 + j] = th[kOB4 + j];
    if ((e = hipMemcpy(SC.w, w.data(), w.size() * 2, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(SC.bias, b.data(), b.size() * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(SC.stats, st, sizeof *st, hipMemcpyHostToDevice)) != hipSuccess)
        return casim_record_hip_error((int)e, hipGetErrorString(e));
    SC.ready = true;
    return CASIM_OK;
}

int casim_surrogate_infer(const float *feat, const uint16_t *gates, int64_t n, float *rates, uint8_t *fallback,
                          void *stream) {
    if (!feat || !gates || !rates || !fallback || n < 0) return CASIM_EINVAL;
    if (!SC.ready) return CASIM_ENOSURROGATE;
    if (n == 0) return CASIM_OK;
    casim_thresholds t;
    casim_default_thresholds(&t);
    const casim_thresholds *cur = casim_current_thresholds();
    if (cur) t = *cur;
    hipError_t e = launch_surrogate_infer(surrogate_dev((float)t.sur_range_margin, (float)t.sur_maha_max), feat,
                                          gates, n, nullptr, 0, rates, fallback, (hipStream_t)stream);
    if (e != hipSuccess) return casim_record_hip_error((int)e, hipGetErrorString(e));
    return CASIM_OK;
}

}  // extern "C"
