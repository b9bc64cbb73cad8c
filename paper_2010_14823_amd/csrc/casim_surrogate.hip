// Inference of the process-rate surrogate on the matrix cores (gfx950).
//
// Each wavefront evaluates the 12-128-128-128-12 SiLU network for 64 points
// with v_mfma_f32_16x16x32_bf16: bfloat16 weights and activations, float32
// accumulation.  Operand layout of that instruction (checked on the device by
// a probe before this kernel was written): lane l supplies A[row l%16][k =
// 8*(l/16) .. +8) and B[k = 8*(l/16) .. +8)[col l%16]; it receives
// C[rows 4*(l/16) .. +4)[col l%16].
//
// Every layer is computed transposed, H^T = W X^T: the weights are the A
// operand (row = output unit; W^T rows with 8 bfloat16 of padding against
// bank conflicts, resident in LDS for the whole block) and the activations
// the B operand (k = input unit, column = point).  The accumulator of output
// tiles 2kk and 2kk+1 then holds, per lane, 4 consecutive units of one point,
// and the next layer's B operand for K-step kk needs 8 consecutive units of
// that point: after SiLU and packing to bfloat16 pairs, one
// v_permlane32_swap and one v_permlane16_swap per 32-bit register move the
// values to the lanes that need them (lane layout of both swaps checked on
// the device by a probe).  Activations therefore never leave the registers,
// LDS holds only the weights, biases and feature statistics, and a block runs
// 8 wavefronts (2 per SIMD).  Per point the kernel also standardises the
// features, checks them against the training range and computes the squared
// Mahalanobis distance |W z|^2 (rows split over the 4 lanes of a point,
// summed with two cross-lane exchanges), and after the last layer undoes the target
// scaling (rate = 1e-12 sinh(y)), applies the gates and the sign/positivity
// rules.
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
constexpr int kInferWaves = 8;                          // two wavefronts per SIMD
// LDS: weights, biases, then per feature j: mean, 1/std, lower and upper
// bound of the standardised range; per output j: target mean and std; the
// 12 x 12 whitening factor of the feature covariance; the Mahalanobis limit.
constexpr int kStatF = 12 * 4 + 12 * 2 + 144 + 4;
constexpr size_t kInferLds = (size_t)kWElems * 2 + (size_t)(kBias + kStatF) * sizeof(float);

typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float fast_silu(float z) {
    // z * sigma(z), sigma via the hardware base-2 exponential and reciprocal
    return z * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-1.44269504088896341f * z));
}

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// two floats -> two bfloat16 (round to nearest even) in one register: one
// v_cvt_pk_bf16_f32
__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){lo, hi}, bf16x2));
}

// SiLU of output tiles 2kk, 2kk+1 (C layout: units 4q..4q+3 of point p in
// lane p + 16q) -> B operand of K-step kk (units 8q..8q+7 of point p).
__device__ __forceinline__ u32x4 silu_to_operand(const f32x4 &c0, const f32x4 &c1) {
    const uint32_t x0 = pack_bf16(fast_silu(c0[0]), fast_silu(c0[1]));
    const uint32_t x1 = pack_bf16(fast_silu(c0[2]), fast_silu(c0[3]));
    const uint32_t y0 = pack_bf16(fast_silu(c1[0]), fast_silu(c1[1]));
    const uint32_t y1 = pack_bf16(fast_silu(c1[2]), fast_silu(c1[3]));
    // rows of 16 lanes: (x, y) -> ([x0 x1 y0 y1], [x2 x3 y2 y3]) -> ([x0 x2 y0 y2], [x1 x3 y1 y3])
    const auto a0 = __builtin_amdgcn_permlane32_swap(x0, y0, false, false);
    const auto b0 = __builtin_amdgcn_permlane16_swap(a0[0], a0[1], false, false);
    const auto a1 = __builtin_amdgcn_permlane32_swap(x1, y1, false, false);
    const auto b1 = __builtin_amdgcn_permlane16_swap(a1[0], a1[1], false, false);
    return u32x4{b0[0], b1[0], b0[1], b1[1]};
}

__device__ __forceinline__ bf16x8 as_bf16x8(const u32x4 &v) { return __builtin_bit_cast(bf16x8, v); }

// One stage of a hidden layer: the products of output tiles 2j, 2j+1
// (acc0/acc1 = bias + W(rows of those tiles) * B, four point tiles, KS
// K-steps) written in program order together with the activation of the
// previous pair (prev0/prev1 -> bout[j - 1]): after every product pair of a
// K-step comes a share of the previous pair's SiLU, so the matrix cores and
// the vector ALUs of one wavefront work at the same time.  Activation units:
// 16 packs (point tile nt, register r: two SiLU values -> two bfloat16), the
// lane swaps of a point tile after its four packs.
template <int KS, bool ACT, bool MUL>
__device__ __forceinline__ void stage(const __bf16 *W, int w_row, const float *bias, const u32x4 (&bin)[4][4], int j,
                                      f32x4 (&acc0)[4], f32x4 (&acc1)[4], const f32x4 (&prev0)[4],
                                      const f32x4 (&prev1)[4], u32x4 (&bout)[4][4], int p, int q) {
    uint32_t pk[4][4];
    int unit = 0;
    auto act_units = [&](int n) {
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            if (u < unit || u >= unit + n) continue;
            const int nt = u >> 2, r = u & 3;
            const f32x4 &c = (r < 2) ? prev0[nt] : prev1[nt];
            const int e = 2 * (r & 1);
            pk[nt][r] = pack_bf16(fast_silu(c[e]), fast_silu(c[e + 1]));
            if (r == 3) {
                // rows of 16 lanes: (x, y) -> ([x0 x1 y0 y1], [x2 x3 y2 y3]) -> ([x0 x2 y0 y2], [x1 x3 y1 y3])
                const auto a0 = __builtin_amdgcn_permlane32_swap(pk[nt][0], pk[nt][2], false, false);
                const auto b0 = __builtin_amdgcn_permlane16_swap(a0[0], a0[1], false, false);
                const auto a1 = __builtin_amdgcn_permlane32_swap(pk[nt][1], pk[nt][3], false, false);
                const auto b1 = __builtin_amdgcn_permlane16_swap(a1[0], a1[1], false, false);
                bout[j - 1][nt] = u32x4{b0[0], b1[0], b0[1], b1[1]};
            }
        }
        unit += n;
    };
    if (MUL) {
        const f32x4 bv0 = *reinterpret_cast<const f32x4 *>(bias + (2 * j) * 16 + 4 * q);
        const f32x4 bv1 = *reinterpret_cast<const f32x4 *>(bias + (2 * j + 1) * 16 + 4 * q);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            acc0[nt] = bv0;
            acc1[nt] = bv1;
        }
    }
    constexpr int per = 16 / (4 * KS) > 0 ? 16 / (4 * KS) : 1;   // activation units per product pair
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
        bf16x8 a0, a1;
        if (MUL) {
            a0 = *reinterpret_cast<const bf16x8 *>(W + ((2 * j) * 16 + p) * w_row + kk * 32 + 8 * q);
            a1 = *reinterpret_cast<const bf16x8 *>(W + ((2 * j + 1) * 16 + p) * w_row + kk * 32 + 8 * q);
        }
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            if (MUL) {
                acc0[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, as_bf16x8(bin[kk][nt]), acc0[nt], 0, 0, 0);
                acc1[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, as_bf16x8(bin[kk][nt]), acc1[nt], 0, 0, 0);
            }
            if (ACT) act_units(MUL ? per : 16);
            if (ACT && !MUL) return;
        }
    }
    if (ACT && unit < 16) act_units(16 - unit);
}

// One hidden layer, bout = SiLU(bias + W * bin) in the next layer's operand
// layout, as four stages over pairs of output tiles; at most two pairs of
// accumulators (64 registers) are live instead of all eight tiles.
template <int KS>
__device__ __forceinline__ void hidden_layer(const __bf16 *W, int w_row, const float *bias, const u32x4 (&bin)[4][4],
                                             u32x4 (&bout)[4][4], int p, int q) {
    f32x4 a0[4], a1[4], c0[4], c1[4];
    stage<KS, false, true>(W, w_row, bias, bin, 0, a0, a1, c0, c1, bout, p, q);
    __builtin_amdgcn_sched_barrier(0);
    stage<KS, true, true>(W, w_row, bias, bin, 1, c0, c1, a0, a1, bout, p, q);
    __builtin_amdgcn_sched_barrier(0);
    stage<KS, true, true>(W, w_row, bias, bin, 2, a0, a1, c0, c1, bout, p, q);
    __builtin_amdgcn_sched_barrier(0);
    stage<KS, true, true>(W, w_row, bias, bin, 3, c0, c1, a0, a1, bout, p, q);
    __builtin_amdgcn_sched_barrier(0);
    stage<KS, true, false>(W, w_row, bias, bin, 4, a0, a1, c0, c1, bout, p, q);
    __builtin_amdgcn_sched_barrier(0);
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

__global__ __launch_bounds__(512) void surrogate_infer_kernel(const uint16_t *__restrict__ wglob,
                                                              const float *__restrict__ bias_g,
                                                              const float *__restrict__ stats_raw,
                                                              float range_margin, float maha_max_arg,
                                                              const float *__restrict__ feat,
                                                              const uint16_t *__restrict__ gates, int64_t n_all,
                                                              const unsigned long long *__restrict__ counters,
                                                              int64_t rcap, int64_t nreg,
                                                              float *__restrict__ rates, uint8_t *__restrict__ fallback) {
    extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
    __bf16 *W = reinterpret_cast<__bf16 *>(lds_raw);
    float *bias = reinterpret_cast<float *>(lds_raw + (size_t)kWElems * 2);
    float *x_mean = bias + kBias, *x_istd = x_mean + 12, *z_lo = x_istd + 12, *z_hi = z_lo + 12;
    float *y_mean = z_hi + 12, *y_std = y_mean + 12, *wht = y_std + 12, *maha = wht + 144;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int p = lane & 15, q = lane >> 4;
    const casim_mlp_stats *S = reinterpret_cast<const casim_mlp_stats *>(stats_raw);

    // weights, biases and statistics -> LDS
    {
        const uint4 *src = reinterpret_cast<const uint4 *>(wglob);
        uint4 *dst = reinterpret_cast<uint4 *>(lds_raw);
        for (int i = threadIdx.x; i < kWElems / 8; i += blockDim.x) dst[i] = src[i];
        for (int i = threadIdx.x; i < kBias; i += blockDim.x) bias[i] = bias_g[i];
        if (threadIdx.x < 12) {
            const int j = threadIdx.x;
            // trust region in standardised units: the range check then tests
            // the same number the network receives
            const float span = S->x_max[j] - S->x_min[j];
            x_mean[j] = S->x_mean[j];
            x_istd[j] = 1.0f / S->x_std[j];
            z_lo[j] = (S->x_min[j] - range_margin * span - S->x_mean[j]) / S->x_std[j];
            z_hi[j] = (S->x_max[j] + range_margin * span - S->x_mean[j]) / S->x_std[j];
            y_mean[j] = S->y_mean[j];
            y_std[j] = S->y_std[j];
        }
        for (int i = threadIdx.x; i < 144; i += blockDim.x) wht[i] = S->whiten[i];
        if (threadIdx.x == 0) maha[0] = maha_max_arg > 0.0f ? maha_max_arg : S->maha_q999;
    }
    __syncthreads();
    const float maha_max = maha[0];

    for (int64_t r = blockIdx.x; r < nreg; r += gridDim.x)
    for (int64_t t = (int64_t)wv * 64, cnt = region_rows(counters, rcap, n_all, r); t < cnt;
         t += kInferWaves * 64) {
        // The statistics are read from LDS at their use in every tile: an
        // opaque zero in the index keeps the compiler from hoisting all of
        // them (some 70 values per lane) into registers for the whole loop.
        int oz;
        asm volatile("v_mov_b32 %0, 0" : "=v"(oz));
        const float *xm = x_mean + oz, *xi = x_istd + oz, *zl = z_lo + oz, *zh = z_hi + oz, *wi = wht + oz;
        // ---- inputs: point 16 nt + p of the tile, features split over q ----
        u32x4 b[4][4];
        bool fb[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const int64_t i0 = t + nt * 16 + p;
            const bool valid = i0 < cnt;
            const int64_t row = r * rcap + i0;
            float z[12];
#pragma unroll
            for (int j = 0; j < 12; ++j) {
                const float x = valid ? feat[row * 12 + j] : xm[j];
                z[j] = (x - xm[j]) * xi[j];
            }
            // range check of features 3q..3q+2 and rows 3q..3q+2 of W z, whose
            // squares sum to the squared Mahalanobis distance (this lane's three
            // features picked by q, not by a register index; W is lower
            // triangular and its zeros above the diagonal are read as zeros)
            bool out = false;
            float part = 0.0f;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int ja = 3 * q + a;
                const float za = q == 0 ? z[a] : q == 1 ? z[3 + a] : q == 2 ? z[6 + a] : z[9 + a];
                out |= (za < zl[ja]) | (za > zh[ja]);
                float s_ = 0.0f;
#pragma unroll
                for (int c = 0; c < 12; ++c) s_ = fmaf(wi[ja * 12 + c], z[c], s_);
                part = fmaf(s_, s_, part);
            }
            part += __shfl_xor(part, 16);
            part += __shfl_xor(part, 32);
            const int o = (int)out;
            const int o2 = o | __shfl_xor(o, 16);
            const int o4 = o2 | __shfl_xor(o2, 32);
            fb[nt] = o4 != 0 || !(part <= maha_max);
            // B operand of layer 1: features 8q..8q+7 (12 features padded to 32)
            float v[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = q == 0 ? z[e] : (q == 1 && e < 4) ? z[8 + e] : 0.0f;
            b[0][nt] = u32x4{pack_bf16(v[0], v[1]), pack_bf16(v[2], v[3]), pack_bf16(v[4], v[5]), pack_bf16(v[6], v[7])};
            __builtin_amdgcn_sched_barrier(0);
        }

        // ---- three hidden layers (operands alternate between b and b2) -----
        u32x4 b2[4][4];
        hidden_layer<1>(W + kW1, kRow1, bias, b, b2, p, q);
        hidden_layer<4>(W + kW2, kRowH, bias + 128, b2, b, p, q);
        hidden_layer<4>(W + kW3, kRowH, bias + 256, b, b2, p, q);

        // ---- output layer: 12 units (one tile), outputs 4q..4q+3 per lane ----
        f32x4 y4[4];
        {
            const f32x4 bv = *reinterpret_cast<const f32x4 *>(bias + 384 + 4 * q);
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) y4[nt] = bv;
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const bf16x8 a = *reinterpret_cast<const bf16x8 *>(W + kW4 + p * kRowH + kk * 32 + 8 * q);
#pragma unroll
                for (int nt = 0; nt < 4; ++nt)
                    y4[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, as_bf16x8(b2[kk][nt]), y4[nt], 0, 0, 0);
            }
        }

        // ---- per point: undo the scaling, gates, signs ----------------------
        // (the four lanes of a point share p, so they take the same branches;
        // a non-finite rate anywhere in the point sends it to the plain rates)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const int64_t i0 = t + nt * 16 + p;
            const bool valid = i0 < cnt;
            const int64_t row = r * rcap + i0;
            const unsigned gw = valid ? gates[row] : 0u;
            const bool supersat_ice = gw & CASIM_GATE_SUPERSAT_ICE;
            float out4[4];
            bool bad = false;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int j = 4 * q + e;
                const float yv = y4[nt][e] * y_std[j] + y_mean[j];
                // sinh: series near 0, exponentials elsewhere
                const float ey = __builtin_amdgcn_exp2f(1.44269504088896341f * yv);
                const float y2 = yv * yv;
                const float sh = fabsf(yv) < 0.5f ? yv * (1.0f + y2 * (1.0f / 6.0f) * (1.0f + y2 * (1.0f / 20.0f)))
                                                  : 0.5f * (ey - __builtin_amdgcn_rcpf(ey));
                float rv = (float)kRateScale * sh;
                if (j == 3 || j == 4) {      // DEPI, DEPS: sign of the ice supersaturation
                    rv = supersat_ice ? fabsf(rv) : -fabsf(rv);
                } else {
                    rv = fmaxf(rv, 0.0f);
                }
                out4[e] = ((gw >> j) & 1u) ? rv : 0.0f;
                bad |= q < 3 && !__builtin_isfinite(out4[e]);
            }
            int bi = (int)bad;
            bi |= __shfl_xor(bi, 16);
            bi |= __shfl_xor(bi, 32);
            if (valid) {
                if (q == 0) fallback[row] = (fb[nt] || bi) ? 1 : 0;
                if (q < 3)
                    *reinterpret_cast<float4 *>(rates + row * 12 + 4 * q) =
                        make_float4(out4[0], out4[1], out4[2], out4[3]);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// Per point (k, c): the rates and trust-region flag of its slot, or zeros
// and flag 2 when it has no slot.  rates_out is [12][nlev][ld], flags
// [nlev][ld].
__global__ __launch_bounds__(256) void slot_scatter_kernel(const int32_t *__restrict__ idx_map, int64_t ncol,
                                                           int64_t nlev, int64_t ld,
                                                           const float *__restrict__ slot_rates,
                                                           const uint8_t *__restrict__ slot_fb,
                                                           float *__restrict__ rates_out,
                                                           uint8_t *__restrict__ flags) {
    const int64_t pid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (pid >= ncol * nlev) return;
    const int64_t k = pid / ncol, c = pid - k * ncol;
    const int64_t ix = k * ld + c, plane = nlev * ld;
    const int32_t slot = idx_map[pid];
#pragma unroll
    for (int j = 0; j < 12; ++j) rates_out[j * plane + ix] = slot >= 0 ? slot_rates[(int64_t)slot * 12 + j] : 0.0f;
    flags[ix] = slot >= 0 ? slot_fb[slot] : (uint8_t)2;
}

hipError_t launch_slot_scatter(const int32_t *idx_map, int64_t ncol, int64_t nlev, int64_t ld,
                               const float *slot_rates, const uint8_t *slot_fb, float *rates_out, uint8_t *flags,
                               hipStream_t stream) {
    const int64_t n = ncol * nlev, blocks = (n + 255) / 256;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(slot_scatter_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, idx_map, ncol, nlev, ld,
                       slot_rates, slot_fb, rates_out, flags);
    return hipGetLastError();
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
    hipLaunchKernelGGL(surrogate_infer_kernel, dim3((unsigned)blocks), dim3(kInferWaves * 64), kInferLds, stream,
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
