// Inference of the process-rate surrogate on the matrix cores (gfx950).
//
// Each wavefront evaluates the 12-128-128-128-12 SiLU network for 32 points
// with v_mfma_f32_16x16x32_bf16: bfloat16 weights and activations, float32
// accumulation.  Operand layout of that instruction (checked on the device by
// a probe before this kernel was written): lane l supplies A[row l%16][k =
// 8*(l/16) .. +8) and B[k = 8*(l/16) .. +8)[col l%16]; it receives
// C[rows 4*(l/16) .. +4)[col l%16].
//
// Every layer is computed transposed, H^T = W X^T: the weights are the A
// operand (row = output unit; W^T rows padded against bank conflicts,
// resident in LDS for the whole block) and the activations
// the B operand (k = input unit, column = point).  The accumulator of output
// tiles 2kk and 2kk+1 then holds, per lane, units 32kk + 4q .. +4 and
// 32kk + 16 + 4q .. +4 of one point (q = lane / 16), and the next layer's B
// operand for K-step kk needs 8 of that point's units at k = 8q .. +8: the
// K order of the next layer's weights is permuted once, when they are
// loaded, so that k = 32kk + 8q + 4h + i is unit 32kk + 16h + 4q + i.  The
// SiLU values, packed to bfloat16 pairs, are then already the operand and
// never move between lanes.  Activations never leave the registers, LDS
// holds only the weights, biases and feature statistics, and a block runs
// 12 wavefronts (3 per SIMD: 32 points per wavefront keep the kernel within
// 168 registers; 64 points needed 256 and ran 2 per SIMD, 7 % slower).
// Per point the kernel also standardises the
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
// LDS row length of W2^T, W3^T, W4^T: 16 bfloat16 of padding (288-byte rows)
// measured 1.4 % of CU cycles in LDS bank conflicts against 13 % for 8 or 32
constexpr int kRowH = 128 + 16;
constexpr int kW1 = 0;                                  // offsets in bfloat16 elements
constexpr int kW2 = kW1 + 128 * kRow1;
constexpr int kW3 = kW2 + 128 * kRowH;
constexpr int kW4 = kW3 + 128 * kRowH;
constexpr int kWElems = kW4 + 16 * kRowH;               // 44,288 bfloat16 = 88,576 bytes
constexpr int kBias = 128 * 3 + 16;
constexpr int kNT = 2;                                  // point tiles of 16 per wavefront
constexpr int kPts = 16 * kNT;                          // points per wavefront task
constexpr int kUnits = 4 * kNT;                         // activation units per pair of output tiles
constexpr int kInferWaves = 12;                         // three wavefronts per SIMD
// LDS: weights, biases, then per feature j: mean, 1/std, lower and upper
// bound of the standardised range; per output j: target mean and std; the
// 12 x 12 whitening factor of the feature covariance; the Mahalanobis limit;
// then the running sum of the regions' row tiles (kSlotRegions + 1 int32)
// and the regions' row counts (kSlotRegions int32).
constexpr int kStatF = 12 * 4 + 12 * 2 + 144 + 4;
constexpr size_t kInferLds = (size_t)kWElems * 2 + (size_t)(kBias + kStatF) * sizeof(float) +
                             (size_t)(2 * kSlotRegions + 1) * sizeof(int32_t);

typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// Activations are carried scaled by s = -log2(e), the base-2 exponent of the
// logistic function: the layer input is bfloat16(s x), the biases in LDS are
// s b, so every accumulator comes out as u = s z, and the next layer's input
// is s silu(z) = u / (1 + 2^u) -- one base-2 exponential, one reciprocal and
// one product, with no scaling of z.  The output layer's accumulator s y is
// multiplied by -ln 2 = 1/s.
constexpr float kNegLog2e = -1.44269504088896341f;
constexpr float kNegLn2 = -0.693147180559945309f;

__device__ __forceinline__ float scaled_silu(float u) {
    return u * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(u));
}

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// two floats -> two bfloat16 (round to nearest even) in one register: one
// v_cvt_pk_bf16_f32
__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){lo, hi}, bf16x2));
}

__device__ __forceinline__ bf16x8 as_bf16x8(const u32x4 &v) { return __builtin_bit_cast(bf16x8, v); }

// Units of activation work done after product group ip (ip = 4 kk + nt) of
// a stage that spreads its kUnits units over its first ngroups groups.
__host__ __device__ constexpr int units_done(int ip, int ngroups) {
    const int u = ngroups <= 0 ? kUnits : ((ip + 1) * kUnits + ngroups - 1) / ngroups;
    return u < kUnits ? u : kUnits;
}

// Issue order of product groups IP .. END - 1 of a stage: each group's
// NTILE MFMAs, then the vector instructions of its activation units
// (9 each: two times exp2, add, reciprocal and product, and one pack).
template <int NTILE, int KA, int IP, int END>
__device__ __forceinline__ void issue_pattern() {
    if constexpr (IP < END) {
        constexpr int units = units_done(IP, kNT * KA) - (IP > 0 ? units_done(IP - 1, kNT * KA) : 0);
        __builtin_amdgcn_sched_group_barrier(0x008, NTILE, 0);
        if constexpr (units > 0) __builtin_amdgcn_sched_group_barrier(0x002, units * 9, 0);
        issue_pattern<NTILE, KA, IP + 1, END>();
    }
}

// One pipeline stage.  Products: NTILE output tiles (tiles NTILE jm + t of
// the layer, 0 <= t < NTILE) over the kNT point tiles and KS K-steps,
// acc = bias + W(rows of those tiles) * bin.  Activation (ACT): SiLU of the
// previous pair of output tiles (prev0 / prev1, of this layer or of the
// layer before) -> bout[ja], as kUnits units (point tile nt, register r: two
// SiLU values -> one bfloat16 pair), spread over the product groups of the
// first KA K-steps so that they are written before a product of this stage
// reads them (bin and bout may be the same array).  Program and issue order
// interleave each group's products with its share of the activation work,
// so the vector ALU works while the matrix core does.
template <int KS, int NTILE, bool ACT, int KA>
__device__ __forceinline__ void stage(const __bf16 *W, int w_row, const float *bias, const u32x4 (&bin)[4][kNT],
                                      int jm, f32x4 (&acc0)[kNT], f32x4 (&acc1)[kNT], const f32x4 (&prev0)[kNT],
                                      const f32x4 (&prev1)[kNT], u32x4 (&bout)[4][kNT], int ja, int p, int q) {
    uint32_t pk[kNT][4];
    int unit = 0;
    auto act_until = [&](int upto) {
#pragma unroll
        for (int u = 0; u < kUnits; ++u) {
            if (u < unit || u >= upto) continue;
            const int nt = u >> 2, r = u & 3;
            const f32x4 &c = (r < 2) ? prev0[nt] : prev1[nt];
            const int e = 2 * (r & 1);
            pk[nt][r] = pack_bf16(scaled_silu(c[e]), scaled_silu(c[e + 1]));
            // k = 8q + 4h + i of K-step ja <- unit 16h + 4q + i of the previous pair
            if (r == 3) bout[ja][nt] = u32x4{pk[nt][0], pk[nt][1], pk[nt][2], pk[nt][3]};
        }
        unit = upto > unit ? upto : unit;
    };
    if (NTILE > 0) {
        // bias address formed here from an opaque zero: left to itself the
        // compiler keeps one address register per tile and layer for the
        // whole kernel
        int oz;
        asm volatile("v_mov_b32 %0, 0" : "=v"(oz));
        const float *bq = bias + oz + 4 * q;
        const f32x4 bv0 = *reinterpret_cast<const f32x4 *>(bq + (NTILE * jm) * 16);
#pragma unroll
        for (int nt = 0; nt < kNT; ++nt) acc0[nt] = bv0;
        if (NTILE > 1) {
            const f32x4 bv1 = *reinterpret_cast<const f32x4 *>(bq + (NTILE * jm + 1) * 16);
#pragma unroll
            for (int nt = 0; nt < kNT; ++nt) acc1[nt] = bv1;
        }
#pragma unroll
        for (int kk = 0; kk < KS; ++kk) {
            const bf16x8 w0 = *reinterpret_cast<const bf16x8 *>(W + ((NTILE * jm) * 16 + p) * w_row + kk * 32 + 8 * q);
            bf16x8 w1;
            if (NTILE > 1)
                w1 = *reinterpret_cast<const bf16x8 *>(W + ((NTILE * jm + 1) * 16 + p) * w_row + kk * 32 + 8 * q);
#pragma unroll
            for (int nt = 0; nt < kNT; ++nt) {
                acc0[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w0, as_bf16x8(bin[kk][nt]), acc0[nt], 0, 0, 0);
                if (NTILE > 1)
                    acc1[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1, as_bf16x8(bin[kk][nt]), acc1[nt], 0, 0, 0);
                if (ACT) act_until(units_done(kk * kNT + nt, kNT * KA));
            }
        }
    }
    if (ACT) act_until(kUnits);
    if constexpr (ACT && NTILE > 0) issue_pattern<NTILE, KA, 0, kNT * KS>();
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

__global__ __launch_bounds__(kInferWaves * 64) void surrogate_infer_kernel(const uint16_t *__restrict__ wglob,
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
    int32_t *tile0 = reinterpret_cast<int32_t *>(bias + kBias + kStatF);
    int32_t *rows_of = tile0 + kSlotRegions + 1;
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
        // tile0[r]: the first of region r's tiles of kPts rows in one
        // numbering of all regions' tiles (exclusive running sum over
        // r < kSlotRegions; regions past nreg have none), tile0[kSlotRegions]
        // their total.  The wavefronts of the grid take these tiles in turn,
        // so every wavefront gets the same share whatever the regions' counts.
        if (wv == 0) {
            static_assert(kSlotRegions % 64 == 0, "regions are summed 64 lanes at a time");
            constexpr int per = kSlotRegions / 64;
            int32_t own[per], sum = 0;
#pragma unroll
            for (int j = 0; j < per; ++j) {
                const int64_t r = (int64_t)lane * per + j;
                const int32_t rows = r < nreg ? (int32_t)region_rows(counters, rcap, n_all, r) : 0;
                rows_of[r] = rows;
                own[j] = (rows + kPts - 1) / kPts;
                sum += own[j];
            }
            int32_t incl = sum;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int32_t v = __shfl_up(incl, o);
                if (lane >= o) incl += v;
            }
            int32_t run = incl - sum;
#pragma unroll
            for (int j = 0; j < per; ++j) {
                tile0[lane * per + j] = run;
                run += own[j];
            }
            if (lane == 63) tile0[kSlotRegions] = incl;
        }
    }
    __syncthreads();
    const float maha_max = maha[0];
    // This lane's share of a point: features f = 4i + q (i = 0, 1, 2).  Their
    // statistics and row p of the whitening factor at those columns stay in
    // registers (15 values).
    float mq[3], iq[3], loq[3], hiq[3], wq[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int f = 4 * i + q;
        mq[i] = x_mean[f];
        iq[i] = x_istd[f];
        loq[i] = z_lo[f];
        hiq[i] = z_hi[f];
        wq[i] = p < 12 ? wht[p * 12 + f] : 0.0f;
    }

    const int64_t ntiles = tile0[kSlotRegions];
    int lo = 0;                    // region of the wavefront's tile; tiles only move forward
    for (int64_t g = (int64_t)blockIdx.x * kInferWaves + wv; g < ntiles; g += (int64_t)gridDim.x * kInferWaves) {
        // the region of tile g is the last r with tile0[r] <= g (one with
        // tiles, since tile0[r + 1] > g).  tile0 never decreases, so of the
        // 64 entries after lo those at or below g are a prefix: the wave
        // advances by their count, 64 at a time.
        for (;;) {
            const int idx = lo + 1 + lane;
            const int adv = __popcll(__ballot(idx <= kSlotRegions && tile0[idx] <= g));
            lo += adv;
            if (adv < 64) break;
        }
        const int64_t r = lo;
        const int64_t t = (g - tile0[lo]) * kPts;
        const int64_t cnt = rows_of[lo];
        // ---- inputs: point 16 nt + p of the tile, features 4i + q ----------
        u32x4 b[4][kNT];
        int fb[kNT];
#pragma unroll
        for (int nt = 0; nt < kNT; ++nt) {
            // a tile's rows past the count read the region's last row (their
            // results are not stored)
            const int64_t i0 = t + nt * 16 + p;
            const int64_t row = r * rcap + (i0 < cnt ? i0 : cnt - 1);
            const float *fr = feat + row * 12 + q;
            float z[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) z[i] = (fr[4 * i] - mq[i]) * iq[i];
            // range check: the largest excess over a bound of the point's 12
            // features (a difference of two floats is positive exactly when
            // the first is larger), the maximum over its four lanes
            float excess = fmaxf(fmaxf(loq[0] - z[0], z[0] - hiq[0]),
                                 fmaxf(fmaxf(loq[1] - z[1], z[1] - hiq[1]), fmaxf(loq[2] - z[2], z[2] - hiq[2])));
            excess = fmaxf(excess, __shfl_xor(excess, 16));
            excess = fmaxf(excess, __shfl_xor(excess, 32));
            // W z on the matrix cores in float32: v_mfma_f32_16x16x4_f32 takes
            // A[row l%16][k = l/16] and B[k = l/16][col l%16] from lane l, so
            // with k = 4i + q the lane supplies W[p][4i + q] and this point's
            // z[4i + q], and receives rows 4q .. 4q+3 of W z (rows 12..15 are
            // zero); their squares summed over the four lanes are the squared
            // Mahalanobis distance.
            f32x4 wz = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int i = 0; i < 3; ++i) wz = __builtin_amdgcn_mfma_f32_16x16x4f32(wq[i], z[i], wz, 0, 0, 0);
            float part = wz[0] * wz[0];
            part = fmaf(wz[1], wz[1], part);
            part = fmaf(wz[2], wz[2], part);
            part = fmaf(wz[3], wz[3], part);
            part += __shfl_xor(part, 16);
            part += __shfl_xor(part, 32);
            // materialised here: otherwise the compiler sinks the checks to
            // the flag's store after the network and keeps their inputs in
            // registers across it
            int fbi = (excess > 0.0f || !(part <= maha_max)) ? 1 : 0;
            asm volatile("" : "+v"(fbi));
            fb[nt] = fbi;
            // B operand of layer 1: k = 8q + i holds s times feature 4i + q
            // (W1's K order is permuted to match when it is loaded), zeros
            // at k = 8q + 3 .. 8q + 7
            b[0][nt] = u32x4{pack_bf16(kNegLog2e * z[0], kNegLog2e * z[1]), pack_bf16(kNegLog2e * z[2], 0.0f), 0u, 0u};
            __builtin_amdgcn_sched_barrier(0);
        }

        // ---- network: three hidden layers and the output tile, as stages ---
        // over pairs of output tiles (operands alternate between b and b2,
        // accumulators between a and c).  A stage's products run beside the
        // previous pair's activation; the stage that starts a layer runs
        // beside the last activation of the layer before, which its products
        // need only at their last K-step.
        u32x4 b2[4][kNT];
        f32x4 a0[kNT], a1[kNT], c0[kNT], c1[kNT], y4[kNT];
        const __bf16 *W1 = W + kW1, *W2 = W + kW2, *W3 = W + kW3, *W4 = W + kW4;
        stage<1, 2, false, 1>(W1, kRow1, bias, b, 0, a0, a1, c0, c1, b2, 0, p, q);
        __builtin_amdgcn_sched_barrier(0);
        stage<1, 2, true, 1>(W1, kRow1, bias, b, 1, c0, c1, a0, a1, b2, 0, p, q);
        __builtin_amdgcn_sched_barrier(0);
        stage<1, 2, true, 1>(W1, kRow1, bias, b, 2, a0, a1, c0, c1, b2, 1, p, q);
        __builtin_amdgcn_sched_barrier(0);
        stage<1, 2, true, 1>(W1, kRow1, bias, b, 3, c0, c1, a0, a1, b2, 2, p, q);
        __builtin_amdgcn_sched_barrier(0);
        stage<4, 2, true, 3>(W2, kRowH, bias + 128, b2, 0, a0, a1, c0, c1, b2, 3, p, q);
        __builtin_amdgcn_sched_barrier(0);
        stage<4, 2, true, 4>(W2, kRowH, bias + 128, b2, 1, c0, c1, a0, a1, b, 0, p, q);
        __builtin_amdgcn_sched_barrier(0);
        stage<4, 2, true, 4>(W2, kRowH, bias + 128, b2, 2, a0, a1, c0, c1, b, 1, p, q);
        __builtin_amdgcn_sched_barrier(0);
        stage<4, 2, true, 4>(W2, kRowH, bias + 128, b2, 3, c0, c1, a0, a1, b, 2, p, q);
        __builtin_amdgcn_sched_barrier(0);
        stage<4, 2, true, 3>(W3, kRowH, bias + 256, b, 0, a0, a1, c0, c1, b, 3, p, q);
        __builtin_amdgcn_sched_barrier(0);
        stage<4, 2, true, 4>(W3, kRowH, bias + 256, b, 1, c0, c1, a0, a1, b2, 0, p, q);
        __builtin_amdgcn_sched_barrier(0);
        stage<4, 2, true, 4>(W3, kRowH, bias + 256, b, 2, a0, a1, c0, c1, b2, 1, p, q);
        __builtin_amdgcn_sched_barrier(0);
        stage<4, 2, true, 4>(W3, kRowH, bias + 256, b, 3, c0, c1, a0, a1, b2, 2, p, q);
        __builtin_amdgcn_sched_barrier(0);
        // output layer: 12 units (one tile, outputs 4q..4q+3 per lane)
        stage<4, 1, true, 3>(W4, kRowH, bias + 384, b2, 0, y4, a1, c0, c1, b2, 3, p, q);
        __builtin_amdgcn_sched_barrier(0);

        // ---- per point: undo the scaling, gates, signs ----------------------
        // (a non-finite rate anywhere in the point sends it to the plain rates)
#pragma unroll
        for (int nt = 0; nt < kNT; ++nt) {
            // row and statistics addresses formed again from an opaque zero,
            // not kept in registers through the network
            int oz;
            asm volatile("v_mov_b32 %0, 0" : "=v"(oz));
            const float *ym = y_mean + oz, *ys = y_std + oz;
            const int64_t i0 = t + nt * 16 + p + oz;
            const bool valid = i0 < cnt;
            const int64_t row = r * rcap + i0;
            const unsigned gw = valid ? gates[row] : 0u;
            const bool supersat_ice = gw & CASIM_GATE_SUPERSAT_ICE;
            float out4[4];
            bool bad = false;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int j = 4 * q + e;
                const float yv = (kNegLn2 * y4[nt][e]) * ys[j] + ym[j];
                // sinh from one exponential and its reciprocal.  Near 0 the
                // difference loses relative accuracy, but its absolute error
                // stays about 1e-7, i.e. 1e-19 kg/kg/s after the rate scale:
                // far below the network's own error.
                const float ey = __builtin_amdgcn_exp2f(1.44269504088896341f * yv);
                const float sh = 0.5f * (ey - __builtin_amdgcn_rcpf(ey));
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
    int cus = 0, cus_device = -1;      // compute units of device cus_device (grid of the inference kernel)
};
SurCtx SC;

uint16_t to_bf16(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);   // quiet NaN
    const uint32_t lsb = (u >> 16) & 1u;
    return (uint16_t)((u + 0x7fffu + lsb) >> 16);                            // round to nearest even
}
// Operand position of feature f in layer 1: lane group q holds features
// 4i + q (i = 0, 1, 2) at k = 8q + i.
int layer1_pos(int f) { return 8 * (f & 3) + (f >> 2); }

// Input unit at operand position k of a layer fed by a hidden layer:
// k = 32kk + 8q + 4h + i holds unit 32kk + 16h + 4q + i.
int hidden_unit_at(int k) {
    const int kk = k >> 5, q = (k >> 3) & 3, h = (k >> 2) & 1, i = k & 3;
    return 32 * kk + 16 * h + 4 * q + i;
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
    // row counts per region and the tiles of all regions are numbered in int32
    if (rcap > INT32_MAX || kSlotRegions * ((rcap + kPts - 1) / kPts) > INT32_MAX) return hipErrorInvalidValue;
    // one block per compute unit (the LDS of one block), each block's
    // wavefronts taking every (blocks x kInferWaves)-th tile
    int dev = 0;
    hipError_t de = hipGetDevice(&dev);
    if (de != hipSuccess) return de;
    if (SC.cus <= 0 || SC.cus_device != dev) {
        int cus = 0;
        de = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (de != hipSuccess) return de;
        SC.cus = cus > 0 ? cus : 1;
        SC.cus_device = dev;
    }
    const int64_t blocks = SC.cus;
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
        for (int f = 0; f < 12; ++f) w[kW1 + n * kRow1 + layer1_pos(f)] = to_bf16(th[kOW1 + f * 128 + n]);
    // layers fed by a hidden layer: operand position k holds input unit
    // hidden_unit_at(k), the order in which the previous layer's SiLU values
    // come out of its accumulators
    for (int n = 0; n < 128; ++n)
        for (int k = 0; k < 128; ++k) {
            const int u = hidden_unit_at(k);
            w[kW2 + n * kRowH + k] = to_bf16(th[kOW2 + u * 128 + n]);
            w[kW3 + n * kRowH + k] = to_bf16(th[kOW3 + u * 128 + n]);
        }
    for (int n = 0; n < 12; ++n)
        for (int k = 0; k < 128; ++k) w[kW4 + n * kRowH + k] = to_bf16(th[kOW4 + hidden_unit_at(k) * 12 + n]);
    for (int j = 0; j < 128; ++j) {
        b[j] = kNegLog2e * th[kOB1 + j];           // biases scaled like the activations
        b[128 + j] = kNegLog2e * th[kOB2 + j];
        b[256 + j] = kNegLog2e * th[kOB3 + j];
    }
    for (int j = 0; j < 12; ++j) b[384 + j] = kNegLog2e * th[kOB4 + j];
    if ((e = hipMemcpy(SC.w, w.data(), w.size() * 2, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(SC.bias, b.data(), b.size() * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(SC.stats, st, sizeof *st, hipMemcpyHostToDevice)) != hipSuccess)
        return casim_record_hip_error((int)e, hipGetErrorString(e));
    SC.ready = true;
    return CASIM_OK;
}

int casim_surrogate_infer(const float *feat, const uint16_t *gates, int64_t n, float *rates, uint8_t *fallback,
                          void *stream) {
    if (!feat || !gates || !rates || !fallback || n < 0 || n > ((int64_t)1 << 36)) return CASIM_EINVAL;
    if (((uintptr_t)feat | (uintptr_t)rates) & 15u) return CASIM_EINVAL;   // 16-byte row vectors
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
