// Binary64 exponential and logarithm for the sweep kernels.
//
// The general-purpose device library routines are built for correct
// rounding over the whole double range and cost about 40 (exp) and 90 (log)
// vector instructions.  The step only needs about one ulp on finite,
// positive, non-huge arguments, so both follow Tang's table-driven methods
// (Tang 1989 for exp, Tang 1990 for log, ACM TOMS 15(2) and 16(4)) with
// small tables that every kernel using them copies into LDS first
// (load_math_tables):
//   exp: x = (64 m + j) ln2/64 + r, |r| <= ln2/128, with ln2/64 split in a
//        part exact in 39 bits and a remainder; exp(x) = 2^m 2^(j/64)
//        (1 + p(r)), p the Taylor polynomial of exp(r) - 1 to degree 5
//        (truncation error below r^6/720 < 4e-17).  16 instructions.
//   log: x = m 2^e, m in [1/2, 1), j = round(256 m) in [128, 256],
//        c_j = 256/j rounded; ln x = e ln2 - ln c_j + log1p(m c_j - 1) with
//        |m c_j - 1| <= 1/256 and the Taylor polynomial of log1p to
//        degree 7 (next term below 2e-18 relative); -ln c_j is tabulated
//        in two parts whose high part, like that of ln 2, lies on the
//        2^-33 grid, so e ln2_hi - ln c_j,hi is exact and ln 1 is exactly
//        0.  23 instructions.  log(0) is -inf.
// Both are checked against the host library by the test-suite through
// casim_debug_math.
#pragma once

#include <hip/hip_runtime.h>

#include "casim_math_tables.h"

namespace casim {

// a*b + c with c a compile-time constant: one v_fma_f64 taking c from a
// scalar register pair.  Left to itself the compiler materialises such an
// addend in the destination vector registers and uses the two-operand
// v_fmac_f64 form, three vector instructions instead of one.  a and b must
// not come straight from a transcendental instruction (v_rcp_f64 etc.): the
// hazard recognizer does not look inside inline assembly.
__device__ __forceinline__ double fma_sc(double a, double b, double c) {
    double d;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "s"(c));
    return d;
}

// c1*a + c0 with both constants from scalar registers (a multiply and an
// add: one instruction cannot read two scalar pairs).
__device__ __forceinline__ double lin_sc(double a, double c1, double c0) {
    double d;
    asm("v_mul_f64 %0, %1, %2\n\tv_add_f64 %0, %0, %3" : "=&v"(d) : "v"(a), "s"(c1), "s"(c0));
    return d;
}

// The tables in LDS (one copy per block).
static __shared__ double s_exp2_tab[kExpTab];
static __shared__ double s_log_tab[kLogTab][3];
constexpr int kMathLdsBytes = (kExpTab + 3 * kLogTab) * 8;

// Every kernel that calls exp64 or log64 runs this first, with all threads
// of the block (it ends with a block barrier).
__device__ __forceinline__ void load_math_tables() {
    for (int i = threadIdx.x; i < kExpTab; i += blockDim.x) s_exp2_tab[i] = kExp2Tab[i];
    for (int i = threadIdx.x; i < 3 * kLogTab; i += blockDim.x) (&s_log_tab[0][0])[i] = (&kLogTabData[0][0])[i];
    __syncthreads();
}

__device__ __forceinline__ double exp64(double x) {
    const double kd = __builtin_rint(x * (64.0 / 0.69314718055994530942));
    const int k = (int)kd;
    double r = __builtin_fma(-kd, kLn2Hi * (1.0 / 64.0), x);   // exact product
    r = __builtin_fma(-kd, kLn2Lo * (1.0 / 64.0), r);
    // exp(r) - 1 = r (1 + r/2 + r^2/6 + r^3/24 + r^4/120)
    double q = lin_sc(r, 1.0 / 120.0, 1.0 / 24.0);
    q = fma_sc(q, r, 1.0 / 6.0);
    q = __builtin_fma(q, r, 0.5);
    q = __builtin_fma(q, r, 1.0);
    const double t = s_exp2_tab[k & (kExpTab - 1)];
    return __builtin_ldexp(__builtin_fma(t, q * r, t), k >> 6);
}

__device__ __forceinline__ double log64(double x) {
    const int e = __builtin_amdgcn_frexp_exp(x);           // x = m 2^e, m in [0.5, 1)
    const double m = __builtin_amdgcn_frexp_mant(x);
    // nearest table point; the clamp (before the conversion) keeps 0, inf
    // and NaN inside the table
    const int j = (int)__builtin_rint(::fmin(::fmax(m * 256.0, 128.0), 256.0));
    const double *T = s_log_tab[j - 128];
    const double r = __builtin_fma(m, T[0], -1.0);
    // log1p(r) = r + r^2 (-1/2 + r/3 - r^2/4 + r^3/5 - r^4/6 + r^5/7)
    double q = lin_sc(r, 1.0 / 7.0, -1.0 / 6.0);
    q = fma_sc(q, r, 1.0 / 5.0);
    q = fma_sc(q, r, -0.25);
    q = fma_sc(q, r, 1.0 / 3.0);
    q = __builtin_fma(q, r, -0.5);
    const double p = __builtin_fma(r * r, q, r);
    const double ed = (double)e;
    const double hi = __builtin_fma(ed, kLn2Hi, T[1]);     // exact: both on the 2^-33 grid
    const double lo = __builtin_fma(ed, kLn2Lo, T[2]) + p;
    return x == 0.0 ? -__builtin_inf() : hi + lo;
}

// 1/x for positive, finite, normal x: the hardware reciprocal estimate
// refined by two Newton-Raphson steps r <- r + r (1 - x r) (within about one
// ulp; no special-case handling, which the IEEE division sequence spends
// most of its instructions on).
__device__ __forceinline__ double rcp64(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}

}  // namespace casim
