// Binary64 exponential and logarithm for the sweep kernels.
//
// The general-purpose device library routines are built for correct
// rounding over the whole double range and cost about 40 (exp) and 90 (log)
// vector instructions.  The step only needs a few ulp on finite, positive,
// non-huge arguments, so these two are written from the textbook methods:
//   exp: Cody & Waite (1980) argument reduction x = k ln2 + r, |r| <= ln2/2,
//        with ln2 split in a high part exact in 32 bits and a low part, then
//        the Taylor polynomial of exp(r) to degree 13 (truncation error below
//        r^14/14! < 5e-18) and a scaling by 2^k.  About 20 instructions.
//   log: x = m 2^e with m in [1/sqrt2, sqrt2), s = (m-1)/(m+1), and
//        ln m = 2 atanh(s) = 2 (s + s^3/3 + ... + s^21/21) (|s| <= 0.172, so
//        the next term is below 3e-18 relative); ln x = e ln2 + ln m.  About
//        30 instructions.  log(0) is -inf.
// Both are checked against the host library by the test-suite through
// casim_debug_math.
#pragma once

#include <hip/hip_runtime.h>

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

__device__ __forceinline__ double exp64(double x) {
    const double log2e = 1.4426950408889634074;
    const double ln2_hi = 6.93147180369123816490e-01;   // upper bits of ln 2
    const double ln2_lo = 1.90821492927058770002e-10;   // ln 2 - ln2_hi
    const double kd = __builtin_rint(x * log2e);
    double r = __builtin_fma(-kd, ln2_hi, x);
    r = __builtin_fma(-kd, ln2_lo, r);
    // Horner form of sum_{n=0}^{13} r^n / n!
    double p = lin_sc(r, 1.0 / 6227020800.0, 1.0 / 479001600.0);   // 1/13!, 1/12!
    p = fma_sc(p, r, 1.0 / 39916800.0);
    p = fma_sc(p, r, 1.0 / 3628800.0);
    p = fma_sc(p, r, 1.0 / 362880.0);
    p = fma_sc(p, r, 1.0 / 40320.0);
    p = fma_sc(p, r, 1.0 / 5040.0);
    p = fma_sc(p, r, 1.0 / 720.0);
    p = fma_sc(p, r, 1.0 / 120.0);
    p = fma_sc(p, r, 1.0 / 24.0);
    p = fma_sc(p, r, 1.0 / 6.0);
    p = __builtin_fma(p, r, 0.5);
    p = __builtin_fma(p, r, 1.0);
    p = __builtin_fma(p, r, 1.0);
    const int k = (int)kd;
    return __builtin_ldexp(p, k);
}

__device__ __forceinline__ double log64(double x) {
    const double ln2_hi = 6.93147180369123816490e-01;
    const double ln2_lo = 1.90821492927058770002e-10;
    int e = __builtin_amdgcn_frexp_exp(x);             // x = m 2^e, m in [0.5, 1)
    double m = __builtin_amdgcn_frexp_mant(x);
    if (m < 0.70710678118654752440) { m *= 2.0; e -= 1; }
    double rm = __builtin_amdgcn_rcp(m + 1.0);              // 1/(m+1), refined twice
    rm = __builtin_fma(rm, __builtin_fma(-(m + 1.0), rm, 1.0), rm);
    rm = __builtin_fma(rm, __builtin_fma(-(m + 1.0), rm, 1.0), rm);
    const double s = (m - 1.0) * rm;
    const double z = s * s;
    // sum_{j=0}^{10} z^j / (2j+1)
    double q = lin_sc(z, 1.0 / 21.0, 1.0 / 19.0);
    q = fma_sc(q, z, 1.0 / 17.0);
    q = fma_sc(q, z, 1.0 / 15.0);
    q = fma_sc(q, z, 1.0 / 13.0);
    q = fma_sc(q, z, 1.0 / 11.0);
    q = fma_sc(q, z, 1.0 / 9.0);
    q = fma_sc(q, z, 1.0 / 7.0);
    q = fma_sc(q, z, 1.0 / 5.0);
    q = fma_sc(q, z, 1.0 / 3.0);
    q = __builtin_fma(q, z, 1.0);
    const double ed = (double)e;
    const double lm = 2.0 * s * q;
    const double r = __builtin_fma(ed, ln2_hi, __builtin_fma(ed, ln2_lo, lm));
    return x == 0.0 ? -__builtin_inf() : r;
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
