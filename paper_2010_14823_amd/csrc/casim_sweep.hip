// Column-sweep kernels of the bulk-microphysics step for gfx950.
//
// Columns are independent (Sec. II of the CASIM port study); the paper maps
// one column to one GPU thread (Sec. III-B).  Here a 64-wide wavefront holds
// a tile of C columns x L = 64/C consecutive levels (lane = g*C + c: column c
// of the wave's column block, level group g, g = 0 the top of the tile), and
// walks its columns from the top level down in chunks of L levels.  C = 64
// would be the paper's one-column-per-lane mapping; C = 16 (one 128-byte row
// of every field per level) is used on large domains and 8 or 4 on small
// ones, for enough wavefronts.  Which tile a wavefront takes is a pure
// schedule: blocks are renumbered so that each XCD streams groups of
// neighbouring tiles, and tiles that were busy in the previous step are kept
// out of the last dispatch round (tile_order_kernel).  Per chunk a wavefront
//   1. reads the 8 fields that decide whether anything can happen at a point
//      (T, p, q_v and the five condensate masses);
//   2. votes: when no point of the chunk has condensate or supersaturation
//      and no sedimentation flux enters it from above, the chunk's 12
//      tendencies are exact zeros and the wavefront moves on (clear sky costs
//      8 loads and 12 stores per point);
//   3. reads the other 6 fields where something can happen, and runs clean-up,
//      instant phase changes, saturation adjustment, the 12 process rates and
//      the source limiter for all 64 points at once;
//   4. sediments rain, ice, snow and graupel.  Explicit flux-form upwind with
//      a static substep count couples level k at substep s only to the flux
//      leaving level k+1 at substep s, so all substeps of a chunk are done in
//      order with every level of the chunk in parallel: the flux from the
//      level above comes from the lane C places lower (a cross-lane shuffle),
//      and for the top level of the chunk from the previous chunk's bottom
//      level, kept in LDS per (category, moment, substep, column);
//   5. writes the tendencies (accumulated increment / dt).
//
// Slopes of the size distributions are handled in log space: lambda^b,
// lambda^-7 etc. become exp(k ln lambda) and the mean-diameter clamp is a
// clamp of ln lambda.
//
// Precision policy: MIX = false runs everything in binary64.  MIX = true
// evaluates the 12 process rates and the fall speeds in binary32 and keeps
// binary64 for saturation pressures, the saturation adjustment, the limiter
// and apply, the sedimentation fluxes, level updates and surface sums.
#include "casim_internal.h"
#include "casim_math.h"
#include "casim_mlp_internal.h"

namespace casim {

__device__ constexpr DevParams kFastParams = kDefaultParams;

template <bool FAST>
__device__ __forceinline__ const DevParams &params(const DevParams &rt) {
    if constexpr (FAST) return kFastParams;
    else return rt;
}

template <class R> struct Mth;
template <> struct Mth<double> {
    static __device__ __forceinline__ double exp(double x) { return exp64(x); }
    static __device__ __forceinline__ double log(double x) { return log64(x); }
    static __device__ __forceinline__ double fmin(double a, double b) { return ::fmin(a, b); }
};
template <> struct Mth<float> {
    // hardware base-2 exponential and logarithm (v_exp_f32 / v_log_f32)
    static __device__ __forceinline__ float exp(float x) { return __builtin_amdgcn_exp2f(x * 1.44269504088896341f); }
    static __device__ __forceinline__ float log(float x) { return __builtin_amdgcn_logf(x) * 0.69314718055994531f; }
    static __device__ __forceinline__ float fmin(float a, float b) { return ::fminf(a, b); }
};

template <class R>
__device__ __forceinline__ R clampv(R x, R lo, R hi) { return x < lo ? lo : (x > hi ? hi : x); }

// The step reads each input and writes each tendency exactly once: streaming
// (non-temporal) accesses keep them from displacing other lines in the caches.
typedef float f32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ double ldnt(const double *p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ void stnt(double *p, double v) { __builtin_nontemporal_store(v, p); }

// 1/b and a/b in the rate precision: the refined reciprocal in binary64, the
// hardware reciprocal (1 ulp) in binary32, whose rates only need binary32
// accuracy
__device__ __forceinline__ double rrcp(double b) { return rcp64(b); }
__device__ __forceinline__ float rrcp(float b) { return 1.0f / b; }
template <class R>
__device__ __forceinline__ R rdiv(R a, R b) { return a * rrcp(b); }

// Working state of one point: values (w) and accumulated increments (d).
struct Pt {
    double T, qv, qc, nc, qr, nr, qi, ni, qs, ns, qg, ng;
};

// Saturation vapour pressure a exp(b Tc / (Tc + c)), Tc = T - T0 (Bolton
// 1980 over liquid, Buck 1981 over ice).  Always evaluated through the same
// expression so a value computed once can be reused for the same T.
__device__ __forceinline__ double esat_liq(const DevParams &P, double T) {
    const double Tc = T - P.T_0;
    return P.esl_a * exp64(P.esl_b * Tc * rcp64(Tc + P.esl_c));
}
__device__ __forceinline__ double esat_ice(const DevParams &P, double T) {
    const double Tc = T - P.T_0;
    return P.esi_a * exp64(P.esi_b * Tc * rcp64(Tc + P.esi_c));
}
__device__ __forceinline__ double q_of_e(const DevParams &P, double e, double p) {
    return P.eps * e * rcp64(p - P.one_m_eps * e);
}
// q_v / q_sat(e) - 1 with one reciprocal (q_sat = eps e / (p - (1 - eps) e)).
__device__ __forceinline__ double sat_m1(const DevParams &P, double qv, double e, double p) {
    return qv * (p - P.one_m_eps * e) * rcp64(P.eps * e) - 1.0;
}
// q_v > q_sat(e) without a division (p - (1 - eps) e > 0 for any e below p).
__device__ __forceinline__ bool supersat(const DevParams &P, double qv, double e, double p) {
    return qv * (p - P.one_m_eps * e) > P.eps * e;
}

// ---- clean-up and instant phase changes ----------------------------------
__device__ __forceinline__ void cleanup(const DevParams &P, Pt &w, Pt &d, double &q, double &dq,
                                        double &n, double &dn, double L) {
    double m = q;
    if (m > 0.0 && m < P.q_min) {
        dq -= m; q = 0.0;
        w.qv += m; d.qv += m;
        dn -= n; n = 0.0;
        double h = -L * m * P.inv_cp;
        w.T += h; d.T += h;
    }
}

__device__ __forceinline__ void adjust(const DevParams &P, bool warm, Pt &w, Pt &d, double p, double rho) {
    cleanup(P, w, d, w.qc, d.qc, w.nc, d.nc, P.L_v);
    cleanup(P, w, d, w.qr, d.qr, w.nr, d.nr, P.L_v);
    if (warm) return;
    cleanup(P, w, d, w.qi, d.qi, w.ni, d.ni, P.L_s);
    cleanup(P, w, d, w.qs, d.qs, w.ns, d.ns, P.L_s);
    cleanup(P, w, d, w.qg, d.qg, w.ng, d.ng, P.L_s);
    if (w.T < P.T_hom && w.qc > 0.0) {           // homogeneous freezing of all cloud
        double m = w.qc, nn = w.nc;
        d.qc -= m; w.qc = 0.0; d.nc -= nn; w.nc = 0.0;
        w.qi += m; d.qi += m; w.ni += nn; d.ni += nn;
        double h = P.L_f * m * P.inv_cp;
        w.T += h; d.T += h;
    }
    if (w.T > P.T_0 && w.qi > 0.0) {             // melting of all ice
        double m = w.qi, nn = w.ni;
        d.qi -= m; w.qi = 0.0; d.ni -= nn; w.ni = 0.0;
        w.qc += m; d.qc += m; w.nc += nn; d.nc += nn;
        double h = -P.L_f * m * P.inv_cp;
        w.T += h; d.T += h;
    }
    if (w.T < P.T_nuc) {                          // Cooper (1986) nucleation
        double qsi = q_of_e(P, esat_ice(P, w.T), p);
        if (w.qv > qsi) {
            double nin = ::fmin(P.cooper_a * exp64(P.cooper_b * (P.T_0 - w.T)), P.cooper_max) * rcp64(rho);
            if (nin > w.ni) {
                double dn = nin - w.ni;
                double dq = ::fmin(dn * P.m_i0, w.qv - qsi);
                w.ni += dn; d.ni += dn;
                w.qv -= dq; d.qv -= dq;
                w.qi += dq; d.qi += dq;
                double h = P.L_s * dq * P.inv_cp;
                w.T += h; d.T += h;
            }
        }
    }
}

// ---- saturation adjustment (binary64 in every mode) -----------------------
// Fixed-count Newton on cp*delta - Lv*(qv - qs(T+delta)) = 0 from delta = 0.
// es_in is the liquid saturation pressure at T_in (already known from the
// activity test); on return es_out holds it at the final temperature.
__device__ __forceinline__ bool satadj(const DevParams &P, int iters, Pt &w, Pt &d, double p,
                                       double T_in, double es_in, double &es_out) {
    double es0 = (w.T == T_in) ? es_in : esat_liq(P, w.T);
    es_out = es0;
    if (!(supersat(P, w.qv, es0, p) || w.qc > 0.0)) return false;
    // f/f' with D = p - (1 - eps) e_s multiplied through by D^2, so that one
    // reciprocal serves both q_sat and the quotient:
    //   f = cp delta - Lv (qv - eps e_s / D),  f' = cp + Lv eps e_s p bc / (D^2 (Tc + c)^2)
    double delta = 0.0, es = es0;
    for (int it = 0; it < iters; ++it) {
        const double Tc = (w.T + delta) - P.T_0;
        const double rtc = rcp64(Tc + P.esl_c);
        if (it > 0) es = P.esl_a * exp64(P.esl_b * Tc * rtc);
        const double D = p - P.one_m_eps * es;
        const double Les = P.L_v * P.eps * es;
        const double num = D * ((P.cp * delta - P.L_v * w.qv) * D + Les);
        const double den = P.cp * (D * D) + Les * p * P.esl_bc * (rtc * rtc);
        delta -= num * rcp64(den);
    }
    const double T1 = w.T + delta;
    const double es1 = esat_liq(P, T1);
    const double qs1 = q_of_e(P, es1, p);
    const bool bad = !(::fabs(P.cp * delta - P.L_v * (w.qv - qs1)) <= P.newton_rtol * (P.L_v * qs1));
    const double dq = P.cp * delta * (1.0 / P.L_v);
    if (w.qc + dq >= 0.0) {
        const bool newcloud = (w.qc == 0.0 && dq > 0.0);
        w.qc += dq; d.qc += dq;
        w.qv -= dq; d.qv -= dq;
        w.T += delta; d.T += delta;
        es_out = es1;
        if (newcloud) {
            const double add = ::fmax(w.nc, P.n_act) - w.nc;
            w.nc += add; d.nc += add;
        }
    } else {                                      // all cloud evaporates
        const double m = w.qc;
        w.qv += m; d.qv += m;
        const double h = -P.L_v * m * P.inv_cp;
        w.T += h; d.T += h;
        d.qc -= m; w.qc = 0.0;
        d.nc -= w.nc; w.nc = 0.0;
        es_out = esat_liq(P, w.T);
    }
    return bad;
}

// ---- the 12 process rates ------------------------------------------------
enum { AUTO, ACCR, REVP, DEPI, DEPS, IAUT, SACI, SACW, GACW, FRZR, SMLT, GMLT };

// esl is the liquid saturation pressure at w.T.  Powers of a slope are built
// from lambda^-1 by multiplication; only the non-integer powers need exp.
template <class R>
__device__ __forceinline__ void rates(const DevParams &P, bool warm, const Pt &w, double p, double rho,
                                      double ln_rho, double rfac, double esl, R r[12]) {
    using M = Mth<R>;
#pragma unroll
    for (int j = 0; j < 12; ++j) r[j] = R(0);
    const double qmin = P.q_min;
    const bool cP = w.qc >= qmin, rP = w.qr >= qmin;
    const bool iP = !warm && w.qi >= qmin, sP = !warm && w.qs >= qmin, gP = !warm && w.qg >= qmin;
    if (!(cP || rP || iP || sP || gP)) return;
    const bool cold = !warm && w.T < P.T_0, hot = !warm && w.T > P.T_0;
    const bool revp = rP && w.qc == 0.0;
    const bool dep = cold && (iP || sP);
    // saturation ratios in binary64
    const double Sl_m1 = sat_m1(P, w.qv, esl, p);
    double esi = 0.0, Si_m1 = 0.0;
    if (dep) {
        esi = esat_ice(P, w.T);
        Si_m1 = sat_m1(P, w.qv, esi, p);
    }

    const R T = R(w.T), irh = rrcp(R(rho)), lrh = R(ln_rho), rf = R(rfac);
    const R dT0 = T - R(P.T_0);
    // ln lambda, clamped to the mean-diameter bounds, and lambda^-1
    R lnqc = R(0), lnqr = R(0), llr = R(0), llg = R(0), lls = R(0);
    R ilr = R(0), ili = R(0), ils = R(0), ilg = R(0);
    if (cP) lnqc = M::log(R(w.qc));
    if (rP) {
        lnqr = M::log(R(w.qr));
        llr = clampv((R(P.ln_lam_coef[0]) + M::log(R(w.nr)) - lnqr) * R(1.0 / 3.0),
                     R(P.ln_lam_lo[0]), R(P.ln_lam_hi[0]));
        ilr = M::exp(-llr);
    }
    if (iP && cold) {
        const R lli = clampv((R(P.ln_lam_coef[1]) + M::log(rdiv(R(w.ni), R(w.qi)))) * R(1.0 / 3.0),
                             R(P.ln_lam_lo[1]), R(P.ln_lam_hi[1]));
        ili = M::exp(-lli);
    }
    if (sP && (cold || hot)) {
        lls = clampv((R(P.ln_lam_coef[2]) - lrh - M::log(R(w.qs))) * R(0.25), R(P.ln_lam_lo[2]), R(P.ln_lam_hi[2]));
        ils = M::exp(-lls);
    }
    if (gP && (cold || hot)) {
        llg = clampv((R(P.ln_lam_coef[3]) - lrh - M::log(R(w.qg))) * R(0.25), R(P.ln_lam_lo[3]), R(P.ln_lam_hi[3]));
        ilg = M::exp(-llg);
    }

    if (cP && w.nc > 0.0) {
        const R lnNc = M::log(R(w.nc)) + lrh + R(P.ln_1e6);
        r[AUTO] = R(P.auto_a) * M::exp(R(P.auto_qc_exp) * lnqc + R(P.auto_nc_exp) * lnNc);
    }
    if (cP && rP) r[ACCR] = R(P.accr_a) * M::exp(R(P.accr_exp) * (lnqc + lnqr));
    const bool do_revp = revp && Sl_m1 < 0.0;
    if (do_revp || dep) {
        const R KRT2 = R(P.K_a) * R(P.R_v) * T * T;
        const R Dv = R(P.Dv0) * M::exp(R(P.Dv_exp) * M::log(T * R(1.0 / P.T_0))) * rdiv(R(1e5), R(p));
        // G = 1 / (L^2/(K R_v T^2) + R_v T/(D_v e)) = K R_v T^2 D_v e / (L^2 D_v e + R_v T K R_v T^2)
        const R RvT_KRT2 = R(P.R_v) * T * KRT2;
        if (do_revp) {
            const R De = Dv * R(esl);
            const R Gl = rdiv(KRT2 * De, R(P.L_v) * R(P.L_v) * De + RvT_KRT2);
            r[REVP] = R(P.two_pi) * Gl * R(-Sl_m1) * R(w.nr) * ilr;
        }
        if (dep) {
            const R De = Dv * R(esi);
            const R Gi = rdiv(KRT2 * De, R(P.L_s) * R(P.L_s) * De + RvT_KRT2);
            if (iP) r[DEPI] = R(P.two_pi) * Gi * R(Si_m1) * R(w.ni) * ili;
            if (sP) r[DEPS] = R(P.two_pi) * Gi * R(Si_m1) * R(P.N0_s) * irh * (ils * ils);
        }
    }
    if (cold) {
        const R eice = M::exp(R(P.ice_t_exp) * dT0);
        if (iP && w.qi > P.q_i0) r[IAUT] = R(P.iaut_a) * eice * (R(w.qi) - R(P.q_i0));
        if (sP && (iP || cP)) {
            // lambda_s^-(3+b) = lambda_s^-3 * exp(-b ln lambda_s)
            const R coll = R(P.coll_s) * (ils * ils * ils) * M::exp(R(P.coll_exp_s + 3.0) * lls) * rf;
            if (iP) r[SACI] = eice * R(w.qi) * coll;
            if (cP) r[SACW] = R(w.qc) * coll;
        }
        if (gP && cP) r[GACW] = R(P.coll_g) * (ilg * ilg * ilg) * M::exp(R(P.coll_exp_g + 3.0) * llg) * rf * R(w.qc);
        if (rP) {
            const R il2 = ilr * ilr, il6 = il2 * il2 * il2;
            r[FRZR] = R(P.frzr_coef) * R(w.nr) * (M::exp(R(P.bigg_a) * (R(P.T_0) - T)) - R(1)) * il6;
        }
    }
    if (hot && (sP || gP)) {
        const R melt = R(P.two_pi) * R(P.K_a) * dT0 * irh * R(1.0 / P.L_f);
        if (sP) r[SMLT] = melt * R(P.N0_s) * (ils * ils);
        if (gP) r[GMLT] = melt * R(P.N0_g) * (ilg * ilg);
    }
}

// ---- limiter and apply (binary64) ------------------------------------------
template <class R>
__device__ __forceinline__ void apply_rates(const DevParams &P, Pt &w, Pt &d, const R rr[12], double dt) {
    double r[12];
#pragma unroll
    for (int j = 0; j < 12; ++j) r[j] = double(rr[j]);
    double depi_v = r[DEPI] > 0.0 ? r[DEPI] : 0.0, depi_i = r[DEPI] < 0.0 ? -r[DEPI] : 0.0;
    double deps_v = r[DEPS] > 0.0 ? r[DEPS] : 0.0, deps_s = r[DEPS] < 0.0 ? -r[DEPS] : 0.0;
    const double Rv = depi_v + deps_v;
    const double Rc = r[AUTO] + r[ACCR] + r[SACW] + r[GACW];
    const double Rr = r[REVP] + r[FRZR];
    const double Ri = r[IAUT] + r[SACI] + depi_i;
    const double Rs = r[SMLT] + deps_s;
    const double Rg = r[GMLT];
    const bool lv = Rv * dt > w.qv, lc = Rc * dt > w.qc, lr = Rr * dt > w.qr;
    const bool li = Ri * dt > w.qi, ls = Rs * dt > w.qs, lg = Rg * dt > w.qg;
    const double fv = lv ? w.qv * rcp64(Rv * dt) : 1.0, fc = lc ? w.qc * rcp64(Rc * dt) : 1.0;
    const double fr = lr ? w.qr * rcp64(Rr * dt) : 1.0, fi = li ? w.qi * rcp64(Ri * dt) : 1.0;
    const double fs = ls ? w.qs * rcp64(Rs * dt) : 1.0, fg = lg ? w.qg * rcp64(Rg * dt) : 1.0;
    const double auto_ = r[AUTO] * fc, accr = r[ACCR] * fc, sacw = r[SACW] * fc, gacw = r[GACW] * fc;
    const double revp = r[REVP] * fr, frzr = r[FRZR] * fr;
    const double iaut = r[IAUT] * fi, saci = r[SACI] * fi;
    const double smlt = r[SMLT] * fs, gmlt = r[GMLT] * fg;
    depi_v *= fv; deps_v *= fv; depi_i *= fi; deps_s *= fs;

    const double mm_c = w.qc > 0.0 ? w.nc * rcp64(w.qc) : 0.0;
    const double mm_r = w.qr > 0.0 ? w.nr * rcp64(w.qr) : 0.0;
    const double mm_i = w.qi > 0.0 ? w.ni * rcp64(w.qi) : 0.0;
    const double mm_s = w.qs > 0.0 ? w.ns * rcp64(w.qs) : 0.0;
    const double mm_g = w.qg > 0.0 ? w.ng * rcp64(w.qg) : 0.0;

    const double sq_v = dt * (depi_v + deps_v), g_v = dt * (revp + depi_i + deps_s);
    const double sq_c = dt * (auto_ + accr + sacw + gacw);
    const double sq_r = dt * (revp + frzr), g_r = dt * (auto_ + accr + smlt + gmlt);
    const double sq_i = dt * (iaut + saci + depi_i), g_i = dt * depi_v;
    const double sq_s = dt * (smlt + deps_s), g_s = dt * (deps_v + iaut + saci + sacw);
    const double sq_g = dt * gmlt, g_g = dt * (gacw + frzr);
    const double ng_r = dt * (auto_ * P.inv_m_r0 + smlt * mm_s + gmlt * mm_g);
    const double ng_s = dt * iaut * P.inv_m_s0;
    const double ng_g = dt * frzr * mm_r;
    const double dTh = dt * ((depi_v + deps_v - depi_i - deps_s) * P.L_s - revp * P.L_v
                             + (sacw + gacw + frzr) * P.L_f - (smlt + gmlt) * P.L_f) * P.inv_cp;

#define CASIM_APPLY(q, n, lim, sq, gq, ns_, gn)                      \
    if (lim) { d.q -= w.q; w.q = 0.0; d.n -= w.n; w.n = 0.0; }        \
    else { w.q -= sq; d.q -= sq; w.n -= ns_; d.n -= ns_; }            \
    w.q += gq; d.q += gq; w.n += gn; d.n += gn;
    if (lv) { d.qv -= w.qv; w.qv = 0.0; } else { w.qv -= sq_v; d.qv -= sq_v; }   // vapour: no number
    w.qv += g_v; d.qv += g_v;
    CASIM_APPLY(qc, nc, lc, sq_c, 0.0, sq_c * mm_c, 0.0)
    CASIM_APPLY(qr, nr, lr, sq_r, g_r, sq_r * mm_r, ng_r)
    CASIM_APPLY(qi, ni, li, sq_i, g_i, sq_i * mm_i, 0.0)
    CASIM_APPLY(qs, ns, ls, sq_s, g_s, sq_s * mm_s, ng_s)
    CASIM_APPLY(qg, ng, lg, sq_g, g_g, sq_g * mm_g, ng_g)
#undef CASIM_APPLY
    w.T += dTh; d.T += dTh;
}


// ---- surrogate interface: gates and features of a post-adjustment state ----
// Bit j is set when rate j's condition holds (the same conditions the plain
// rates test); bit 12 when the point is supersaturated over ice.
__device__ __forceinline__ unsigned gate_bits(const DevParams &P, bool warm, const Pt &w, double p, double esl) {
    const double qmin = P.q_min;
    const bool cP = w.qc >= qmin, rP = w.qr >= qmin;
    const bool iP = !warm && w.qi >= qmin, sP = !warm && w.qs >= qmin, gP = !warm && w.qg >= qmin;
    const bool cold = !warm && w.T < P.T_0, hot = !warm && w.T > P.T_0;
    unsigned g = 0;
    if (cP && w.nc > 0.0) g |= 1u << AUTO;
    if (cP && rP) g |= 1u << ACCR;
    if (rP && w.qc == 0.0 && sat_m1(P, w.qv, esl, p) < 0.0) g |= 1u << REVP;
    if (iP && cold) g |= (1u << DEPI);
    if (sP && cold) g |= (1u << DEPS);
    if (iP && cold && w.qi > P.q_i0) g |= 1u << IAUT;
    if (sP && iP && cold) g |= 1u << SACI;
    if (sP && cP && cold) g |= 1u << SACW;
    if (gP && cP && cold) g |= 1u << GACW;
    if (rP && cold) g |= 1u << FRZR;
    if (sP && hot) g |= 1u << SMLT;
    if (gP && hot) g |= 1u << GMLT;
    if (cold && (iP || sP) && sat_m1(P, w.qv, esat_ice(P, w.T), p) > 0.0) g |= CASIM_GATE_SUPERSAT_ICE;
    return g;
}

// ln T, ln p, ln rho, ln(q + 1e-12) for v, c; ln(n + 1) for c; (q, n) for r
// and i; q for s and g.  The features are float32, so the float32 hardware
// logarithm (v_log_f32, base 2) is accurate enough.
__device__ __forceinline__ float flog(double x) { return __builtin_amdgcn_logf((float)x) * 0.69314718055994531f; }

__device__ __forceinline__ void features(const Pt &w, double p, double rho, float f[12]) {
    const double qf = kQFloor;
    f[0] = flog(w.T);
    f[1] = flog(p);
    f[2] = flog(rho);
    f[3] = flog(w.qv + qf);
    f[4] = flog(w.qc + qf);
    f[5] = flog(w.nc + 1.0);
    f[6] = flog(w.qr + qf);
    f[7] = flog(w.nr + 1.0);
    f[8] = flog(w.qi + qf);
    f[9] = flog(w.ni + 1.0);
    f[10] = flog(w.qs + qf);
    f[11] = flog(w.qg + qf);
}

// Smallest limiter factor min_x min(1, q_x / (R_x dt)) over the source
// categories for rates r.
__device__ __forceinline__ double limiter_min_f(const Pt &w, const double r[12], double dt) {
    const double depi_v = r[DEPI] > 0.0 ? r[DEPI] : 0.0, depi_i = r[DEPI] < 0.0 ? -r[DEPI] : 0.0;
    const double deps_v = r[DEPS] > 0.0 ? r[DEPS] : 0.0, deps_s = r[DEPS] < 0.0 ? -r[DEPS] : 0.0;
    const double R[6] = {depi_v + deps_v, r[AUTO] + r[ACCR] + r[SACW] + r[GACW], r[REVP] + r[FRZR],
                         r[IAUT] + r[SACI] + depi_i, r[SMLT] + deps_s, r[GMLT]};
    const double q[6] = {w.qv, w.qc, w.qr, w.qi, w.qs, w.qg};
    double f = 1.0;
#pragma unroll
    for (int c = 0; c < 6; ++c)
        if (R[c] * dt > q[c]) f = ::fmin(f, q[c] * rcp64(R[c] * dt));
    return f;
}

// ---- sedimentation of one category over one chunk --------------------------
// Mass- and number-weighted fall speeds a Gamma(4+b)/6 lambda^-b and
// a Gamma(1+b) lambda^-b, times (rho_0/rho)^1/2, capped at v_max.
// carry_in: some flux of this category left the chunk above (its carries in
// LDS are not all zero).  Returns whether some flux leaves this chunk.  With
// no flux entering and no lane holding mass at or above q_min, every flux of
// every substep is zero (mass moves at most one level per substep, and only
// out of a level at or above q_min), so the chunk is skipped: its carries
// stay the zeros they are, and q, n and the tendencies stay as they are.
template <class R, int C>
__device__ __forceinline__ bool sediment(const DevParams &P, int cat, int ns, double dts, double *lds,
                                         int g, int c, bool need, double rho, double ln_rho, double rfac,
                                         double inv_rdz, bool surf, bool carry_in, double &q, double &n,
                                         double &dq, double &dn, double *psq, double *psn, bool &out_nz) {
    using M = Mth<R>;
    constexpr int L = kWave / C;
    if (!carry_in && __ballot((int)(need && q >= P.q_min)) == 0ull) return false;
    bool nz = false;
    double *cq = lds;                 // [s][c] flux of mass leaving the previous chunk
    double *cn = lds + ns * C;        // [s][c] flux of number
    const R ln_coef = R(P.ln_lam_coef[cat]), lo = R(P.ln_lam_lo[cat]), hi = R(P.ln_lam_hi[cat]);
    const R mb = R(-P.fall_b[cat]), vqc = R(P.vq_coef[cat]), vnc = R(P.vn_coef[cat]), vmax = R(P.v_max[cat]);
    for (int s = 0; s < ns; ++s) {
        double Fq = 0.0, Fn = 0.0;
        if (need && q >= P.q_min) {
            R ll;
            if (cat < 2) ll = (ln_coef + M::log(rdiv(R(n), R(q)))) * R(1.0 / 3.0);
            else         ll = (ln_coef - R(ln_rho) - M::log(R(q))) * R(0.25);
            ll = clampv(ll, lo, hi);
            const R e = M::exp(mb * ll) * R(rfac);
            const double vq = double(M::fmin(vqc * e, vmax));
            const double vn = double(M::fmin(vnc * e, vmax));
            Fq = rho * q * vq;
            Fn = rho * n * vn;
        }
        double in_q, in_n;
        if constexpr (L == 1) {
            in_q = cq[s * C + c];
            in_n = cn[s * C + c];
        } else {
            const double up_q = __shfl_up(Fq, C), up_n = __shfl_up(Fn, C);
            const double cr_q = cq[s * C + c], cr_n = cn[s * C + c];
            in_q = g == 0 ? cr_q : up_q;
            in_n = g == 0 ? cr_n : up_n;
        }
        if (need) {
            const double iq = dts * (in_q - Fq) * inv_rdz;
            const double in_ = dts * (in_n - Fn) * inv_rdz;
            q += iq; dq += iq; n += in_; dn += in_;
        }
        if (g == L - 1) { cq[s * C + c] = Fq; cn[s * C + c] = Fn; }
        nz |= (Fq != 0.0) | (Fn != 0.0);
        if (surf) { *psq += Fq * dts; *psn += Fn * dts; }
    }
    out_nz |= nz;
    return __ballot((int)(g == L - 1 && nz)) != 0ull;
}

// Kernel variants: VAR_GENERIC takes the constants and the stage/warm
// switches at run time; VAR_COLD and VAR_WARM have the default constants and
// all four stages compiled in (cold or warm configuration), which keeps the
// switches and constants out of the scalar registers.
enum { VAR_GENERIC = 0, VAR_COLD = 1, VAR_WARM = 2 };

// Where the 12 rates of an active point come from: evaluated in the sweep
// (SRC_PLAIN), the surrogate network's output for the point's slot
// (SRC_NET), or the dense rate kernel's output for its slot (SRC_DENSE).
// SRC_STREAM is the step's memory traffic without its physics: the same
// tiles, launch order, activity test and loads (the 6 extra fields where a
// chunk is busy), then 12 stores of zeros per point -- the streaming floor
// of the step's own access pattern (a diagnostic; it computes nothing).
enum { SRC_PLAIN = 0, SRC_NET = 1, SRC_DENSE = 2, SRC_STREAM = 3 };

template <bool MIX, int VAR, int C, int SRC>
__global__ __launch_bounds__(256, (MIX && VAR != VAR_GENERIC) ? 4 : 3) void sweep_kernel(DevParams Prt, SweepArgs a) {
    using R = typename std::conditional<MIX, float, double>::type;
    constexpr int L = kWave / C;
    constexpr bool FAST = VAR != VAR_GENERIC;
    const DevParams &P = params<FAST>(Prt);
    extern __shared__ double lds_all[];
    // the layer thicknesses, one copy per block at the start of the dynamic
    // LDS (a fixed address: no register holds it), the wavefronts' carries
    // after them (read per busy chunk; a global load there would wait on the
    // vector memory counter, and with it on the next chunk's loads)
    double *const lds_dz = lds_all;
    for (int j = threadIdx.x; j < a.nlev; j += blockDim.x) lds_dz[j] = a.dz[j];
    load_math_tables();          // ends with a block barrier
    const int lane = threadIdx.x & (kWave - 1);
    const int wib = threadIdx.x / kWave;
    const int g = lane / C, c = lane % C;
    double *lds = lds_all + a.nlev + (size_t)wib * (a.nslots + 8) * C;
    // wavefront -> tile of C columns: the virtual position of the wavefront
    // (XCD groups, see virtual_block), then the launch order derived from the
    // previous step's activity, else the identity (a corrupt entry falls back
    // to the identity, so no wavefront can leave the domain)
    const uint32_t vb = virtual_block(blockIdx.x, xcd_map(gridDim.x, (uint32_t)a.nxcd, (uint32_t)a.xcd_group));
    const int64_t wave_id = (int64_t)vb * (blockDim.x / kWave) + wib;
    int64_t tile = wave_id;
    if (a.order && wave_id < a.ntiles) {
        const int64_t o = a.order[wave_id];
        tile = (o >= 0 && o < a.ntiles) ? o : wave_id;
    }
    const int64_t col = tile * C + c;
    const bool colvalid = col < a.ncol;
    bool wave_busy = false;
    const double dt = a.dt, inv_dt = 1.0 / dt;
    const bool warm = FAST ? VAR == VAR_WARM : a.warm != 0;
    const int ncat = warm ? 1 : 4;
    const bool do_adj = FAST || (a.stages & CASIM_STAGE_ADJUST), do_sat = FAST || (a.stages & CASIM_STAGE_SATADJ);
    const bool do_rates = FAST || (a.stages & CASIM_STAGE_RATES), do_sed = FAST || (a.stages & CASIM_STAGE_SED);

    for (int j = lane; j < (a.nslots + 8) * C; j += kWave) lds[j] = 0.0;
    unsigned long long carry_cols = 0;   // bit c: a flux enters column c's next chunk from above
    unsigned carry_cat = 0;              // bit j: a flux of category j enters the next chunk
    const unsigned long long cmask = (C == 64) ? ~0ull : ((1ull << C) - 1ull);
    // surface sums of the wave's columns, [8][C] in LDS after the carries
    double *psurf = lds + (size_t)a.nslots * C + c;
    // the lane holding level 0 of its column accumulates and writes the surface sums
    const bool surf_lane = colvalid && g == (a.nlev - 1) % L;
    unsigned newton_bad = 0, nonfinite = 0, n_fallback = 0, n_inferred = 0;

    // Every field of the next chunk is loaded while the current one is
    // processed: the 8 that decide activity for all lanes, the other 6 for
    // lanes whose column was busy in this chunk (the next chunk of a busy
    // column is usually busy too).  A lane that turns busy without them loads
    // them itself.  Loading ahead keeps a chunk from waiting on the previous
    // chunk's stores, which share the vector-memory counter with loads.
    // With rates from a slot (SRC_NET, SRC_DENSE) the point's slot index comes
    // one chunk ahead too, which takes one of the two dependent loads of a
    // slotted point off the chunk's critical path.
    struct Ahead { double T, p, qv, qc, qr, qi, qs, qg, rho, nc, nr, ni, ns, ng; bool extra; int slot; };
    auto load_ahead = [&](int kk0, bool extra) {
        Ahead v{0.0, 1.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 0.0, 0.0, false, -1};
        const int kk = kk0 - g;
        if (colvalid && kk >= 0) {
            if constexpr (SRC != SRC_PLAIN) v.slot = a.sur_idx[(int64_t)kk * a.ncol + col];
            // the warm configuration never reads the ice, snow and graupel fields
            const int64_t jx = (int64_t)kk * a.ld + col;
            v.T = ldnt(a.in[0] + jx); v.p = ldnt(a.in[1] + jx); v.qv = ldnt(a.in[3] + jx);
            v.qc = ldnt(a.in[4] + jx); v.qr = ldnt(a.in[6] + jx);
            if (!warm) { v.qi = ldnt(a.in[8] + jx); v.qs = ldnt(a.in[10] + jx); v.qg = ldnt(a.in[12] + jx); }
            if (extra) {
                v.rho = ldnt(a.in[2] + jx);
                v.nc = ldnt(a.in[5] + jx); v.nr = ldnt(a.in[7] + jx);
                if (!warm) { v.ni = ldnt(a.in[9] + jx); v.ns = ldnt(a.in[11] + jx); v.ng = ldnt(a.in[13] + jx); }
                v.extra = true;
            }
        }
        return v;
    };
    // the 6 other fields of the next chunk into v (for a lane whose column is busy)
    auto load_extra = [&](Ahead &v, int kk0) {
        const int kk = kk0 - g;
        if (colvalid && kk >= 0) {
            const int64_t jx = (int64_t)kk * a.ld + col;
            v.rho = ldnt(a.in[2] + jx);
            v.nc = ldnt(a.in[5] + jx); v.nr = ldnt(a.in[7] + jx);
            if (!warm) { v.ni = ldnt(a.in[9] + jx); v.ns = ldnt(a.in[11] + jx); v.ng = ldnt(a.in[13] + jx); }
            v.extra = true;
        }
    };
    Ahead nxt = load_ahead(a.nlev - 1, false);

    for (int k0 = a.nlev - 1; k0 >= 0; k0 -= L) {
        const int k = k0 - g;
        const bool vp = colvalid && k >= 0;
        const int64_t ix = (int64_t)(k < 0 ? 0 : k) * a.ld + col;
        const Ahead cur = nxt;
        Pt w{}, d{};
        double p = 1.0, rho = 1.0, es_l = 1.0;
        bool act = false;
        if (vp) {
            w.T = cur.T; p = cur.p; w.qv = cur.qv;
            w.qc = cur.qc; w.qr = cur.qr; w.qi = cur.qi;
            w.qs = cur.qs; w.qg = cur.qg;
            act = (w.qc > 0.0) | (w.qr > 0.0) | (!warm & ((w.qi > 0.0) | (w.qs > 0.0) | (w.qg > 0.0)));
            es_l = esat_liq(P, w.T);
            // a condensate-free point changes only if supersaturated
            if (!act && do_sat) act = supersat(P, w.qv, es_l, p);
            if (!act && do_adj && !warm && w.T < P.T_nuc) act = supersat(P, w.qv, esat_ice(P, w.T), p);
        }
        const double T_in = w.T;
        const unsigned long long bal = __ballot((int)act);
        if constexpr (SRC == SRC_STREAM) {
            // the loads a busy chunk makes, stores of zeros (0 * x keeps the loads)
            double x = 0.0;
            bool busy_col = false;
            if (bal != 0ull) {
                unsigned long long cb = 0;
#pragma unroll
                for (int gg = 0; gg < L; ++gg) cb |= (bal >> (gg * C)) & cmask;
                busy_col = (cb >> c) & 1ull;
                if (vp && (act || busy_col))
                    x = cur.extra ? cur.rho + cur.nc + cur.nr + cur.ni + cur.ns + cur.ng
                                  : a.in[2][ix] + a.in[5][ix] + a.in[7][ix] + a.in[9][ix] + a.in[11][ix] +
                                        a.in[13][ix];
                wave_busy = true;
            }
            nxt = load_ahead(k0 - L, busy_col);
            if (vp) {
#pragma unroll
                for (int f = 0; f < CASIM_NTEND; ++f) stnt(a.tend[f] + ix, 0.0 * x);
            }
            continue;
        }
        if (bal == 0ull && carry_cols == 0ull) {
            nxt = load_ahead(k0 - L, false);
            if (vp) {
#pragma unroll
                for (int f = 0; f < CASIM_NTEND; ++f) stnt(a.tend[f] + ix, 0.0);
            }
            continue;
        }
        wave_busy = true;
        unsigned long long colbits = carry_cols;
#pragma unroll
        for (int gg = 0; gg < L; ++gg) colbits |= (bal >> (gg * C)) & cmask;
        const bool col_busy = (colbits >> c) & 1ull;
        const bool need = vp && (act || col_busy);
        double ln_rho = 0.0;
        if (need) {
            if (cur.extra) {
                rho = cur.rho;
                w.nc = cur.nc; w.nr = cur.nr; w.ni = cur.ni; w.ns = cur.ns; w.ng = cur.ng;
            } else {
                rho = a.in[2][ix];
                w.nc = a.in[5][ix]; w.nr = a.in[7][ix];
                if (!warm) { w.ni = a.in[9][ix]; w.ns = a.in[11][ix]; w.ng = a.in[13][ix]; }
            }
        }
        // The binary64 kernel issues the next chunk's 8 activity fields before
        // the point physics (longest cover of their latency) and its other 6
        // after it: all 14 held through the physics spilled registers.  The
        // mixed kernel issues all of them after it, which keeps them out of
        // the registers of the rate block and lets the kernel fit 128 VGPRs
        // (4 wavefronts per SIMD; measured faster).
        if constexpr (!MIX) nxt = load_ahead(k0 - L, false);
        if (need) ln_rho = log64(rho);
        const double rfac = ::sqrt(P.rho_0 * rcp64(rho));
        const int slot = cur.slot;
        if (act) {
            if (do_adj) adjust(P, warm, w, d, p, rho);
            double es_now = es_l;
            if (do_sat) newton_bad += satadj(P, a.newton_iters, w, d, p, T_in, es_l, es_now) ? 1u : 0u;
            if (do_rates) {
                // without the adjustment stage the clean-up may still have moved T
                if (!do_sat && w.T != T_in) es_now = esat_liq(P, w.T);
                bool plain = SRC == SRC_PLAIN;
                if constexpr (SRC == SRC_DENSE) {
                    // no slot: every rate gate is closed and all 12 rates are zero
                    if (slot >= 0) {
                        double rr[12];
#pragma unroll
                        for (int j = 0; j < 12; ++j) rr[j] = a.cmp_rates[(int64_t)j * a.cmp_ld + slot];
                        apply_rates<double>(P, w, d, rr, dt);
                    }
                }
                if constexpr (SRC == SRC_NET) {
                    plain = true;
                    // network rates for this point, unless it falls back
                    if (slot >= 0) {
                        // the slot's 12 rates (48 bytes: three 16-byte loads,
                        // all of them whatever the gates, whose closed rates
                        // are zero) and its flag, issued together and waited
                        // for once (the empty asm keeps the compiler from
                        // moving the rate loads behind the flag's test, which
                        // costs a second round trip)
                        const f32x4 *src = reinterpret_cast<const f32x4 *>(a.sur_rates + (int64_t)slot * 12);
                        f32x4 v0 = src[0], v1 = src[1], v2 = src[2];
                        int fbv = a.sur_fallback[slot];
                        asm volatile("" : "+v"(v0), "+v"(v1), "+v"(v2), "+v"(fbv));
                        bool use = fbv == 0;
                        if (use) {
                            const unsigned gb = gate_bits(P, warm, w, p, es_now);
                            const float f[12] = {v0[0], v0[1], v0[2], v0[3], v1[0], v1[1], v1[2], v1[3],
                                                 v2[0], v2[1], v2[2], v2[3]};
                            double rr[12];
#pragma unroll
                            for (int j = 0; j < 12; ++j) rr[j] = ((gb >> j) & 1u) ? (double)f[j] : 0.0;
                            use = limiter_min_f(w, rr, dt) >= a.sur_f_min;
                            if (use) {
                                apply_rates<double>(P, w, d, rr, dt);
                                plain = false;
                                ++n_inferred;
                            }
                        }
                        if (!use) ++n_fallback;
                    }
                }
                if (plain) {
                    R r[12];
                    rates<R>(P, warm, w, p, rho, ln_rho, rfac, es_now, r);
                    apply_rates<R>(P, w, d, r, dt);
                }
            }
        }
        if constexpr (MIX) nxt = load_ahead(k0 - L, col_busy);
        else if (col_busy) load_extra(nxt, k0 - L);
        bool out_nz = false;
        if (do_sed) {
            double inv_rdz = 0.0;
            if (need) inv_rdz = rcp64(rho * lds_dz[k < 0 ? 0 : k]);
            const bool surf = vp && k == 0;
            unsigned cc = 0;
            cc |= sediment<R, C>(P, 0, a.nsub[0], a.dts[0], lds + a.slot0[0] * C, g, c, need, rho, ln_rho,
                                 rfac, inv_rdz, surf, carry_cat & 1u, w.qr, w.nr, d.qr, d.nr, psurf + 0 * C,
                                 psurf + 4 * C, out_nz) ? 1u : 0u;
            if (ncat > 1) {
                cc |= sediment<R, C>(P, 1, a.nsub[1], a.dts[1], lds + a.slot0[1] * C, g, c, need, rho, ln_rho,
                                     rfac, inv_rdz, surf, carry_cat & 2u, w.qi, w.ni, d.qi, d.ni, psurf + 1 * C,
                                     psurf + 5 * C, out_nz) ? 2u : 0u;
                cc |= sediment<R, C>(P, 2, a.nsub[2], a.dts[2], lds + a.slot0[2] * C, g, c, need, rho, ln_rho,
                                     rfac, inv_rdz, surf, carry_cat & 4u, w.qs, w.ns, d.qs, d.ns, psurf + 2 * C,
                                     psurf + 6 * C, out_nz) ? 4u : 0u;
                cc |= sediment<R, C>(P, 3, a.nsub[3], a.dts[3], lds + a.slot0[3] * C, g, c, need, rho, ln_rho,
                                     rfac, inv_rdz, surf, carry_cat & 8u, w.qg, w.ng, d.qg, d.ng, psurf + 3 * C,
                                     psurf + 7 * C, out_nz) ? 8u : 0u;
            }
            carry_cat = cc;
        }
        carry_cols = (__ballot((int)(g == L - 1 && out_nz)) >> ((L - 1) * C)) & cmask;
        if (vp) {
            const double o[12] = {d.T * inv_dt, d.qv * inv_dt, d.qc * inv_dt, d.nc * inv_dt,
                                  d.qr * inv_dt, d.nr * inv_dt, d.qi * inv_dt, d.ni * inv_dt,
                                  d.qs * inv_dt, d.ns * inv_dt, d.qg * inv_dt, d.ng * inv_dt};
            double sum = 0.0;
#pragma unroll
            for (int f = 0; f < CASIM_NTEND; ++f) { stnt(a.tend[f] + ix, o[f]); sum += ::fabs(o[f]); }
            nonfinite += ::isfinite(sum) ? 0u : 1u;
        }
    }
    if (surf_lane) {
#pragma unroll
        for (int j = 0; j < 8; ++j) a.sfc[j][col] = psurf[j * C];
    }
    if (a.tile_busy && lane == 0) {            // lane 0 holds column c = 0 of the tile
        const int64_t t = col / C;
        if (t < a.ntiles) a.tile_busy[t] = wave_busy ? 1 : 0;
    }
    if (newton_bad) atomicAdd(&a.status[0], (unsigned long long)newton_bad);
    if (nonfinite) atomicAdd(&a.status[1], (unsigned long long)nonfinite);
    if (n_fallback) atomicAdd(&a.status[2], (unsigned long long)n_fallback);
    if (n_inferred) atomicAdd(&a.status[3], (unsigned long long)n_inferred);
}

// ---- point-parallel passes: rate samples and surrogate inputs -------------
// One thread per point p = k*ncol + c.  POINT_COUNT counts the points a dump
// selects per 256-point block; POINT_DUMP writes each selected point's
// features, plain binary64 rates (as float32) and gate word at its block
// offset plus its rank in the block (point order, so the output does not
// depend on scheduling); POINT_SURR computes features and gates of every
// point where a rate can be non-zero, reserves it a slot and records the slot
// in idx_map.
// One 256-point block lb of the pass (all threads of the block call it).
__device__ __forceinline__ void point_block(const DevParams &P, const PointArgs &pa, int64_t lb, int *wave_cnt) {
    const SweepArgs &a = pa.s;
    const int64_t pid = lb * 256 + threadIdx.x;
    const int64_t npts = (int64_t)a.nlev * a.ncol;
    const bool valid = pid < npts;
    const int64_t k = valid ? pid / a.ncol : 0, col = valid ? pid - k * a.ncol : 0;
    const int64_t ix = k * a.ld + col;
    const bool warm = a.warm != 0;
    const bool do_adj = a.stages & CASIM_STAGE_ADJUST, do_sat = a.stages & CASIM_STAGE_SATADJ;
    Pt w{}, d{};
    double p = 1.0, rho = 1.0, es_l = 1.0;
    bool act = false;
    if (valid) {
        w.T = a.in[0][ix]; p = a.in[1][ix]; w.qv = a.in[3][ix];
        w.qc = a.in[4][ix]; w.qr = a.in[6][ix]; w.qi = a.in[8][ix];
        w.qs = a.in[10][ix]; w.qg = a.in[12][ix];
        act = (w.qc > 0.0) | (w.qr > 0.0) | (!warm & ((w.qi > 0.0) | (w.qs > 0.0) | (w.qg > 0.0)));
        es_l = esat_liq(P, w.T);
        if (!act && do_sat) act = supersat(P, w.qv, es_l, p);
        if (!act && do_adj && !warm && w.T < P.T_nuc) act = supersat(P, w.qv, esat_ice(P, w.T), p);
    }
    // slotted passes take every active point; the rate dump draws a sample
    const bool slotted = pa.mode == POINT_SURR || pa.mode == POINT_CSTATE;
    bool sel = act;
    if (!slotted) sel = act && hash_uniform(pa.seed, (uint64_t)pid) < pa.keep;
    unsigned g = 0;
    float f[12];
    double r[12];
    double es_now = es_l;
    if (sel) {
        rho = a.in[2][ix];
        w.nc = a.in[5][ix]; w.nr = a.in[7][ix]; w.ni = a.in[9][ix];
        w.ns = a.in[11][ix]; w.ng = a.in[13][ix];
        const double T_in = w.T;
        if (do_adj) adjust(P, warm, w, d, p, rho);
        if (do_sat) satadj(P, a.newton_iters, w, d, p, T_in, es_l, es_now);
        if (!do_sat && w.T != T_in) es_now = esat_liq(P, w.T);
        g = gate_bits(P, warm, w, p, es_now);
        if (slotted) sel = (g & 0xFFFu) != 0;
        if (sel && pa.mode != POINT_CSTATE) {
            features(w, p, rho, f);
            if (pa.mode == POINT_DUMP)
                rates<double>(P, warm, w, p, rho, log64(rho), ::sqrt(P.rho_0 / rho), es_now, r);
        }
    }
    // rank of this point among the selected ones of its wave and block
    const unsigned long long bal = __ballot((int)sel);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int in_wave = __popcll(bal & ((1ull << lane) - 1ull));
    if (slotted) {
        // one atomic per wavefront reserves the wave's slots; a point's slot is
        // the wave's base plus its rank among the selected lanes (mbcnt)
        const int64_t region = lb % kSlotRegions;
        unsigned long long base = 0;
        if (lane == 0 && bal)
            base = atomicAdd(pa.counter + region * kCounterStride, (unsigned long long)__popcll(bal));
        base = __shfl(base, 0);
        const int64_t slot = region * pa.rcap + (int64_t)(base + in_wave);
        if (valid) pa.idx_map[pid] = sel ? (int32_t)slot : -1;
        if (sel) {
            if (pa.mode == POINT_SURR) {
#pragma unroll
                for (int j = 0; j < 12; ++j) pa.feat[slot * 12 + j] = f[j];
                pa.gates[slot] = (uint16_t)g;
            } else {
                const double v[kCmpState] = {w.T, p, rho, w.qv, w.qc, w.nc, w.qr, w.nr,
                                             w.qi, w.ni, w.qs, w.qg, es_now};
#pragma unroll
                for (int j = 0; j < kCmpState; ++j) pa.cstate[(int64_t)j * a.cmp_ld + slot] = v[j];
            }
        }
        return;
    }
    if (lane == 0) wave_cnt[wv] = __popcll(bal);
    __syncthreads();
    if (pa.mode == POINT_COUNT) {
        if (threadIdx.x == 0) pa.block_counts[lb] = wave_cnt[0] + wave_cnt[1] + wave_cnt[2] + wave_cnt[3];
        return;
    }
    int before = 0;
    for (int j = 0; j < wv; ++j) before += wave_cnt[j];
    if (sel) {
        const int64_t pos = pa.block_offsets[lb] + before + in_wave;
        if (pos < pa.max_out) {
#pragma unroll
            for (int j = 0; j < 12; ++j) {
                pa.feat[pos * 12 + j] = f[j];
                pa.rates[pos * 12 + j] = (float)r[j];
            }
            pa.gates[pos] = (uint16_t)g;
        }
    }
}

// The blocks of the pass loop over the 256-point blocks, so that the math
// tables are copied into LDS once per resident block, not once per 256 points.
template <bool FAST>
__global__ __launch_bounds__(256) void point_kernel(DevParams Prt, PointArgs pa) {
    const DevParams &P = params<FAST>(Prt);
    load_math_tables();
    __shared__ int wave_cnt[4];
    const int64_t nlb = ((int64_t)pa.s.nlev * pa.s.ncol + 255) / 256;
    for (int64_t lb = blockIdx.x; lb < nlb; lb += gridDim.x) {
        point_block(P, pa, lb, wave_cnt);
        __syncthreads();                       // wave_cnt is reused
    }
}

// The 12 binary64 rates of compacted points, one point per lane with every
// lane of a wavefront busy (grid-stride over the slots the point pass filled).
// ln rho and (rho_0/rho)^1/2 are formed exactly as in the sweep.
template <bool FAST>
__global__ __launch_bounds__(256) void dense_rates_kernel(DevParams Prt, const double *cs, int64_t ld,
                                                          const unsigned long long *counters, int64_t rcap,
                                                          double *out, int warm_i) {
    const DevParams &P = params<FAST>(Prt);
    load_math_tables();
    const bool warm = warm_i != 0;
    // block r works through region r (one block per region)
    const int64_t r = blockIdx.x;
    const unsigned long long c = counters[r * kCounterStride];
    const int64_t n = (int64_t)(c < (unsigned long long)rcap ? c : (unsigned long long)rcap);
    for (int64_t i0 = threadIdx.x; i0 < n; i0 += blockDim.x) {
        const int64_t i = r * rcap + i0;
        Pt w{};
        w.T = cs[i];
        const double p = cs[ld + i], rho = cs[2 * ld + i];
        w.qv = cs[3 * ld + i]; w.qc = cs[4 * ld + i]; w.nc = cs[5 * ld + i];
        w.qr = cs[6 * ld + i]; w.nr = cs[7 * ld + i]; w.qi = cs[8 * ld + i];
        w.ni = cs[9 * ld + i]; w.qs = cs[10 * ld + i]; w.qg = cs[11 * ld + i];
        const double es = cs[12 * ld + i];
        double r[12];
        rates<double>(P, warm, w, p, rho, log64(rho), ::sqrt(P.rho_0 * rcp64(rho)), es, r);
#pragma unroll
        for (int j = 0; j < 12; ++j) out[(int64_t)j * ld + i] = r[j];
    }
}

hipError_t launch_dense_rates(const DevParams &P, bool fast, bool warm, const double *cstate, int64_t ld,
                              const unsigned long long *counters, int64_t rcap, double *rates, hipStream_t stream) {
    if (ld < (int64_t)kSlotRegions * rcap) return hipErrorInvalidValue;
    const dim3 grid(kSlotRegions), block(256);
    if (fast)
        hipLaunchKernelGGL(dense_rates_kernel<true>, grid, block, 0, stream, P, cstate, ld, counters, rcap, rates,
                           warm ? 1 : 0);
    else
        hipLaunchKernelGGL(dense_rates_kernel<false>, grid, block, 0, stream, P, cstate, ld, counters, rcap, rates,
                           warm ? 1 : 0);
    return hipGetLastError();
}

__global__ void zero_u64_kernel(unsigned long long *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

hipError_t launch_zero_u64(unsigned long long *p, int64_t n, hipStream_t stream) {
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(zero_u64_kernel, dim3((unsigned)(blocks < 1 ? 1 : blocks)), dim3(256), 0, stream, p, n);
    return hipGetLastError();
}

// Exclusive prefix sum of n block counts in one block (fixed order).
__global__ __launch_bounds__(256) void scan_kernel(const int64_t *counts, int64_t n, int64_t *offsets,
                                                   int64_t *total) {
    __shared__ int64_t part[256];
    const int64_t per = (n + 255) / 256;
    const int64_t b = threadIdx.x * per, e = b + per < n ? b + per : n;
    int64_t s = 0;
    for (int64_t i = b; i < e; ++i) s += counts[i];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t acc = 0;
        for (int j = 0; j < 256; ++j) { const int64_t v = part[j]; part[j] = acc; acc += v; }
        *total = acc;
    }
    __syncthreads();
    int64_t acc = part[threadIdx.x];
    for (int64_t i = b; i < e; ++i) { offsets[i] = acc; acc += counts[i]; }
}

// Launch order of the sweep's tiles for the next step.  The paper found a
// guided schedule best for the unequal work of its columns (Sec. IV); on the
// GPU the hardware hands out wavefronts in launch order, so a busy tile
// launched in the last round would end the kernel late.  Order: every tile
// that was busy in the previous step and the clear tiles except the last
// `reserve` of them, in index order (so busy and clear tiles stay mixed for
// the overlap of arithmetic and streaming), then those reserved clear tiles,
// which fill the last dispatch round.  One block; busy[i] in {0, 1}.
// Exclusive prefix sum of one value per thread over a 1024-thread block
// (Hillis-Steele in LDS); *total receives the sum.
__device__ __forceinline__ int64_t block_exclusive_scan(int64_t v, int64_t *buf, int64_t *total) {
    const int t = threadIdx.x;
    buf[t] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int64_t add = t >= off ? buf[t - off] : 0;
        __syncthreads();
        buf[t] += add;
        __syncthreads();
    }
    const int64_t incl = buf[t];
    if (t == 1023) *total = incl;
    __syncthreads();
    return incl - v;
}

// One block per XCD x: the tiles of the wavefront positions x runs, in its
// dispatch order.
struct XcdPositions {
    XcdMap m;
    int32_t wpb;
    uint32_t x;
    __device__ int64_t operator()(int64_t i) const {       // i-th position of XCD x
        return (int64_t)xcd_block(x, (uint32_t)(i / wpb), m) * wpb + i % wpb;
    }
};

__global__ __launch_bounds__(1024) void tile_order_kernel(const int32_t *busy, int64_t ntiles, uint32_t nb,
                                                          int32_t wpb, int32_t nxcd, int32_t group,
                                                          int64_t reserve, int32_t *order) {
    __shared__ int64_t buf[1024];
    __shared__ int64_t total;
    const int t = threadIdx.x;
    const XcdPositions pos{xcd_map(nb, (uint32_t)nxcd, (uint32_t)group), wpb, blockIdx.x};
    // positions past the last tile are the last wavefronts of the last block
    int64_t n = (int64_t)xcd_blocks(blockIdx.x, pos.m) * wpb;
    while (n > 0 && pos(n - 1) >= ntiles) --n;
    if (n == 0) return;                        // the same for the whole block
    const int64_t per = (n + 1023) / 1024;
    const int64_t b = (int64_t)t * per < n ? (int64_t)t * per : n;
    const int64_t e = b + per < n ? b + per : n;
    int64_t nclear = 0;
    for (int64_t i = b; i < e; ++i) nclear += busy[pos(i)] == 0;
    // clear tiles of the XCD after this thread's part
    const int64_t before = block_exclusive_scan(nclear, buf, &total);
    const int64_t after = total - before - nclear;
    // reserved tiles of this part: clear, with at most `reserve` clear tiles at or after them
    int64_t ns = 0, suffix = after;
    for (int64_t i = e - 1; i >= b; --i)
        if (busy[pos(i)] == 0 && ++suffix <= reserve) ++ns;
    int64_t rank = block_exclusive_scan(ns, buf, &total);     // reserved tiles before this part
    const int64_t first_reserved = n - total;
    int64_t clear_seen = 0;
    for (int64_t i = b; i < e; ++i) {
        const int64_t tile = pos(i);
        const bool clear = busy[tile] == 0;
        const bool reserved = clear && after + (nclear - clear_seen) <= reserve;
        order[pos(reserved ? first_reserved + rank : i - rank)] = (int32_t)tile;
        rank += reserved;
        clear_seen += clear;
    }
}

hipError_t launch_tile_order(const int32_t *busy, const SweepGeometry &geo, int32_t nxcd, int32_t group,
                             int64_t reserve, int32_t *order, hipStream_t stream) {
    if (nxcd < 1 || group < 1 || geo.blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(tile_order_kernel, dim3((unsigned)nxcd), dim3(1024), 0, stream, busy, geo.tiles,
                       (uint32_t)geo.blocks, geo.wpb, nxcd, group, reserve, order);
    return hipGetLastError();
}

// X += dt * tend for the 12 prognostic fields; q and n clipped at 0.
__global__ __launch_bounds__(256) void apply_kernel(SweepArgs a, double dt, int64_t npts) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npts) return;
    const int64_t k = i / a.ncol, c = i - k * a.ncol;
    const int64_t ix = k * a.ld + c;
    double *T = const_cast<double *>(a.in[0]);
    T[ix] = T[ix] + dt * a.tend[0][ix];
#pragma unroll
    for (int f = 1; f < CASIM_NTEND; ++f) {
        double *x = const_cast<double *>(a.in[f + 2]);
        const double v = x[ix] + dt * a.tend[f][ix];
        x[ix] = v > 0.0 ? v : 0.0;
    }
}

namespace {

int env_int(const char *name, int dflt) {
    const char *e = getenv(name);
    return e ? atoi(e) : dflt;
}

template <bool MIX, int VAR, int SRC>
hipError_t launch_c(int C, dim3 grid, dim3 block, size_t lds, hipStream_t s, const DevParams &P,
                    const SweepArgs &a) {
    switch (C) {
        case 4: hipLaunchKernelGGL((sweep_kernel<MIX, VAR, 4, SRC>), grid, block, lds, s, P, a); break;
        case 8: hipLaunchKernelGGL((sweep_kernel<MIX, VAR, 8, SRC>), grid, block, lds, s, P, a); break;
        case 16: hipLaunchKernelGGL((sweep_kernel<MIX, VAR, 16, SRC>), grid, block, lds, s, P, a); break;
        case 32: hipLaunchKernelGGL((sweep_kernel<MIX, VAR, 32, SRC>), grid, block, lds, s, P, a); break;
        default: hipLaunchKernelGGL((sweep_kernel<MIX, VAR, 64, SRC>), grid, block, lds, s, P, a); break;
    }
    return hipGetLastError();
}

template <bool MIX, int SRC>
hipError_t launch_var(int var, int C, dim3 grid, dim3 block, size_t lds, hipStream_t s, const DevParams &P,
                      const SweepArgs &a) {
    if (var == VAR_COLD) return launch_c<MIX, VAR_COLD, SRC>(C, grid, block, lds, s, P, a);
    if (var == VAR_WARM) return launch_c<MIX, VAR_WARM, SRC>(C, grid, block, lds, s, P, a);
    return launch_c<MIX, VAR_GENERIC, SRC>(C, grid, block, lds, s, P, a);
}

// Columns per wavefront.  16-column tiles (16 x 4 levels, one 128-byte row
// per level) measured best for the binary64 kernel on the large domains;
// the FP32-mixed kernel, which runs at the streaming floor of its access
// pattern, gains from 32-column tiles (256-byte rows, 2 levels per chunk)
// on domains of at least 262,144 columns; narrower tiles keep at least 2048
// wavefronts (two per SIMD) on small ones.
int columns_per_wave(int64_t ncol, int mode) {
    const int forced = env_int("CASIM_COLS_PER_WAVE", 0);
    if (forced == 4 || forced == 8 || forced == 16 || forced == 32 || forced == 64) return forced;
    if (mode == CASIM_MODE_FP32MIX && ncol / 32 >= 8192) return 32;
    if (ncol / 16 >= 2048) return 16;
    if (ncol / 8 >= 2048) return 8;
    return 4;
}

}  // namespace

hipError_t sweep_geometry(int64_t ncol, int32_t nslots, int32_t nlev, int mode, SweepGeometry *geo) {
    const int C = columns_per_wave(ncol, mode);
    // narrow tiles: enough wavefronts per block to cover whole 128-byte rows,
    // so the halves of a line are fetched by one CU
    int wpb = env_int("CASIM_WAVES_PER_BLOCK", C >= 16 ? 1 : 16 / C);
    if (wpb < 1 || wpb > 4) wpb = 1;
    const size_t per_wave = (size_t)(nslots + 8) * C * sizeof(double);   // carries + surface sums
    const size_t dz_bytes = (size_t)nlev * sizeof(double);                 // layer thicknesses
    size_t lds = (size_t)wpb * per_wave + dz_bytes;
    // 64 KiB per block, the math tables included
    const size_t lds_max = 65536 - kMathLdsBytes;
    while (wpb > 1 && lds > lds_max) { --wpb; lds = (size_t)wpb * per_wave + dz_bytes; }
    if (lds > lds_max) return hipErrorInvalidValue;
    geo->C = C;
    geo->wpb = wpb;
    geo->tiles = (ncol + C - 1) / C;
    geo->blocks = (geo->tiles + wpb - 1) / wpb;
    geo->lds = lds;
    return geo->blocks > 0x7fffffff ? hipErrorInvalidValue : hipSuccess;
}

hipError_t launch_sweep(const DevParams &P, bool fast, const SweepArgs &a, hipStream_t stream) {
    SweepGeometry geo;
    const hipError_t ge = sweep_geometry(a.ncol, a.nslots, a.nlev, a.mode, &geo);
    if (ge != hipSuccess) return ge;
    if ((a.order || a.tile_busy) && a.ntiles != geo.tiles) return hipErrorInvalidValue;
    if (a.nxcd < 1 || a.xcd_group < 1) return hipErrorInvalidValue;
    const int C = geo.C;
    const dim3 grid((unsigned)geo.blocks), block(geo.wpb * kWave);
    const size_t lds = geo.lds;
    // the compiled-in variants need the default constants and all stages
    const int var = !(fast && a.stages == CASIM_STAGE_ALL) ? VAR_GENERIC : (a.warm ? VAR_WARM : VAR_COLD);
    if (a.mode == CASIM_MODE_FP32MIX) return launch_var<true, SRC_PLAIN>(var, C, grid, block, lds, stream, P, a);
    if (a.mode == CASIM_MODE_SURROGATE) return launch_var<false, SRC_NET>(var, C, grid, block, lds, stream, P, a);
    if (a.mode == CASIM_MODE_FP64_COMPACT)
        return launch_var<false, SRC_DENSE>(var, C, grid, block, lds, stream, P, a);
    if (a.mode == kModeStream) return launch_c<false, VAR_COLD, SRC_STREAM>(C, grid, block, lds, stream, P, a);
    return launch_var<false, SRC_PLAIN>(var, C, grid, block, lds, stream, P, a);
}

hipError_t launch_points(const DevParams &P, bool fast, const PointArgs &pa, hipStream_t stream) {
    const int64_t npts = (int64_t)pa.s.nlev * pa.s.ncol;
    // 32 blocks of 256 threads per compute unit of an MI355X, at most
    const int64_t blocks = ::min((npts + 255) / 256, (int64_t)8192);
    if (blocks == 0) return hipSuccess;
    if (fast) hipLaunchKernelGGL(point_kernel<true>, dim3((unsigned)blocks), dim3(256), 0, stream, P, pa);
    else hipLaunchKernelGGL(point_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, stream, P, pa);
    return hipGetLastError();
}

hipError_t launch_scan(const int64_t *counts, int64_t n, int64_t *offsets, int64_t *total, hipStream_t stream) {
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(256), 0, stream, counts, n, offsets, total);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void math_kernel(const double *x, int64_t n, double *e, double *l) {
    load_math_tables();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (e) e[i] = exp64(x[i]);
    if (l) l[i] = log64(x[i]);
}

hipError_t launch_math(const double *x, int64_t n, double *e, double *l, hipStream_t stream) {
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(math_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, x, n, e, l);
    return hipGetLastError();
}

hipError_t launch_apply(const SweepArgs &a, double dt, hipStream_t stream) {
    const int64_t n = (int64_t)a.nlev * a.ncol;
    const int threads = 256;
    const int64_t blocks = (n + threads - 1) / threads;
    hipLaunchKernelGGL(apply_kernel, dim3((unsigned)blocks), dim3(threads), 0, stream, a, dt, n);
    return hipGetLastError();
}

}  // namespace casim
