// Column-sweep kernels of the bulk-microphysics step for gfx950.
//
// Mapping (the paper's Sec. III-B mapping of one column per GPU thread, kept
// because columns are independent, Sec. II): one column per lane of a
// 64-wide wavefront, the lane walking its column from the top level down.
// At each level a lane
//   1. reads the 8 fields that decide whether anything can happen there
//      (T, p, q_v and the five condensate masses);
//   2. takes part in a wavefront ballot: when no lane of the wave has
//      condensate, supersaturation or sedimentation inflow at this level,
//      the wave writes exact zeros and moves on (clear sky costs 8 loads and
//      12 stores per point);
//   3. otherwise reads the remaining 6 fields and runs clean-up, instant
//      phase changes, saturation adjustment, the 12 process rates and the
//      limiter in registers;
//   4. advances sedimentation of rain, ice, snow and graupel for every
//      substep at once: explicit upwind sedimentation with a static substep
//      count needs, at level k and substep s, only the flux leaving level
//      k+1 at substep s, so the fluxes of the level above are carried down
//      in LDS, one slot per (category, moment, substep) and lane;
//   5. writes the 12 tendencies (accumulated increment / dt).
// The surface outputs are the fluxes leaving level 0, summed over substeps.
//
// Precision policy: MIX = false runs everything in binary64.  MIX = true
// evaluates the 12 process rates and the fall speeds in binary32 and keeps
// binary64 for saturation pressures, the saturation adjustment, the limiter
// and apply, the sedimentation fluxes, level updates and surface sums.
#include "casim_internal.h"

namespace casim {

template <class R> struct Mth;
template <> struct Mth<double> {
    static __device__ __forceinline__ double exp(double x) { return ::exp(x); }
    static __device__ __forceinline__ double pow(double x, double y) { return ::pow(x, y); }
    static __device__ __forceinline__ double cbrt(double x) { return ::cbrt(x); }
    static __device__ __forceinline__ double sqrt(double x) { return ::sqrt(x); }
    static __device__ __forceinline__ double fmin(double a, double b) { return ::fmin(a, b); }
    static __device__ __forceinline__ double fmax(double a, double b) { return ::fmax(a, b); }
};
template <> struct Mth<float> {
    static __device__ __forceinline__ float exp(float x) { return ::expf(x); }
    static __device__ __forceinline__ float pow(float x, float y) { return ::powf(x, y); }
    static __device__ __forceinline__ float cbrt(float x) { return ::cbrtf(x); }
    static __device__ __forceinline__ float sqrt(float x) { return ::sqrtf(x); }
    static __device__ __forceinline__ float fmin(float a, float b) { return ::fminf(a, b); }
    static __device__ __forceinline__ float fmax(float a, float b) { return ::fmaxf(a, b); }
};

template <class R>
__device__ __forceinline__ R clampv(R x, R lo, R hi) { return x < lo ? lo : (x > hi ? hi : x); }

// Working state of one point: values (w) and accumulated increments (d).
struct Pt {
    double T, qv, qc, nc, qr, nr, qi, ni, qs, ns, qg, ng;
};

__device__ __forceinline__ double esat_liq(const DevParams &P, double T) {
    double Tc = T - P.T_0;
    return P.esl_a * ::exp(P.esl_b * Tc / (Tc + P.esl_c));
}
__device__ __forceinline__ double esat_ice(const DevParams &P, double T) {
    double Tc = T - P.T_0;
    return P.esi_a * ::exp(P.esi_b * Tc / (Tc + P.esi_c));
}
__device__ __forceinline__ double q_of_e(const DevParams &P, double e, double p) {
    return P.eps * e / (p - P.one_m_eps * e);
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

__device__ __forceinline__ void adjust(const DevParams &P, Pt &w, Pt &d, double p, double rho) {
    cleanup(P, w, d, w.qc, d.qc, w.nc, d.nc, P.L_v);
    cleanup(P, w, d, w.qr, d.qr, w.nr, d.nr, P.L_v);
    if (P.warm) return;
    cleanup(P, w, d, w.qi, d.qi, w.ni, d.ni, P.L_s);
    cleanup(P, w, d, w.qs, d.qs, w.ns, d.ns, P.L_s);
    cleanup(P, w, d, w.qg, d.qg, w.ng, d.ng, P.L_s);
    // homogeneous freezing of all cloud
    if (w.T < P.T_hom && w.qc > 0.0) {
        double m = w.qc, nn = w.nc;
        d.qc -= m; w.qc = 0.0; d.nc -= nn; w.nc = 0.0;
        w.qi += m; d.qi += m; w.ni += nn; d.ni += nn;
        double h = P.L_f * m * P.inv_cp;
        w.T += h; d.T += h;
    }
    // melting of all ice
    if (w.T > P.T_0 && w.qi > 0.0) {
        double m = w.qi, nn = w.ni;
        d.qi -= m; w.qi = 0.0; d.ni -= nn; w.ni = 0.0;
        w.qc += m; d.qc += m; w.nc += nn; d.nc += nn;
        double h = -P.L_f * m * P.inv_cp;
        w.T += h; d.T += h;
    }
    // Cooper (1986) nucleation where ice-supersaturated
    if (w.T < P.T_nuc) {
        double qsi = q_of_e(P, esat_ice(P, w.T), p);
        if (w.qv > qsi) {
            double nin = ::fmin(P.cooper_a * ::exp(P.cooper_b * (P.T_0 - w.T)), P.cooper_max) / rho;
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
__device__ __forceinline__ bool satadj(const DevParams &P, Pt &w, Pt &d, double p) {
    double qsl = q_of_e(P, esat_liq(P, w.T), p);
    if (!(w.qv > qsl || w.qc > 0.0)) return false;
    double delta = 0.0;
    for (int it = 0; it < P.newton_iters; ++it) {
        double Tc = (w.T + delta) - P.T_0;
        double rtc = 1.0 / (Tc + P.esl_c);
        double es = P.esl_a * ::exp(P.esl_b * Tc * rtc);
        double rden = 1.0 / (p - P.one_m_eps * es);
        double qs = P.eps * es * rden;
        double f = P.cp * delta - P.L_v * (w.qv - qs);
        double fp = P.cp + P.L_v * qs * (p * rden) * P.esl_bc * (rtc * rtc);
        delta -= f / fp;
    }
    bool bad;
    {
        double qs = q_of_e(P, esat_liq(P, w.T + delta), p);
        double res = ::fabs(P.cp * delta - P.L_v * (w.qv - qs)) / (P.L_v * qs);
        bad = !(res <= P.newton_rtol);
    }
    double dq = P.cp * delta / P.L_v;
    if (w.qc + dq >= 0.0) {
        bool newcloud = (w.qc == 0.0 && dq > 0.0);
        w.qc += dq; d.qc += dq;
        w.qv -= dq; d.qv -= dq;
        w.T += delta; d.T += delta;
        if (newcloud) {
            double target = ::fmax(w.nc, P.n_act);
            double add = target - w.nc;
            w.nc += add; d.nc += add;
        }
    } else {
        double m = w.qc;
        w.qv += m; d.qv += m;
        double h = -P.L_v * m * P.inv_cp;
        w.T += h; d.T += h;
        d.qc -= m; w.qc = 0.0;
        d.nc -= w.nc; w.nc = 0.0;
    }
    return bad;
}

// ---- the 12 process rates ------------------------------------------------
enum { AUTO, ACCR, REVP, DEPI, DEPS, IAUT, SACI, SACW, GACW, FRZR, SMLT, GMLT };

template <class R>
__device__ __forceinline__ void rates(const DevParams &P, const Pt &w, double p, double rho,
                                      double rfac_d, R r[12]) {
    using M = Mth<R>;
#pragma unroll
    for (int j = 0; j < 12; ++j) r[j] = R(0);
    const double qmin = P.q_min;
    const bool cP = w.qc >= qmin, rP = w.qr >= qmin;
    const bool iP = !P.warm && w.qi >= qmin, sP = !P.warm && w.qs >= qmin, gP = !P.warm && w.qg >= qmin;
    if (!(cP || rP || iP || sP || gP)) return;
    const bool cold = !P.warm && w.T < P.T_0, hot = !P.warm && w.T > P.T_0;
    // saturation pressures and ratios in binary64
    const double esl = esat_liq(P, w.T), esi = esat_ice(P, w.T);
    const double Sl_m1 = w.qv / q_of_e(P, esl, p) - 1.0;
    const double Si_m1 = w.qv / q_of_e(P, esi, p) - 1.0;

    const R T = R(w.T), rh = R(rho), rf = R(rfac_d);
    const R dT0 = T - R(P.T_0);
    const R Dv = R(P.Dv0) * M::pow(T / R(P.T_0), R(P.Dv_exp)) * (R(1e5) / R(p));
    const R KRT2 = R(P.K_a) * R(P.R_v) * T * T;
    const R twopi = R(6.283185307179586);
    const R qc = R(w.qc), qr = R(w.qr), qi = R(w.qi), qs = R(w.qs), qg = R(w.qg);

    R lr = R(0), li = R(0), ls = R(0), lg = R(0);
    if (rP) lr = clampv(M::cbrt(R(P.lam_coef[0]) * R(w.nr) / qr), R(P.lam_lo[0]), R(P.lam_hi[0]));
    if (iP) li = clampv(M::cbrt(R(P.lam_coef[1]) * R(w.ni) / qi), R(P.lam_lo[1]), R(P.lam_hi[1]));
    if (sP) ls = clampv(M::sqrt(M::sqrt(R(P.lam_coef[2]) / (rh * qs))), R(P.lam_lo[2]), R(P.lam_hi[2]));
    if (gP) lg = clampv(M::sqrt(M::sqrt(R(P.lam_coef[3]) / (rh * qg))), R(P.lam_lo[3]), R(P.lam_hi[3]));

    if (cP && w.nc > 0.0) {
        const R Nc = R(w.nc) * rh * R(1e-6);
        r[AUTO] = R(P.auto_a) * M::pow(qc, R(P.auto_qc_exp)) * M::pow(Nc, R(P.auto_nc_exp));
    }
    if (cP && rP) r[ACCR] = R(P.accr_a) * M::pow(qc * qr, R(P.accr_exp));
    if (rP && w.qc == 0.0 && Sl_m1 < 0.0) {
        const R Gl = R(1) / (R(P.L_v) * R(P.L_v) / KRT2 + R(P.R_v) * T / (Dv * R(esl)));
        r[REVP] = twopi * Gl * R(-Sl_m1) * R(w.nr) / lr;
    }
    if (cold && (iP || sP)) {
        const R Gi = R(1) / (R(P.L_s) * R(P.L_s) / KRT2 + R(P.R_v) * T / (Dv * R(esi)));
        if (iP) r[DEPI] = twopi * Gi * R(Si_m1) * R(w.ni) / li;
        if (sP) r[DEPS] = twopi * Gi * R(Si_m1) * R(P.N0_s) / (rh * ls * ls);
    }
    if (cold) {
        const R eice = M::exp(R(P.ice_t_exp) * dT0);
        if (iP && w.qi > P.q_i0) r[IAUT] = R(P.iaut_a) * eice * (qi - R(P.q_i0));
        if (sP) {
            const R coll = R(P.coll_s) * M::pow(ls, -(R(3) + R(P.fall_b[2]))) * rf;
            if (iP) r[SACI] = eice * qi * coll;
            if (cP) r[SACW] = qc * coll;
        }
        if (gP && cP) r[GACW] = R(P.coll_g) * M::pow(lg, -(R(3) + R(P.fall_b[3]))) * rf * qc;
        if (rP) {
            const R n0r = rh * R(w.nr) * lr;
            const R l2 = lr * lr, l7 = l2 * l2 * l2 * lr;
            r[FRZR] = R(P.frzr_coef) * n0r / rh * (M::exp(R(P.bigg_a) * (R(P.T_0) - T)) - R(1)) / l7;
        }
    }
    if (hot) {
        const R melt = twopi * R(P.K_a) * dT0 / (rh * R(P.L_f));
        if (sP) r[SMLT] = melt * R(P.N0_s) / (ls * ls);
        if (gP) r[GMLT] = melt * R(P.N0_g) / (lg * lg);
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
    const double fv = lv ? w.qv / (Rv * dt) : 1.0, fc = lc ? w.qc / (Rc * dt) : 1.0;
    const double fr = lr ? w.qr / (Rr * dt) : 1.0, fi = li ? w.qi / (Ri * dt) : 1.0;
    const double fs = ls ? w.qs / (Rs * dt) : 1.0, fg = lg ? w.qg / (Rg * dt) : 1.0;
    const double auto_ = r[AUTO] * fc, accr = r[ACCR] * fc, sacw = r[SACW] * fc, gacw = r[GACW] * fc;
    const double revp = r[REVP] * fr, frzr = r[FRZR] * fr;
    const double iaut = r[IAUT] * fi, saci = r[SACI] * fi;
    const double smlt = r[SMLT] * fs, gmlt = r[GMLT] * fg;
    depi_v *= fv; deps_v *= fv; depi_i *= fi; deps_s *= fs;

    const double mm_c = w.qc > 0.0 ? w.nc / w.qc : 0.0;
    const double mm_r = w.qr > 0.0 ? w.nr / w.qr : 0.0;
    const double mm_i = w.qi > 0.0 ? w.ni / w.qi : 0.0;
    const double mm_s = w.qs > 0.0 ? w.ns / w.qs : 0.0;
    const double mm_g = w.qg > 0.0 ? w.ng / w.qg : 0.0;

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
    // vapour has no number
    if (lv) { d.qv -= w.qv; w.qv = 0.0; } else { w.qv -= sq_v; d.qv -= sq_v; }
    w.qv += g_v; d.qv += g_v;
    CASIM_APPLY(qc, nc, lc, sq_c, 0.0, sq_c * mm_c, 0.0)
    CASIM_APPLY(qr, nr, lr, sq_r, g_r, sq_r * mm_r, ng_r)
    CASIM_APPLY(qi, ni, li, sq_i, g_i, sq_i * mm_i, 0.0)
    CASIM_APPLY(qs, ns, ls, sq_s, g_s, sq_s * mm_s, ng_s)
    CASIM_APPLY(qg, ng, lg, sq_g, g_g, sq_g * mm_g, ng_g)
#undef CASIM_APPLY
    w.T += dTh; d.T += dTh;
}

// Fall speeds of category c (0..3 = r, i, s, g) for mass and number.
template <class R>
__device__ __forceinline__ void fall(const DevParams &P, int c, double q, double n, double rho,
                                     double rfac, double &vq, double &vn) {
    using M = Mth<R>;
    R lam;
    if (c < 2) lam = M::cbrt(R(P.lam_coef[c]) * R(n) / R(q));
    else       lam = M::sqrt(M::sqrt(R(P.lam_coef[c]) / (R(rho) * R(q))));
    lam = clampv(lam, R(P.lam_lo[c]), R(P.lam_hi[c]));
    const R lb = M::pow(lam, R(P.fall_b[c]));
    vq = double(M::fmin(R(P.vq_coef[c]) / lb * R(rfac), R(P.v_max[c])));
    vn = double(M::fmin(R(P.vn_coef[c]) / lb * R(rfac), R(P.v_max[c])));
}

// All substeps of one sedimenting category at one level.  carry holds, per
// (moment, substep), the flux that left the level above during that substep;
// on return it holds the fluxes leaving this level.
template <class R>
__device__ __forceinline__ void sediment(const DevParams &P, const SweepArgs &a, int c, double *carry,
                                         double rho, double rfac, double inv_rdz, bool surf,
                                         double &q, double &n, double &dq, double &dn,
                                         double &psq, double &psn, bool &out_nz) {
    const int ns = a.nsub[c];
    const double dts = a.dt / ns;
    double *cq = carry + (size_t)a.slot0[c] * kWave;
    double *cn = cq + (size_t)ns * kWave;
    for (int s = 0; s < ns; ++s) {
        double Fq = 0.0, Fn = 0.0;
        if (q >= P.q_min) {
            double vq, vn;
            fall<R>(P, c, q, n, rho, rfac, vq, vn);
            Fq = rho * q * vq;
            Fn = rho * n * vn;
        }
        const double iq = dts * (cq[s * kWave] - Fq) * inv_rdz;
        const double in_ = dts * (cn[s * kWave] - Fn) * inv_rdz;
        q += iq; dq += iq; n += in_; dn += in_;
        cq[s * kWave] = Fq; cn[s * kWave] = Fn;
        out_nz |= (Fq != 0.0) | (Fn != 0.0);
        if (surf) { psq += Fq * dts; psn += Fn * dts; }
    }
}

template <bool MIX>
__global__ __launch_bounds__(256) void sweep_kernel(DevParams P, SweepArgs a) {
    using R = typename std::conditional<MIX, float, double>::type;
    extern __shared__ double carry_lds[];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    double *carry = carry_lds + (size_t)wave * a.nslots * kWave + lane;   // slot j at carry[j*64]
    const int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = col < a.ncol;
    const double dt = a.dt;
    const double inv_dt = 1.0 / dt;
    const int ncat = P.warm ? 1 : 4;
    const bool do_adj = P.stages & CASIM_STAGE_ADJUST, do_sat = P.stages & CASIM_STAGE_SATADJ;
    const bool do_rates = P.stages & CASIM_STAGE_RATES, do_sed = P.stages & CASIM_STAGE_SED;

    for (int j = 0; j < a.nslots; ++j) carry[j * kWave] = 0.0;
    bool inflow = false;            // a flux from the level above is non-zero
    double psurf[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) psurf[j] = 0.0;
    unsigned newton_bad = 0, nonfinite = 0;

    for (int k = a.nlev - 1; k >= 0; --k) {
        const int64_t ix = (int64_t)k * a.ld + col;
        Pt w{}, d{};
        double p = 1.0, rho = 1.0;
        bool act = false;
        if (valid) {
            w.T = a.in[0][ix]; p = a.in[1][ix]; w.qv = a.in[3][ix];
            w.qc = a.in[4][ix]; w.qr = a.in[6][ix]; w.qi = a.in[8][ix];
            w.qs = a.in[10][ix]; w.qg = a.in[12][ix];
            const bool cond = (w.qc > 0.0) | (w.qr > 0.0) | (!P.warm & ((w.qi > 0.0) | (w.qs > 0.0) | (w.qg > 0.0)));
            act = cond;
            if (!cond && (do_adj || do_sat)) {
                // a condensate-free point changes only if supersaturated
                if (do_sat) act = w.qv > q_of_e(P, esat_liq(P, w.T), p);
                if (!act && do_adj && !P.warm && w.T < P.T_nuc)
                    act = w.qv > q_of_e(P, esat_ice(P, w.T), p);
            }
        }
        const unsigned long long bal = __ballot((int)(act || inflow));
        if (bal == 0ull) {
            if (valid) {
#pragma unroll
                for (int f = 0; f < CASIM_NTEND; ++f) a.tend[f][ix] = 0.0;
            }
            continue;
        }
        if (act || inflow) {
            rho = a.in[2][ix];
            w.nc = a.in[5][ix]; w.nr = a.in[7][ix]; w.ni = a.in[9][ix];
            w.ns = a.in[11][ix]; w.ng = a.in[13][ix];
        }
        const double rfac = ::sqrt(P.rho_0 / rho);
        if (act) {
            if (do_adj) adjust(P, w, d, p, rho);
            if (do_sat) newton_bad += satadj(P, w, d, p) ? 1u : 0u;
            if (do_rates) {
                R r[12];
                rates<R>(P, w, p, rho, rfac, r);
                apply_rates<R>(P, w, d, r, dt);
            }
        }
        bool out_nz = false;
        if ((act || inflow) && do_sed) {
            const double inv_rdz = 1.0 / (rho * a.dz[k]);
            const bool surf = (k == 0);
            sediment<R>(P, a, 0, carry, rho, rfac, inv_rdz, surf, w.qr, w.nr, d.qr, d.nr, psurf[0], psurf[4], out_nz);
            if (ncat > 1) {
                sediment<R>(P, a, 1, carry, rho, rfac, inv_rdz, surf, w.qi, w.ni, d.qi, d.ni, psurf[1], psurf[5], out_nz);
                sediment<R>(P, a, 2, carry, rho, rfac, inv_rdz, surf, w.qs, w.ns, d.qs, d.ns, psurf[2], psurf[6], out_nz);
                sediment<R>(P, a, 3, carry, rho, rfac, inv_rdz, surf, w.qg, w.ng, d.qg, d.ng, psurf[3], psurf[7], out_nz);
            }
        }
        inflow = out_nz;
        if (valid) {
            double o[12] = {d.T * inv_dt, d.qv * inv_dt, d.qc * inv_dt, d.nc * inv_dt,
                            d.qr * inv_dt, d.nr * inv_dt, d.qi * inv_dt, d.ni * inv_dt,
                            d.qs * inv_dt, d.ns * inv_dt, d.qg * inv_dt, d.ng * inv_dt};
            double sum = 0.0;
#pragma unroll
            for (int f = 0; f < CASIM_NTEND; ++f) { a.tend[f][ix] = o[f]; sum += ::fabs(o[f]); }
            nonfinite += ::isfinite(sum) ? 0u : 1u;
        }
    }
    if (valid) {
#pragma unroll
        for (int j = 0; j < 8; ++j) a.sfc[j][col] = psurf[j];
    }
    if (newton_bad) atomicAdd(&a.status[0], (unsigned long long)newton_bad);
    if (nonfinite) atomicAdd(&a.status[1], (unsigned long long)nonfinite);
}

// X += dt * tend for the 12 prognostic fields; q and n clipped at 0.
__global__ __launch_bounds__(256) void apply_kernel(SweepArgs a, double dt, int64_t npts_ld) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npts_ld) return;
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

hipError_t launch_sweep(const DevParams &P, const SweepArgs &a, hipStream_t stream) {
    static int wpb = 0;
    if (wpb == 0) {
        const char *e = getenv("CASIM_WAVES_PER_BLOCK");
        wpb = e ? atoi(e) : 1;
        if (wpb < 1 || wpb > 4) wpb = 1;
    }
    int w = wpb;
    size_t lds = (size_t)w * a.nslots * kWave * sizeof(double);
    while (w > 1 && lds > 65536) { --w; lds = (size_t)w * a.nslots * kWave * sizeof(double); }
    if (lds > 65536) return hipErrorInvalidValue;
    const int threads = w * kWave;
    const int64_t blocks = (a.ncol + threads - 1) / threads;
    if (P.mode == CASIM_MODE_FP32MIX)
        hipLaunchKernelGGL(sweep_kernel<true>, dim3((unsigned)blocks), dim3(threads), lds, stream, P, a);
    else
        hipLaunchKernelGGL(sweep_kernel<false>, dim3((unsigned)blocks), dim3(threads), lds, stream, P, a);
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
