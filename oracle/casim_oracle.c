/*
 * casim_oracle.c -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
 *
 * Plain FP64 CPU oracle of the per-column bulk-microphysics step.  Only the
 * tests, the smoke check and the benchmark's CPU-baseline leg may use it; the
 * product path never links or calls it.  Build: gcc -O2 -fno-fast-math
 * -ffp-contract=off -fopenmp -shared -fPIC (see oracle/__init__.py).
 *
 * What the paper fixes (arXiv 2010.14823):
 *   - Sec. II: a column is processed independently of every other column;
 *     inside a column the processes include autoconversion (cloud -> rain),
 *     accretion and sedimentation, advanced in sub-timesteps; the cold
 *     configuration carries every moisture category.
 *   - Sec. III-A/B: the whole scheme (loops, conditionals and all) runs per
 *     column and writes one source term per prognostic field.
 * The paper prints no formula or constant.  Each process below therefore
 * follows a named published parametrisation (cited at the function), with
 * the operator order adjust -> saturation adjustment -> rates -> limiter ->
 * sedimentation:
 *   S1 clean-up of sub-threshold condensate, S2 instant phase changes
 *   (homogeneous freezing, melting, Cooper 1986 nucleation), S3 liquid
 *   saturation adjustment (Bolton 1980 e_s, fixed-count Newton), S4 twelve
 *   process rates (Khairoutdinov & Kogan 2000 warm rain; Lin et al. 1983 ice
 *   collection/autoconversion; Bigg 1953 rain freezing; diffusional growth
 *   and melting of exponential size distributions), S5 source limiter and
 *   forward-Euler apply with number rules, S6 flux-form upwind sedimentation
 *   with a static substep count, S7 tendencies = accumulated increment / dt.
 *
 * Every increment is accumulated in its own variable (delta) next to the
 * working state; a tendency is never formed as new - old.
 */
#include "casim_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- constants (the oracle's own copy) -------------------------------- */
#define PI        3.14159265358979323846
#define R_D       287.04       /* J kg-1 K-1 */
#define R_V       461.5
#define EPS       (R_D / R_V)
#define CP        1005.0
#define LV        2.501e6      /* J kg-1 */
#define LS        2.834e6
#define LF        (LS - LV)
#define T_0       273.15       /* K */
#define T_HOM     233.15
#define T_NUC     268.15
#define RHO_W     1000.0       /* kg m-3 */
#define RHO_I     500.0
#define RHO_S     100.0
#define RHO_G     400.0
#define RHO_0     1.225
#define K_A       2.4e-2       /* W m-1 K-1 */
#define DV0       2.11e-5      /* m2 s-1 */
#define DV_EXP    1.94
#define Q_MIN     1e-12        /* kg/kg: "present" threshold */
#define N_ACT     1e8          /* /kg: number given to new cloud */
#define M_I0      1e-12        /* kg: mass of a nucleated crystal */
#define M_R0      6.545e-11    /* kg: KK2000 new-drop mass (25 um radius) */
#define Q_I0      1e-4         /* kg/kg: ice autoconversion threshold */
#define N0_S      3e6          /* m-4 */
#define N0_G      4e6
#define BIGG_A    0.66         /* K-1 */
#define BIGG_B    100.0        /* m-3 s-1 */
#define NEWTON_RTOL 1e-10

/* categories */
enum { V = 0, C = 1, R = 2, I = 3, S = 4, G = 5 };
/* rate indices */
enum { AUTO, ACCR, REVP, DEPI, DEPS, IAUT, SACI, SACW, GACW, FRZR, SMLT, GMLT, NRATE };
/* tendency slots */
enum { TD_T, TD_QV, TD_QC, TD_NC, TD_QR, TD_NR, TD_QI, TD_NI, TD_QS, TD_NS, TD_QG, TD_NG };

/* Fall-speed law V(D) = a D^b (rho0/rho)^1/2 per sedimenting category
 * r, i, s, g: rain Liu & Orville (1969), ice (700, 1), snow and graupel
 * Locatelli & Hobbs (1974); moment-weighted speeds capped at V_MAX. */
static const double FALL_A[4] = {842.0, 700.0, 11.72, 19.3};
static const double FALL_B[4] = {0.8, 1.0, 0.41, 0.37};
static const double V_MAX[4]  = {10.0, 3.0, 3.0, 20.0};
/* mean-diameter (1/lambda) bounds per category r, i, s, g, metres */
static const double D_LO[4] = {2e-5, 1e-6, 1e-5, 1e-5};
static const double D_HI[4] = {5e-3, 1e-3, 1e-2, 1e-2};

/* ---- saturation (Bolton 1980 over liquid, Buck 1981 over ice) ---------- */
double oracle_esat_liquid(double T)
{
    double Tc = T - T_0;
    return 611.2 * exp(17.67 * Tc / (Tc + 243.5));
}

double oracle_esat_ice(double T)
{
    double Tc = T - T_0;
    return 611.15 * exp(22.452 * Tc / (Tc + 272.55));
}

static double q_from_e(double e, double p) { return EPS * e / (p - (1.0 - EPS) * e); }

double oracle_qsat_liquid(double T, double p) { return q_from_e(oracle_esat_liquid(T), p); }
double oracle_qsat_ice(double T, double p) { return q_from_e(oracle_esat_ice(T), p); }

static double clampd(double x, double lo, double hi) { return x < lo ? lo : (x > hi ? hi : x); }

/* slope of an exponential distribution: rain and ice from (q, n) with
 * spheres of density rho_x (q = pi rho_x n / lambda^3); snow and graupel from
 * a fixed intercept N0 (rho q = pi rho_x N0 / lambda^4); clamped so that the
 * mean diameter 1/lambda stays within [D_LO, D_HI]. */
static double slope_rain_ice(int cat, double q, double n)
{
    double rx = (cat == 0) ? RHO_W : RHO_I;
    double lam = cbrt(PI * rx * n / q);
    return clampd(lam, 1.0 / D_HI[cat], 1.0 / D_LO[cat]);
}

static double slope_snow_graupel(int cat, double q, double rho)
{
    double rx = (cat == 2) ? RHO_S : RHO_G;
    double n0 = (cat == 2) ? N0_S : N0_G;
    double lam = pow(PI * rx * n0 / (rho * q), 0.25);
    return clampd(lam, 1.0 / D_HI[cat], 1.0 / D_LO[cat]);
}

/* ---- per-point working state -------------------------------------------- */
typedef struct {
    double T, q[6], n[6];      /* working values X'  */
} pstate;

typedef struct {
    double T, q[6], n[6];      /* accumulated increments (Delta X) */
} pdelta;

static void addT(pstate *w, pdelta *d, double x) { w->T += x; d->T += x; }
static void addq(pstate *w, pdelta *d, int c, double x) { w->q[c] += x; d->q[c] += x; }
static void addn(pstate *w, pdelta *d, int c, double x) { w->n[c] += x; d->n[c] += x; }
/* remove everything of a moment: the working value becomes exactly zero */
static void zeroq(pstate *w, pdelta *d, int c) { d->q[c] -= w->q[c]; w->q[c] = 0.0; }
static void zeron(pstate *w, pdelta *d, int c) { d->n[c] -= w->n[c]; w->n[c] = 0.0; }

static double latent(int c) { return (c == C || c == R) ? LV : LS; }

/* S1: condensate below the presence threshold (0 < q < Q_MIN) returns to
 * vapour with its latent heat; its number is removed. */
static void s1_cleanup(pstate *w, pdelta *d, int warm)
{
    int last = warm ? R : G;
    for (int c = C; c <= last; ++c) {
        double m = w->q[c];
        if (m > 0.0 && m < Q_MIN) {
            zeroq(w, d, c);
            addq(w, d, V, m);
            zeron(w, d, c);
            addT(w, d, -latent(c) * m / CP);
        }
    }
}

/* S2: instant phase changes, in order: homogeneous freezing of cloud below
 * T_HOM, melting of ice above T_0, and Cooper (1986) ice nucleation below
 * T_NUC when supersaturated over ice, n_IN = min(5 exp(0.304 (T0 - T)), 5e5)
 * per m3, each new crystal of mass M_I0. */
static void s2_phase(pstate *w, pdelta *d, double p, double rho)
{
    if (w->T < T_HOM && w->q[C] > 0.0) {
        double m = w->q[C], nn = w->n[C];
        zeroq(w, d, C); zeron(w, d, C);
        addq(w, d, I, m); addn(w, d, I, nn);
        addT(w, d, LF * m / CP);
    }
    if (w->T > T_0 && w->q[I] > 0.0) {
        double m = w->q[I], nn = w->n[I];
        zeroq(w, d, I); zeron(w, d, I);
        addq(w, d, C, m); addn(w, d, C, nn);
        addT(w, d, -LF * m / CP);
    }
    if (w->T < T_NUC) {
        double qsi = oracle_qsat_ice(w->T, p);
        if (w->q[V] > qsi) {
            double nin = fmin(5.0 * exp(0.304 * (T_0 - w->T)), 5e5) / rho;
            if (nin > w->n[I]) {
                double dn = nin - w->n[I];
                double dq = fmin(dn * M_I0, w->q[V] - qsi);
                addn(w, d, I, dn);
                addq(w, d, V, -dq);
                addq(w, d, I, dq);
                addT(w, d, LS * dq / CP);
            }
        }
    }
}

/* S3: liquid saturation adjustment.  With q_s(T) from Bolton's e_s, solve
 * f(delta) = cp delta - Lv (qv - q_s(T + delta, p)) = 0 by a fixed number of
 * Newton steps from delta = 0, then move dq = cp delta / Lv from vapour to
 * cloud; if that would leave negative cloud, all cloud evaporates instead.
 * New cloud takes at least N_ACT drops per kg.  Returns iterations run and
 * sets *bad when the final relative residual exceeds NEWTON_RTOL. */
static int s3_satadj(pstate *w, pdelta *d, double p, int iters, int *bad)
{
    *bad = 0;
    double qsl = oracle_qsat_liquid(w->T, p);
    if (!(w->q[V] > qsl || w->q[C] > 0.0)) return 0;
    double delta = 0.0;
    for (int it = 0; it < iters; ++it) {
        double T1 = w->T + delta;
        double Tc = T1 - T_0;
        double es = oracle_esat_liquid(T1);
        double qs = q_from_e(es, p);
        double f = CP * delta - LV * (w->q[V] - qs);
        double dqdT = qs * (p / (p - (1.0 - EPS) * es)) * 17.67 * 243.5 / ((Tc + 243.5) * (Tc + 243.5));
        double fp = CP + LV * dqdT;
        delta = delta - f / fp;
    }
    {
        double qs = oracle_qsat_liquid(w->T + delta, p);
        double res = fabs(CP * delta - LV * (w->q[V] - qs)) / (LV * qs);
        if (!(res <= NEWTON_RTOL)) *bad = 1;
    }
    double dq = CP * delta / LV;
    if (w->q[C] + dq >= 0.0) {
        int newcloud = (w->q[C] == 0.0 && dq > 0.0);
        addq(w, d, C, dq);
        addq(w, d, V, -dq);
        addT(w, d, delta);
        if (newcloud) {
            double target = fmax(w->n[C], N_ACT);
            addn(w, d, C, target - w->n[C]);
        }
    } else {
        double m = w->q[C];
        addq(w, d, V, m);
        addT(w, d, -LV * m / CP);
        zeroq(w, d, C);
        zeron(w, d, C);
    }
    return iters;
}

/* S4: the twelve process rates (kg/kg/s) on the post-adjustment state.
 *   AUTO, ACCR: Khairoutdinov & Kogan (2000), N_c in cm-3.
 *   REVP: rain evaporation, 2 pi G_l (1 - S_l) n_r / lambda_r (unventilated),
 *         only where no cloud remains and S_l < 1.
 *   DEPI, DEPS: signed vapour deposition on ice and snow, 2 pi G_i (S_i - 1)
 *         times the first moment of the size distribution.
 *   IAUT: Lin et al. (1983) ice -> snow, 1e-3 exp(0.025 (T - T0)) (q_i - Q_I0).
 *   SACI, SACW, GACW: Lin et al. (1983) continuous collection by snow or
 *         graupel, (pi/4) E q_x a N0 Gamma(3+b) lambda^-(3+b) (rho0/rho)^1/2,
 *         E = exp(0.025 (T - T0)) for ice, 1 for cloud.
 *   FRZR: Bigg (1953) rain freezing via Lin et al. (1983),
 *         20 pi^2 B' N0_r (rho_w/rho) (exp(A' (T0 - T)) - 1) lambda_r^-7.
 *   SMLT, GMLT: melting, 2 pi K_a (T - T0) N0 / (rho L_f lambda^2).
 * G(T, p) = 1 / (L^2 / (K_a R_v T^2) + R_v T / (D_v e_s)),
 * D_v = DV0 (T/T0)^1.94 (1e5/p). */
void oracle_point_rates(double T, double p, double rho, const double q[6],
                        const double n[6], int32_t warm, double r[12])
{
    for (int k = 0; k < NRATE; ++k) r[k] = 0.0;
    int cP = q[C] >= Q_MIN, rP = q[R] >= Q_MIN;
    int iP = !warm && q[I] >= Q_MIN, sP = !warm && q[S] >= Q_MIN, gP = !warm && q[G] >= Q_MIN;
    int cold = !warm && T < T_0, hot = !warm && T > T_0;

    double esl = oracle_esat_liquid(T), esi = oracle_esat_ice(T);
    double qsl = q_from_e(esl, p), qsi = q_from_e(esi, p);
    double Sl = q[V] / qsl, Si = q[V] / qsi;
    double Dv = DV0 * pow(T / T_0, DV_EXP) * (1e5 / p);
    double Gl = 1.0 / (LV * LV / (K_A * R_V * T * T) + R_V * T / (Dv * esl));
    double Gi = 1.0 / (LS * LS / (K_A * R_V * T * T) + R_V * T / (Dv * esi));
    double rfac = sqrt(RHO_0 / rho);

    double lr = rP ? slope_rain_ice(0, q[R], n[R]) : 0.0;
    double li = iP ? slope_rain_ice(1, q[I], n[I]) : 0.0;
    double ls = sP ? slope_snow_graupel(2, q[S], rho) : 0.0;
    double lg = gP ? slope_snow_graupel(3, q[G], rho) : 0.0;

    if (cP && n[C] > 0.0) {
        double Nc = n[C] * rho * 1e-6;
        r[AUTO] = 1350.0 * pow(q[C], 2.47) * pow(Nc, -1.79);
    }
    if (cP && rP) r[ACCR] = 67.0 * pow(q[C] * q[R], 1.15);
    if (rP && q[C] == 0.0 && Sl < 1.0) r[REVP] = 2.0 * PI * Gl * (1.0 - Sl) * n[R] / lr;
    if (iP && cold) r[DEPI] = 2.0 * PI * Gi * (Si - 1.0) * n[I] / li;
    if (sP && cold) r[DEPS] = 2.0 * PI * Gi * (Si - 1.0) * N0_S / (rho * ls * ls);
    if (iP && cold && q[I] > Q_I0) r[IAUT] = 1e-3 * exp(0.025 * (T - T_0)) * (q[I] - Q_I0);
    if (sP && cold) {
        double bs = FALL_B[2];
        double coll = 0.25 * PI * FALL_A[2] * N0_S * tgamma(3.0 + bs) * pow(ls, -(3.0 + bs)) * rfac;
        if (iP) r[SACI] = exp(0.025 * (T - T_0)) * q[I] * coll;
        if (cP) r[SACW] = q[C] * coll;
    }
    if (gP && cold && cP) {
        double bg = FALL_B[3];
        r[GACW] = 0.25 * PI * FALL_A[3] * N0_G * tgamma(3.0 + bg) * pow(lg, -(3.0 + bg)) * rfac * q[C];
    }
    if (rP && cold) {
        double n0r = rho * n[R] * lr;
        r[FRZR] = 20.0 * PI * PI * BIGG_B * n0r * (RHO_W / rho) * (exp(BIGG_A * (T_0 - T)) - 1.0) * pow(lr, -7.0);
    }
    if (sP && hot) r[SMLT] = 2.0 * PI * K_A * (T - T_0) * N0_S / (rho * LF * ls * ls);
    if (gP && hot) r[GMLT] = 2.0 * PI * K_A * (T - T_0) * N0_G / (rho * LF * lg * lg);
}

/* S5: limiter and forward-Euler apply.  For each source category the sum of
 * its sinks R_x is capped so that at most the available mass leaves:
 * f_x = min(1, q_x / (R_x dt)); every rate is scaled by the f of the category
 * it draws from (signed deposition draws from vapour when positive, from the
 * condensate when negative).  A limited category loses exactly its mass (and
 * number).  Sinks remove number at the source's mean mass; AUTO adds rain
 * drops of mass M_R0, IAUT adds snow of mass M_S0; melting and rain freezing
 * carry number at the source's mean mass; collection and deposition add no
 * number.  Latent heat goes into T. */
static void s5_apply(pstate *w, pdelta *d, const double r_in[12], double dt)
{
    const double M_S0 = PI / 6.0 * RHO_S * 1e-12;   /* (pi/6) rho_s (100 um)^3 */
    double r[12];
    memcpy(r, r_in, sizeof r);
    double depi_v = r[DEPI] > 0.0 ? r[DEPI] : 0.0, depi_i = r[DEPI] < 0.0 ? -r[DEPI] : 0.0;
    double deps_v = r[DEPS] > 0.0 ? r[DEPS] : 0.0, deps_s = r[DEPS] < 0.0 ? -r[DEPS] : 0.0;

    /* total sink of each category */
    double Rs[6];
    Rs[V] = depi_v + deps_v;
    Rs[C] = r[AUTO] + r[ACCR] + r[SACW] + r[GACW];
    Rs[R] = r[REVP] + r[FRZR];
    Rs[I] = r[IAUT] + r[SACI] + depi_i;
    Rs[S] = r[SMLT] + deps_s;
    Rs[G] = r[GMLT];
    double f[6];
    int lim[6];
    for (int c = 0; c < 6; ++c) {
        lim[c] = Rs[c] * dt > w->q[c];
        f[c] = lim[c] ? w->q[c] / (Rs[c] * dt) : 1.0;
    }
    /* scaled rates */
    double auto_ = r[AUTO] * f[C], accr = r[ACCR] * f[C], sacw = r[SACW] * f[C], gacw = r[GACW] * f[C];
    double revp = r[REVP] * f[R], frzr = r[FRZR] * f[R];
    double iaut = r[IAUT] * f[I], saci = r[SACI] * f[I];
    double smlt = r[SMLT] * f[S], gmlt = r[GMLT] * f[G];
    depi_v *= f[V]; deps_v *= f[V]; depi_i *= f[I]; deps_s *= f[S];

    /* mean masses before the transfer */
    double mm_c = w->q[C] > 0.0 ? w->n[C] / w->q[C] : 0.0;
    double mm_r = w->q[R] > 0.0 ? w->n[R] / w->q[R] : 0.0;
    double mm_i = w->q[I] > 0.0 ? w->n[I] / w->q[I] : 0.0;
    double mm_s = w->q[S] > 0.0 ? w->n[S] / w->q[S] : 0.0;
    double mm_g = w->q[G] > 0.0 ? w->n[G] / w->q[G] : 0.0;

    double gain[6], sinkq[6];
    gain[V] = dt * (revp + depi_i + deps_s);
    gain[C] = 0.0;
    gain[R] = dt * (auto_ + accr + smlt + gmlt);
    gain[I] = dt * depi_v;
    gain[S] = dt * (deps_v + iaut + saci + sacw);
    gain[G] = dt * (gacw + frzr);
    sinkq[V] = dt * (depi_v + deps_v);
    sinkq[C] = dt * (auto_ + accr + sacw + gacw);
    sinkq[R] = dt * (revp + frzr);
    sinkq[I] = dt * (iaut + saci + depi_i);
    sinkq[S] = dt * (smlt + deps_s);
    sinkq[G] = dt * gmlt;

    double nsink[6] = {0, 0, 0, 0, 0, 0}, ngain[6] = {0, 0, 0, 0, 0, 0};
    nsink[C] = sinkq[C] * mm_c;
    nsink[R] = sinkq[R] * mm_r;
    nsink[I] = sinkq[I] * mm_i;
    nsink[S] = sinkq[S] * mm_s;
    nsink[G] = sinkq[G] * mm_g;
    ngain[R] = dt * (auto_ / M_R0 + smlt * mm_s + gmlt * mm_g);
    ngain[S] = dt * iaut / M_S0;
    ngain[G] = dt * frzr * mm_r;

    double dT = dt * ((depi_v + deps_v - depi_i - deps_s) * LS - revp * LV
                      + (sacw + gacw + frzr) * LF - (smlt + gmlt) * LF) / CP;

    for (int c = 0; c < 6; ++c) {
        if (lim[c]) {
            zeroq(w, d, c);
            if (c != V) zeron(w, d, c);
        } else {
            addq(w, d, c, -sinkq[c]);
            if (c != V) addn(w, d, c, -nsink[c]);
        }
        addq(w, d, c, gain[c]);
        if (c != V) addn(w, d, c, ngain[c]);
    }
    addT(w, d, dT);
}

/* ---- sedimentation ------------------------------------------------------- */
void oracle_nsub(const double *dz, int32_t nlev, double dt, int32_t nsub[4])
{
    double dzmin = dz[0];
    for (int k = 1; k < nlev; ++k) dzmin = fmin(dzmin, dz[k]);
    for (int c = 0; c < 4; ++c) {
        double m = ceil(V_MAX[c] * dt / dzmin);
        nsub[c] = m < 1.0 ? 1 : (int32_t)m;
    }
}

/* mass- and number-weighted fall speeds of an exponential distribution with
 * V(D) = a D^b (rho0/rho)^1/2: V_q = a Gamma(4+b) / (6 lambda^b) * rfac,
 * V_n = a Gamma(1+b) / lambda^b * rfac, each capped at V_MAX. */
static void fall_speeds(int cat, double q, double n, double rho, double *vq, double *vn)
{
    double lam = (cat <= 1) ? slope_rain_ice(cat, q, n) : slope_snow_graupel(cat, q, rho);
    double a = FALL_A[cat], b = FALL_B[cat];
    double rfac = sqrt(RHO_0 / rho);
    double lb = pow(lam, b);
    *vq = fmin(a * tgamma(4.0 + b) / (6.0 * lb) * rfac, V_MAX[cat]);
    *vn = fmin(a * tgamma(1.0 + b) / lb * rfac, V_MAX[cat]);
}

/* S6: explicit flux-form upwind sedimentation of category cat (both moments)
 * through one column.  Each of nsub substeps of dt_s = dt/nsub: the downward
 * flux through the bottom face of level k is F_k = rho_k q_k V_k (zero through
 * the model top), q_k += dt_s (F_{k+1} - F_k) / (rho_k dz_k), and the surface
 * receives F_0 dt_s.  Speeds are recomputed each substep. */
static void s6_sediment(int cat, int nlev, int nsub, double dt, const double *rho,
                        const double *dz, double *q, double *n, double *dq, double *dn,
                        double *psurf, double *nsurf, double *Fq, double *Fn)
{
    double dts = dt / nsub;
    for (int s = 0; s < nsub; ++s) {
        for (int k = 0; k < nlev; ++k) {
            if (q[k] >= Q_MIN) {
                double vq, vn;
                fall_speeds(cat, q[k], n[k], rho[k], &vq, &vn);
                Fq[k] = rho[k] * q[k] * vq;
                Fn[k] = rho[k] * n[k] * vn;
            } else {
                Fq[k] = 0.0;
                Fn[k] = 0.0;
            }
        }
        for (int k = 0; k < nlev; ++k) {
            double fin_q = (k + 1 < nlev) ? Fq[k + 1] : 0.0;
            double fin_n = (k + 1 < nlev) ? Fn[k + 1] : 0.0;
            double incq = dts * (fin_q - Fq[k]) / (rho[k] * dz[k]);
            double incn = dts * (fin_n - Fn[k]) / (rho[k] * dz[k]);
            q[k] += incq; dq[k] += incq;
            n[k] += incn; dn[k] += incn;
        }
        *psurf += Fq[0] * dts;
        *nsurf += Fn[0] * dts;
    }
}

/* ---- driver ------------------------------------------------------------- */
void oracle_default_opts(oracle_opts *o)
{
    o->stages = ORACLE_ST_ALL;
    o->newton_iters = 5;
    o->nthreads = 0;
    o->warm = 0;
}

int oracle_saturation_adjust(double *T, double p, double *qv, double *qc, double *nc, int32_t iters)
{
    pstate w; pdelta d;
    memset(&w, 0, sizeof w); memset(&d, 0, sizeof d);
    w.T = *T; w.q[V] = *qv; w.q[C] = *qc; w.n[C] = *nc;
    int bad;
    int r = s3_satadj(&w, &d, p, iters, &bad);
    *T = w.T; *qv = w.q[V]; *qc = w.q[C]; *nc = w.n[C];
    return r;
}

/* S1-S3 on one point given its 14 input values (T, p, rho, qv, qc, nc, qr,
 * nr, qi, ni, qs, ns, qg, ng); returns the adjusted state (T, qv, qc, nc, qr,
 * nr, qi, ni, qs, ns, qg, ng) and the 12 rates S4 evaluates on it. */
void oracle_point_process(const double in14[14], int32_t warm, int32_t newton_iters,
                          double state12[12], double rates[12])
{
    pstate w; pdelta d;
    memset(&w, 0, sizeof w); memset(&d, 0, sizeof d);
    double p = in14[1], rho = in14[2];
    w.T = in14[0];
    w.q[V] = in14[3];
    w.q[C] = in14[4]; w.n[C] = in14[5];
    w.q[R] = in14[6]; w.n[R] = in14[7];
    w.q[I] = in14[8]; w.n[I] = in14[9];
    w.q[S] = in14[10]; w.n[S] = in14[11];
    w.q[G] = in14[12]; w.n[G] = in14[13];
    s1_cleanup(&w, &d, warm);
    if (!warm) s2_phase(&w, &d, p, rho);
    int bad;
    s3_satadj(&w, &d, p, newton_iters, &bad);
    state12[0] = w.T; state12[1] = w.q[V];
    state12[2] = w.q[C]; state12[3] = w.n[C];
    state12[4] = w.q[R]; state12[5] = w.n[R];
    state12[6] = w.q[I]; state12[7] = w.n[I];
    state12[8] = w.q[S]; state12[9] = w.n[S];
    state12[10] = w.q[G]; state12[11] = w.n[G];
    oracle_point_rates(w.T, p, rho, w.q, w.n, warm, rates);
}

/* S1-S3 on one point, then S5 with the supplied 12 rates in place of the
 * S4 rates (how a learned surrogate's rates enter the step); tend12 receives
 * the point's 12 tendencies (increment / dt) in the tendency order. */
void oracle_point_apply(const double in14[14], const double rates[12], double dt, int32_t warm,
                        int32_t newton_iters, double tend12[12])
{
    pstate w; pdelta d;
    memset(&w, 0, sizeof w); memset(&d, 0, sizeof d);
    double p = in14[1], rho = in14[2];
    w.T = in14[0];
    w.q[V] = in14[3];
    w.q[C] = in14[4]; w.n[C] = in14[5];
    w.q[R] = in14[6]; w.n[R] = in14[7];
    w.q[I] = in14[8]; w.n[I] = in14[9];
    w.q[S] = in14[10]; w.n[S] = in14[11];
    w.q[G] = in14[12]; w.n[G] = in14[13];
    s1_cleanup(&w, &d, warm);
    if (!warm) s2_phase(&w, &d, p, rho);
    int bad;
    s3_satadj(&w, &d, p, newton_iters, &bad);
    s5_apply(&w, &d, rates, dt);
    tend12[0] = d.T / dt; tend12[1] = d.q[V] / dt;
    tend12[2] = d.q[C] / dt; tend12[3] = d.n[C] / dt;
    tend12[4] = d.q[R] / dt; tend12[5] = d.n[R] / dt;
    tend12[6] = d.q[I] / dt; tend12[7] = d.n[I] / dt;
    tend12[8] = d.q[S] / dt; tend12[9] = d.n[S] / dt;
    tend12[10] = d.q[G] / dt; tend12[11] = d.n[G] / dt;
}

/* column c: S1-S5 at every level (pointwise), then S6 over the column. */
static int64_t column(const double *const in[14], const double *dz, int64_t col, int64_t ld,
                      int nlev, double dt, double *const tend[12], double *const sfc[8],
                      const oracle_opts *o, const int32_t nsub[4], double *work)
{
    int64_t fails = 0;
    /* per-level copies of the state after S5, and the accumulated increments */
    double *rho = work, *qs8 = work + nlev, *ns8 = qs8 + 4 * nlev;
    double *dq8 = ns8 + 4 * nlev, *dn8 = dq8 + 4 * nlev, *Fq = dn8 + 4 * nlev, *Fn = Fq + nlev;
    static const int sedcat[4] = {R, I, S, G};

    for (int k = nlev - 1; k >= 0; --k) {
        int64_t ix = (int64_t)k * ld + col;
        double p = in[1][ix];
        rho[k] = in[2][ix];
        pstate w; pdelta d;
        memset(&d, 0, sizeof d);
        w.T = in[0][ix];
        w.q[V] = in[3][ix];
        w.q[C] = in[4][ix]; w.n[C] = in[5][ix];
        w.q[R] = in[6][ix]; w.n[R] = in[7][ix];
        w.q[I] = in[8][ix]; w.n[I] = in[9][ix];
        w.q[S] = in[10][ix]; w.n[S] = in[11][ix];
        w.q[G] = in[12][ix]; w.n[G] = in[13][ix];
        w.n[V] = 0.0;

        if (o->stages & ORACLE_ST_ADJUST) {
            s1_cleanup(&w, &d, o->warm);
            if (!o->warm) s2_phase(&w, &d, p, rho[k]);
        }
        if (o->stages & ORACLE_ST_SATADJ) {
            int bad;
            s3_satadj(&w, &d, p, o->newton_iters, &bad);
            fails += bad;
        }
        if (o->stages & ORACLE_ST_RATES) {
            double r[12];
            oracle_point_rates(w.T, p, rho[k], w.q, w.n, o->warm, r);
            s5_apply(&w, &d, r, dt);
        }
        tend[TD_T][ix] = d.T / dt;
        tend[TD_QV][ix] = d.q[V] / dt;
        tend[TD_QC][ix] = d.q[C] / dt;
        tend[TD_NC][ix] = d.n[C] / dt;
        for (int j = 0; j < 4; ++j) {
            qs8[j * nlev + k] = w.q[sedcat[j]];
            ns8[j * nlev + k] = w.n[sedcat[j]];
            dq8[j * nlev + k] = d.q[sedcat[j]];
            dn8[j * nlev + k] = d.n[sedcat[j]];
        }
    }
    double ps[4] = {0, 0, 0, 0}, nsf[4] = {0, 0, 0, 0};
    if (o->stages & ORACLE_ST_SED) {
        int ncat = o->warm ? 1 : 4;
        for (int j = 0; j < ncat; ++j)
            s6_sediment(j, nlev, nsub[j], dt, rho, dz, qs8 + j * nlev, ns8 + j * nlev,
                        dq8 + j * nlev, dn8 + j * nlev, &ps[j], &nsf[j], Fq, Fn);
    }
    for (int k = 0; k < nlev; ++k) {
        int64_t ix = (int64_t)k * ld + col;
        for (int j = 0; j < 4; ++j) {
            tend[TD_QR + 2 * j][ix] = dq8[j * nlev + k] / dt;
            tend[TD_NR + 2 * j][ix] = dn8[j * nlev + k] / dt;
        }
    }
    for (int j = 0; j < 4; ++j) {
        sfc[j][col] = ps[j];
        sfc[4 + j][col] = nsf[j];
    }
    return fails;
}

int oracle_step(const double *const in[14], const double *dz, int64_t ncol, int64_t ld,
                int32_t nlev, double dt, double *const tend[12], double *const sfc[8],
                const oracle_opts *o, int64_t *newton_fail)
{
    oracle_opts def;
    if (!o) { oracle_default_opts(&def); o = &def; }
    if (ncol < 0 || nlev <= 0 || ld < ncol || !(dt > 0.0) || !dz) return -1;
    for (int f = 0; f < 14; ++f) if (!in[f]) return -1;
    for (int f = 0; f < 12; ++f) if (!tend[f]) return -1;
    for (int f = 0; f < 8; ++f) if (!sfc[f]) return -1;
    int32_t nsub[4];
    oracle_nsub(dz, nlev, dt, nsub);
    int64_t fails = 0;
    int nth = o->nthreads;
#ifdef _OPENMP
    if (nth <= 0) nth = omp_get_max_threads();
#else
    nth = 1;
#endif
    #pragma omp parallel num_threads(nth) reduction(+:fails)
    {
        double *work = (double *)malloc(sizeof(double) * (size_t)nlev * 19);
        #pragma omp for schedule(guided)
        for (int64_t c = 0; c < ncol; ++c)
            fails += column(in, dz, c, ld, nlev, dt, tend, sfc, o, nsub, work);
        free(work);
    }
    if (newton_fail) *newton_fail = fails;
    return 0;
}
