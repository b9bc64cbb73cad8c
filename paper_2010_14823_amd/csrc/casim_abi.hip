// Host side of libcasim: the process-wide context, argument validation,
// constant upload and kernel dispatch behind the C ABI of include/casim.h.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "casim_internal.h"

using namespace casim;

namespace {

struct Context {
    bool init = false;
    int device = -1;
    casim_constants c{};
    casim_thresholds t{};
    DevParams P{};
    double *d_dz = nullptr;                 // device copy of the vertical grid
    std::vector<double> h_dz;               // what d_dz holds
    unsigned long long *d_status = nullptr; // 4 counters
    char last_hip[256] = "";
};

Context g;

int hip_fail(hipError_t e) {
    snprintf(g.last_hip, sizeof g.last_hip, "HIP error %d: %s", (int)e, hipGetErrorString(e));
    return CASIM_EHIP;
}

#define HIP_TRY(x)                                  \
    do {                                            \
        hipError_t e_ = (x);                        \
        if (e_ != hipSuccess) return hip_fail(e_);  \
    } while (0)

bool pos_finite(double x) { return isfinite(x) && x > 0.0; }

int validate_constants(const casim_constants *c, const casim_thresholds *t) {
    if (!c || !t) return CASIM_EINVAL;
    if (c->mode < CASIM_MODE_FP64 || c->mode > CASIM_MODE_SURROGATE) return CASIM_EINVAL;
    if (c->stages < 0 || c->stages > CASIM_STAGE_ALL) return CASIM_EINVAL;
    const double pos[] = {c->R_d, c->R_v, c->cp, c->L_v, c->L_s, c->T_0, c->rho_w, c->rho_i,
                          c->rho_s, c->rho_g, c->rho_0, c->K_a, c->Dv0, c->esl_a, c->esi_a,
                          c->m_r0, c->m_s0, c->m_i0, c->N0_s, c->N0_g, t->q_min};
    for (double v : pos)
        if (!pos_finite(v)) return CASIM_EINVAL;
    if (!(c->L_s > c->L_v)) return CASIM_EINVAL;
    for (int j = 0; j < 4; ++j) {
        if (!pos_finite(c->fall_a[j]) || !pos_finite(c->v_max[j]) || !pos_finite(c->d_min[j]) ||
            !(c->d_max[j] > c->d_min[j]) || !isfinite(c->fall_b[j]))
            return CASIM_EINVAL;
    }
    if (t->newton_iters < 0 || t->newton_iters > 64) return CASIM_EINVAL;
    if (c->capacity_points < 0) return CASIM_EINVAL;
    return CASIM_OK;
}

DevParams derive(const casim_constants &c, const casim_thresholds &t) {
    const double pi = 3.14159265358979323846;
    DevParams P{};
    P.mode = c.mode;
    P.stages = c.stages;
    P.warm = c.warm ? 1 : 0;
    P.newton_iters = t.newton_iters;
    P.eps = c.R_d / c.R_v;
    P.one_m_eps = 1.0 - P.eps;
    P.cp = c.cp;
    P.inv_cp = 1.0 / c.cp;
    P.L_v = c.L_v;
    P.L_s = c.L_s;
    P.L_f = c.L_s - c.L_v;
    P.R_v = c.R_v;
    P.T_0 = c.T_0;
    P.T_hom = t.T_hom;
    P.T_nuc = t.T_nuc;
    P.rho_0 = c.rho_0;
    P.K_a = c.K_a;
    P.Dv0 = c.Dv0;
    P.Dv_exp = c.Dv_exp;
    P.esl_a = c.esl_a; P.esl_b = c.esl_b; P.esl_c = c.esl_c; P.esl_bc = c.esl_b * c.esl_c;
    P.esi_a = c.esi_a; P.esi_b = c.esi_b; P.esi_c = c.esi_c;
    P.auto_a = c.auto_a; P.auto_qc_exp = c.auto_qc_exp; P.auto_nc_exp = c.auto_nc_exp;
    P.accr_a = c.accr_a; P.accr_exp = c.accr_exp;
    P.inv_m_r0 = 1.0 / c.m_r0;
    P.inv_m_s0 = 1.0 / c.m_s0;
    P.m_i0 = c.m_i0;
    P.n_act = c.n_act;
    P.iaut_a = c.iaut_a;
    P.ice_t_exp = c.ice_t_exp;
    P.q_i0 = t.q_i0;
    P.bigg_a = c.bigg_a;
    P.frzr_coef = 20.0 * pi * pi * c.bigg_b * c.rho_w;
    P.cooper_a = c.cooper_a; P.cooper_b = c.cooper_b; P.cooper_max = c.cooper_max;
    P.N0_s = c.N0_s;
    P.N0_g = c.N0_g;
    P.coll_s = 0.25 * pi * c.fall_a[2] * c.N0_s * tgamma(3.0 + c.fall_b[2]);
    P.coll_g = 0.25 * pi * c.fall_a[3] * c.N0_g * tgamma(3.0 + c.fall_b[3]);
    P.lam_coef[0] = pi * c.rho_w;
    P.lam_coef[1] = pi * c.rho_i;
    P.lam_coef[2] = pi * c.rho_s * c.N0_s;
    P.lam_coef[3] = pi * c.rho_g * c.N0_g;
    for (int j = 0; j < 4; ++j) {
        P.lam_lo[j] = 1.0 / c.d_max[j];
        P.lam_hi[j] = 1.0 / c.d_min[j];
        P.fall_b[j] = c.fall_b[j];
        P.vq_coef[j] = c.fall_a[j] * tgamma(4.0 + c.fall_b[j]) / 6.0;
        P.vn_coef[j] = c.fall_a[j] * tgamma(1.0 + c.fall_b[j]);
        P.v_max[j] = c.v_max[j];
    }
    P.q_min = t.q_min;
    P.newton_rtol = t.newton_rtol;
    return P;
}

void nsub_of(const casim_constants &c, const double *dz, int nlev, double dt, int32_t out[4]) {
    double dzmin = dz[0];
    for (int k = 1; k < nlev; ++k) dzmin = fmin(dzmin, dz[k]);
    for (int j = 0; j < 4; ++j) {
        const double m = ceil(c.v_max[j] * dt / dzmin);
        out[j] = m < 1.0 ? 1 : (int32_t)m;
    }
}

int check_state(const casim_state *s, int64_t ncol, int32_t nlev, double dt) {
    if (!g.init) return CASIM_ENOINIT;
    if (!s) return CASIM_EINVAL;
    if (ncol < 0 || nlev < 1 || nlev > CASIM_MAX_NLEV) return CASIM_EINVAL;
    if (s->ld < ncol || s->ld < 0) return CASIM_EINVAL;
    if (!isfinite(dt) || !(dt > 0.0)) return CASIM_EINVAL;
    if (ncol == 0) return CASIM_OK;
    for (int f = 0; f < CASIM_NIN; ++f)
        if (!s->in[f]) return CASIM_EINVAL;
    for (int f = 0; f < CASIM_NTEND; ++f)
        if (!s->tend[f]) return CASIM_EINVAL;
    if ((int64_t)nlev * s->ld > (int64_t)1 << 40) return CASIM_EINVAL;
    return CASIM_OK;
}

// Make d_dz hold dz[0..nlev).  The grid normally stays the same from step to
// step; on a change the device is drained before the copy so no step still in
// flight reads a half-written grid.
int upload_dz(const double *dz, int32_t nlev) {
    if ((int)g.h_dz.size() == nlev && memcmp(g.h_dz.data(), dz, sizeof(double) * nlev) == 0)
        return CASIM_OK;
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(g.d_dz, dz, sizeof(double) * nlev, hipMemcpyHostToDevice));
    g.h_dz.assign(dz, dz + nlev);
    return CASIM_OK;
}

int fill_args(const casim_state *s, int64_t ncol, int32_t nlev, double dt, SweepArgs &a) {
    for (int f = 0; f < CASIM_NIN; ++f) a.in[f] = s->in[f];
    for (int f = 0; f < CASIM_NTEND; ++f) a.tend[f] = s->tend[f];
    for (int f = 0; f < CASIM_NSFC; ++f) a.sfc[f] = s->sfc[f];
    a.dz = g.d_dz;
    a.ld = s->ld;
    a.ncol = ncol;
    a.nlev = nlev;
    a.dt = dt;
    a.status = g.d_status;
    return CASIM_OK;
}

}  // namespace

extern "C" {

int casim_default_constants(casim_constants *c) {
    if (!c) return CASIM_EINVAL;
    memset(c, 0, sizeof *c);
    c->mode = CASIM_MODE_FP64;
    c->stages = CASIM_STAGE_ALL;
    c->warm = 0;
    c->R_d = 287.04; c->R_v = 461.5; c->cp = 1005.0; c->L_v = 2.501e6; c->L_s = 2.834e6;
    c->T_0 = 273.15; c->g = 9.80665;
    c->rho_w = 1000.0; c->rho_i = 500.0; c->rho_s = 100.0; c->rho_g = 400.0; c->rho_0 = 1.225;
    c->K_a = 2.4e-2; c->Dv0 = 2.11e-5; c->Dv_exp = 1.94;
    c->esl_a = 611.2; c->esl_b = 17.67; c->esl_c = 243.5;       // Bolton (1980)
    c->esi_a = 611.15; c->esi_b = 22.452; c->esi_c = 272.55;    // Buck (1981), ice
    c->auto_a = 1350.0; c->auto_qc_exp = 2.47; c->auto_nc_exp = -1.79;   // KK2000
    c->accr_a = 67.0; c->accr_exp = 1.15;
    c->m_r0 = 6.545e-11;
    c->m_s0 = 3.14159265358979323846 / 6.0 * 100.0 * 1e-12;   // (pi/6) rho_s (100 um)^3
    c->m_i0 = 1e-12;
    c->n_act = 1e8;
    c->iaut_a = 1e-3; c->ice_t_exp = 0.025;                    // Lin et al. (1983)
    c->bigg_a = 0.66; c->bigg_b = 100.0;                       // Bigg (1953)
    c->cooper_a = 5.0; c->cooper_b = 0.304; c->cooper_max = 5e5; // Cooper (1986)
    c->N0_s = 3e6; c->N0_g = 4e6;
    const double fa[4] = {842.0, 700.0, 11.72, 19.3}, fb[4] = {0.8, 1.0, 0.41, 0.37};
    const double vm[4] = {10.0, 3.0, 3.0, 20.0};
    const double dmin[4] = {2e-5, 1e-6, 1e-5, 1e-5}, dmax[4] = {5e-3, 1e-3, 1e-2, 1e-2};
    for (int j = 0; j < 4; ++j) {
        c->fall_a[j] = fa[j]; c->fall_b[j] = fb[j]; c->v_max[j] = vm[j];
        c->d_min[j] = dmin[j]; c->d_max[j] = dmax[j];
    }
    c->capacity_points = 0;
    return CASIM_OK;
}

int casim_default_thresholds(casim_thresholds *t) {
    if (!t) return CASIM_EINVAL;
    memset(t, 0, sizeof *t);
    t->q_min = 1e-12;
    t->T_hom = 233.15;
    t->T_nuc = 268.15;
    t->q_i0 = 1e-4;
    t->newton_iters = 5;
    t->newton_rtol = 1e-10;
    t->sur_range_margin = 0.05;
    t->sur_maha_max = 0.0;
    t->sur_f_min = 0.5;
    return CASIM_OK;
}

int casim_init(const casim_constants *c, const casim_thresholds *t) {
    int rc = validate_constants(c, t);
    if (rc) return rc;
    if (g.init) HIP_TRY(hipDeviceSynchronize());
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (!g.d_dz || g.device != dev) {
        HIP_TRY(hipMalloc(&g.d_dz, sizeof(double) * CASIM_MAX_NLEV));
        HIP_TRY(hipMalloc(&g.d_status, sizeof(unsigned long long) * 4));
        HIP_TRY(hipMemset(g.d_status, 0, sizeof(unsigned long long) * 4));
        g.h_dz.clear();
        g.device = dev;
    }
    g.c = *c;
    g.t = *t;
    g.P = derive(*c, *t);
    g.init = true;
    return CASIM_OK;
}

int casim_nsub(const double *dz_host, int32_t nlev, double dt, int32_t nsub_out[4]) {
    if (!dz_host || !nsub_out || nlev < 1 || nlev > CASIM_MAX_NLEV || !isfinite(dt) || !(dt > 0))
        return CASIM_EINVAL;
    for (int k = 0; k < nlev; ++k)
        if (!pos_finite(dz_host[k])) return CASIM_EINVAL;
    casim_constants c;
    if (g.init) c = g.c; else casim_default_constants(&c);
    nsub_of(c, dz_host, nlev, dt, nsub_out);
    return CASIM_OK;
}

int casim_step(const casim_state *s, int64_t ncol, int32_t nlev, double dt, void *stream) {
    int rc = check_state(s, ncol, nlev, dt);
    if (rc) return rc;
    if (ncol == 0) return CASIM_OK;
    if (!s->dz) return CASIM_EINVAL;
    for (int f = 0; f < CASIM_NSFC; ++f)
        if (!s->sfc[f]) return CASIM_EINVAL;
    for (int k = 0; k < nlev; ++k)
        if (!pos_finite(s->dz[k])) return CASIM_EINVAL;
    if (g.P.mode == CASIM_MODE_SURROGATE) return CASIM_ENOSURROGATE;
    SweepArgs a{};
    fill_args(s, ncol, nlev, dt, a);
    nsub_of(g.c, s->dz, nlev, dt, a.nsub);
    int slot = 0;
    for (int j = 0; j < 4; ++j) {
        a.slot0[j] = slot;
        slot += 2 * a.nsub[j];
    }
    a.nslots = slot;
    if (slot > kMaxCarrySlots) return CASIM_ECAPACITY;
    rc = upload_dz(s->dz, nlev);
    if (rc) return rc;
    HIP_TRY(launch_sweep(g.P, a, (hipStream_t)stream));
    return CASIM_OK;
}

int casim_apply_tendencies(const casim_state *s, int64_t ncol, int32_t nlev, double dt, void *stream) {
    int rc = check_state(s, ncol, nlev, dt);
    if (rc) return rc;
    if (ncol == 0) return CASIM_OK;
    SweepArgs a{};
    fill_args(s, ncol, nlev, dt, a);
    HIP_TRY(launch_apply(a, dt, (hipStream_t)stream));
    return CASIM_OK;
}

int casim_status(void *stream, casim_step_status *out) {
    if (!g.init) return CASIM_ENOINIT;
    if (!out) return CASIM_EINVAL;
    unsigned long long h[4];
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    HIP_TRY(hipMemcpy(h, g.d_status, sizeof h, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemset(g.d_status, 0, sizeof h));
    out->newton_fail = (int64_t)h[0];
    out->nonfinite = (int64_t)h[1];
    out->fallback = (int64_t)h[2];
    out->inferred = (int64_t)h[3];
    return CASIM_OK;
}

int casim_finalize(void) {
    if (g.d_dz || g.d_status) hipDeviceSynchronize();
    if (g.d_dz) hipFree(g.d_dz);
    if (g.d_status) hipFree(g.d_status);
    g.d_dz = nullptr;
    g.d_status = nullptr;
    g.h_dz.clear();
    g.init = false;
    g.device = -1;
    return CASIM_OK;
}

const char *casim_strerror(int code) {
    switch (code) {
        case CASIM_OK: return "success";
        case CASIM_EINVAL: return "invalid argument";
        case CASIM_ENOINIT: return "casim_init has not been called";
        case CASIM_ECAPACITY: return "request exceeds a configured capacity";
        case CASIM_EHIP: return g.last_hip[0] ? g.last_hip : "HIP runtime error";
        case CASIM_ENOSURROGATE: return "surrogate mode without loaded weights";
        default: return "unknown error code";
    }
}

}  // extern "C"
