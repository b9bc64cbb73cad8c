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
    bool fast = false;                      // defaults compiled into the kernels
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

GammaTable gamma_table(const casim_constants &c) {
    GammaTable gm{};
    for (int j = 0; j < 4; ++j) {
        gm.g4[j] = tgamma(4.0 + c.fall_b[j]);
        gm.g1[j] = tgamma(1.0 + c.fall_b[j]);
    }
    gm.g3s = tgamma(3.0 + c.fall_b[2]);
    gm.g3g = tgamma(3.0 + c.fall_b[3]);
    return gm;
}

bool close_rel(double a, double b) { return fabs(a - b) <= 1e-14 * fabs(b); }

// The compiled-in parameters serve a constant set equal to the defaults in
// every physical value (mode, stages, warm, flags, capacity and the Newton
// count stay run-time choices).
bool defaults_apply(const casim_constants &c, const casim_thresholds &t) {
    if (c.flags & CASIM_FLAG_GENERIC) return false;
    casim_constants cc = c;
    const casim_constants dc = default_constants();
    cc.mode = dc.mode; cc.stages = dc.stages; cc.warm = dc.warm; cc.flags = dc.flags;
    cc.capacity_points = dc.capacity_points;
    if (memcmp(&cc, &dc, sizeof cc) != 0) return false;
    const casim_thresholds dt = default_thresholds();
    if (t.q_min != dt.q_min || t.T_hom != dt.T_hom || t.T_nuc != dt.T_nuc || t.q_i0 != dt.q_i0 ||
        t.newton_rtol != dt.newton_rtol)
        return false;
    const GammaTable gm = gamma_table(dc);
    for (int j = 0; j < 4; ++j)
        if (!close_rel(kDefaultGamma.g4[j], gm.g4[j]) || !close_rel(kDefaultGamma.g1[j], gm.g1[j]))
            return false;
    return close_rel(kDefaultGamma.g3s, gm.g3s) && close_rel(kDefaultGamma.g3g, gm.g3g);
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
    a.stages = g.c.stages;
    a.warm = g.c.warm ? 1 : 0;
    a.newton_iters = g.t.newton_iters;
    a.mode = g.c.mode;
    return CASIM_OK;
}

}  // namespace

extern "C" {

int casim_default_constants(casim_constants *c) {
    if (!c) return CASIM_EINVAL;
    *c = default_constants();
    return CASIM_OK;
}

int casim_default_thresholds(casim_thresholds *t) {
    if (!t) return CASIM_EINVAL;
    *t = default_thresholds();
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
    g.P = derive(*c, *t, gamma_table(*c));
    g.fast = defaults_apply(*c, *t);
    g.init = true;
    return CASIM_OK;
}

int casim_nsub(const double *dz_host, int32_t nlev, double dt, int32_t nsub_out[4]) {
    if (!dz_host || !nsub_out || nlev < 1 || nlev > CASIM_MAX_NLEV || !isfinite(dt) || !(dt > 0))
        return CASIM_EINVAL;
    for (int k = 0; k < nlev; ++k)
        if (!pos_finite(dz_host[k])) return CASIM_EINVAL;
    const casim_constants c = g.init ? g.c : default_constants();
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
    if (g.c.mode == CASIM_MODE_SURROGATE) return CASIM_ENOSURROGATE;
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
    HIP_TRY(launch_sweep(g.P, g.fast, a, (hipStream_t)stream));
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

int casim_debug_math(const double *x, int64_t n, double *exp_out, double *log_out, void *stream) {
    if (!x || n < 0) return CASIM_EINVAL;
    if (n == 0) return CASIM_OK;
    HIP_TRY(launch_math(x, n, exp_out, log_out, (hipStream_t)stream));
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
