// Internal declarations shared by the host ABI and the device kernels of
// libcasim.  Not part of the public interface (include/casim.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "casim.h"

namespace casim {

constexpr int kWave = 64;            // CDNA wavefront width: one column per lane
constexpr int kMaxCarrySlots = 64;   // 2 moments x sum of substeps over r,i,s,g

// Device copy of the scheme's constants, with every derived quantity the
// kernels need folded in at initialisation (no Gamma function or division of
// constants in the sweep).  Passed by value as a kernel argument.
struct DevParams {
    int32_t mode, stages, warm, newton_iters;
    double eps, one_m_eps, cp, inv_cp, L_v, L_s, L_f, R_v, T_0, T_hom, T_nuc;
    double rho_0, K_a, Dv0, Dv_exp;
    double esl_a, esl_b, esl_c, esl_bc;   // bc = b*c, slope numerator of the Newton derivative
    double esi_a, esi_b, esi_c;
    double auto_a, auto_qc_exp, auto_nc_exp, accr_a, accr_exp;
    double inv_m_r0, inv_m_s0, m_i0, n_act;
    double iaut_a, ice_t_exp, q_i0;
    double bigg_a, frzr_coef;             // frzr_coef = 20 pi^2 B' rho_w
    double cooper_a, cooper_b, cooper_max;
    double N0_s, N0_g;
    double coll_s, coll_g;                // (pi/4) a N0 Gamma(3+b) for snow, graupel
    double lam_coef[4];                   // pi rho_w, pi rho_i, pi rho_s N0_s, pi rho_g N0_g
    double lam_lo[4], lam_hi[4];          // 1/d_max, 1/d_min
    double fall_b[4], vq_coef[4], vn_coef[4], v_max[4];  // a Gamma(4+b)/6, a Gamma(1+b)
    double q_min, newton_rtol;
};

struct SweepArgs {
    const double *in[CASIM_NIN];
    double *tend[CASIM_NTEND];
    double *sfc[CASIM_NSFC];
    const double *dz;          // device, nlev
    int64_t ld, ncol;
    int32_t nlev, nsub[4], slot0[4], nslots;
    double dt;
    unsigned long long *status;   // device counters: newton_fail, nonfinite, fallback, inferred
};

// Launchers (casim_sweep.hip).  Return a hipError_t from the launch.
hipError_t launch_sweep(const DevParams &P, const SweepArgs &a, hipStream_t stream);
hipError_t launch_apply(const SweepArgs &a, double dt, hipStream_t stream);

}  // namespace casim
