// Default constants of the scheme and their derivation into the device
// parameter block.  Everything here is constexpr so that the default
// parameter set can be compiled into the kernels as immediates (no constant
// has to live in scalar registers for the whole sweep), while the same
// derivation serves constants chosen at run time.
#pragma once

#include "casim.h"

namespace casim {

constexpr double kPi = 3.14159265358979323846;

// Published values: Bolton (1980) and Buck (1981) saturation pressures;
// Khairoutdinov & Kogan (2000) warm rain; Lin et al. (1983) ice
// autoconversion and collection; Bigg (1953) rain freezing; Cooper (1986)
// nucleation; Liu & Orville (1969) and Locatelli & Hobbs (1974) fall speeds.
constexpr casim_constants default_constants() {
    casim_constants c{};
    c.mode = CASIM_MODE_FP64;
    c.stages = CASIM_STAGE_ALL;
    c.warm = 0;
    c.flags = 0;
    c.R_d = 287.04; c.R_v = 461.5; c.cp = 1005.0; c.L_v = 2.501e6; c.L_s = 2.834e6;
    c.T_0 = 273.15; c.g = 9.80665;
    c.rho_w = 1000.0; c.rho_i = 500.0; c.rho_s = 100.0; c.rho_g = 400.0; c.rho_0 = 1.225;
    c.K_a = 2.4e-2; c.Dv0 = 2.11e-5; c.Dv_exp = 1.94;
    c.esl_a = 611.2; c.esl_b = 17.67; c.esl_c = 243.5;
    c.esi_a = 611.15; c.esi_b = 22.452; c.esi_c = 272.55;
    c.auto_a = 1350.0; c.auto_qc_exp = 2.47; c.auto_nc_exp = -1.79;
    c.accr_a = 67.0; c.accr_exp = 1.15;
    c.m_r0 = 6.545e-11;
    c.m_s0 = kPi / 6.0 * 100.0 * 1e-12;      // (pi/6) rho_s (100 um)^3
    c.m_i0 = 1e-12;
    c.n_act = 1e8;
    c.iaut_a = 1e-3; c.ice_t_exp = 0.025;
    c.bigg_a = 0.66; c.bigg_b = 100.0;
    c.cooper_a = 5.0; c.cooper_b = 0.304; c.cooper_max = 5e5;
    c.N0_s = 3e6; c.N0_g = 4e6;
    c.fall_a[0] = 842.0; c.fall_b[0] = 0.8;  c.v_max[0] = 10.0; c.d_min[0] = 2e-5; c.d_max[0] = 5e-3;
    c.fall_a[1] = 700.0; c.fall_b[1] = 1.0;  c.v_max[1] = 3.0;  c.d_min[1] = 1e-6; c.d_max[1] = 1e-3;
    c.fall_a[2] = 11.72; c.fall_b[2] = 0.41; c.v_max[2] = 3.0;  c.d_min[2] = 1e-5; c.d_max[2] = 1e-2;
    c.fall_a[3] = 19.3;  c.fall_b[3] = 0.37; c.v_max[3] = 20.0; c.d_min[3] = 1e-5; c.d_max[3] = 1e-2;
    c.capacity_points = 0;
    return c;
}

constexpr casim_thresholds default_thresholds() {
    casim_thresholds t{};
    t.q_min = 1e-12;
    t.T_hom = 233.15;
    t.T_nuc = 268.15;
    t.q_i0 = 1e-4;
    t.newton_iters = 5;
    t.newton_rtol = 1e-10;
    t.sur_range_margin = 0.05;
    t.sur_maha_max = 0.0;
    t.sur_f_min = 0.5;
    return t;
}

// Gamma-function values the fall-speed and collection laws need.
struct GammaTable {
    double g4[4];   // Gamma(4 + b) for r, i, s, g
    double g1[4];   // Gamma(1 + b)
    double g3s;     // Gamma(3 + b_s)
    double g3g;     // Gamma(3 + b_g)
};

// Gamma(x) at the default exponents b = 0.8, 1, 0.41, 0.37; casim_init checks
// this table against tgamma before it selects the compiled-in parameters.
constexpr GammaTable kDefaultGamma = {
    {17.8378619818136, 24.0, 10.275404092015203, 9.730915531905126},
    {0.9313837709802428, 1.0, 0.8867646576015011, 0.8893135074291018},
    3.013314982995661,
    2.8875120272715504,
};

// Natural logarithm usable in constant expressions (argument reduction by
// powers of two, then the atanh series ln x = 2 atanh((x-1)/(x+1))).
constexpr double cx_log(double x) {
    const double ln2 = 0.69314718055994530942;
    int e = 0;
    while (x > 1.4142135623730951) { x *= 0.5; ++e; }
    while (x < 0.7071067811865476) { x *= 2.0; --e; }
    const double z = (x - 1.0) / (x + 1.0), z2 = z * z;
    double term = z, sum = 0.0;
    for (int n = 1; n < 60; n += 2) { sum += term / n; term *= z2; }
    return 2.0 * sum + e * ln2;
}

}  // namespace casim
