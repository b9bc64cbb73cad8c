// Internal declarations shared by the host ABI and the device kernels of
// libcasim.  Not part of the public interface (include/casim.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "casim.h"
#include "casim_defaults.h"

namespace casim {

constexpr int kWave = 64;            // CDNA wavefront width
// SweepArgs.mode of the streaming-floor diagnostic (no public mode value)
constexpr int kModeStream = 100;
constexpr int kMaxCarrySlots = 64;   // 2 moments x sum of substeps over r,i,s,g

// The scheme's constants with every derived quantity folded in, so the
// sweep evaluates no Gamma function, logarithm of a constant or division of
// constants.  Built by derive(); for the default constants it is a compile
// time constant of the specialised kernels.
struct DevParams {
    double eps, one_m_eps, cp, inv_cp, L_v, L_s, L_f, R_v, T_0, T_hom, T_nuc;
    double rho_0, K_a, Dv0, Dv_exp;
    double esl_a, esl_b, esl_c, esl_bc;   // bc = b*c: slope numerator of the Newton derivative
    double esi_a, esi_b, esi_c;
    double auto_a, auto_qc_exp, auto_nc_exp, accr_a, accr_exp;
    double inv_m_r0, inv_m_s0, m_i0, n_act;
    double iaut_a, ice_t_exp, q_i0;
    double bigg_a, frzr_coef;             // frzr_coef = 20 pi^2 B' rho_w
    double cooper_a, cooper_b, cooper_max;
    double N0_s, N0_g;
    double coll_s, coll_g;                // (pi/4) a N0 Gamma(3+b) for snow, graupel
    double coll_exp_s, coll_exp_g;        // -(3 + b)
    double ln_lam_coef[4];                // ln(pi rho_w), ln(pi rho_i), ln(pi rho_s N0_s), ln(pi rho_g N0_g)
    double ln_lam_lo[4], ln_lam_hi[4];    // ln(1/d_max), ln(1/d_min)
    double fall_b[4], vq_coef[4], vn_coef[4], v_max[4];  // a Gamma(4+b)/6, a Gamma(1+b)
    double q_min, newton_rtol;
    double ln_1e6;                        // ln(1e-6): kg-1 -> cm-3 factor in log space
    double two_pi;
};

constexpr DevParams derive(const casim_constants &c, const casim_thresholds &t, const GammaTable &gm) {
    DevParams P{};
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
    P.frzr_coef = 20.0 * kPi * kPi * c.bigg_b * c.rho_w;
    P.cooper_a = c.cooper_a; P.cooper_b = c.cooper_b; P.cooper_max = c.cooper_max;
    P.N0_s = c.N0_s;
    P.N0_g = c.N0_g;
    P.coll_s = 0.25 * kPi * c.fall_a[2] * c.N0_s * gm.g3s;
    P.coll_g = 0.25 * kPi * c.fall_a[3] * c.N0_g * gm.g3g;
    P.coll_exp_s = -(3.0 + c.fall_b[2]);
    P.coll_exp_g = -(3.0 + c.fall_b[3]);
    P.ln_lam_coef[0] = cx_log(kPi * c.rho_w);
    P.ln_lam_coef[1] = cx_log(kPi * c.rho_i);
    P.ln_lam_coef[2] = cx_log(kPi * c.rho_s * c.N0_s);
    P.ln_lam_coef[3] = cx_log(kPi * c.rho_g * c.N0_g);
    for (int j = 0; j < 4; ++j) {
        P.ln_lam_lo[j] = -cx_log(c.d_max[j]);
        P.ln_lam_hi[j] = -cx_log(c.d_min[j]);
        P.fall_b[j] = c.fall_b[j];
        P.vq_coef[j] = c.fall_a[j] * gm.g4[j] / 6.0;
        P.vn_coef[j] = c.fall_a[j] * gm.g1[j];
        P.v_max[j] = c.v_max[j];
    }
    P.q_min = t.q_min;
    P.newton_rtol = t.newton_rtol;
    P.ln_1e6 = cx_log(1e-6);
    P.two_pi = 2.0 * kPi;
    return P;
}

// Parameters of the default constant set, as a compile-time constant.
constexpr DevParams kDefaultParams = derive(default_constants(), default_thresholds(), kDefaultGamma);

struct SweepArgs {
    const double *in[CASIM_NIN];
    double *tend[CASIM_NTEND];
    double *sfc[CASIM_NSFC];
    const double *dz;          // device, nlev
    int64_t ld, ncol;
    int32_t nlev, nsub[4], slot0[4], nslots;
    int32_t stages, warm, newton_iters, mode;
    double dt;
    double dts[4];             // dt / nsub per category
    unsigned long long *status;   // device counters: newton_fail, nonfinite, fallback, inferred
    // surrogate mode: slot of each point (-1: none), network rates and fallback flags per slot
    const int32_t *sur_idx;
    const float *sur_rates;
    const uint8_t *sur_fallback;
    double sur_f_min;
    // compacted binary64 mode: rates[j * cmp_ld + slot] from the dense rate kernel
    const double *cmp_rates;
    int64_t cmp_ld;
    // tiles (C columns each): launch order (null: wavefront w takes tile w)
    // and, per tile, whether any chunk was busy (written for the next step)
    const int32_t *order;
    int32_t *tile_busy;
    int64_t ntiles;
    int32_t nxcd, xcd_group;   // block renumbering, see virtual_block (nxcd 1: none)
};

// The hardware deals the blocks of a launch to the XCDs round-robin (block b
// to XCD b mod nx), each XCD with its own L2.  The sweep renumbers them so
// that each XCD runs groups of G consecutive virtual blocks: virtual blocks
// [G (nx j + x), G (nx j + x) + G) are the j-th group of XCD x, in its
// dispatch order.  Neighbouring tiles, whose rows share DRAM pages, then
// stream through one L2 at about the same time, while the groups of the
// XCDs alternate across the domain, so clustered cloud still spreads evenly
// over the XCDs.  Blocks past the last whole round of groups keep their
// number.  The renumbering is a bijection of [0, nb) for any nx, G >= 1.
struct XcdMap {
    uint32_t nb, nx, G, nbf;       // nbf: blocks in whole rounds of groups
};
__host__ __device__ inline XcdMap xcd_map(uint32_t nb, uint32_t nx, uint32_t G) {
    return XcdMap{nb, nx, G, nx * G > 0 ? nb / (nx * G) * (nx * G) : 0u};
}
__host__ __device__ inline uint32_t virtual_block(uint32_t b, const XcdMap &m) {
    if (m.nx <= 1 || b >= m.nbf) return b;
    const uint32_t x = b % m.nx, i = b / m.nx;
    return m.G * (m.nx * (i / m.G) + x) + i % m.G;
}
// Blocks XCD x runs, and the virtual block of the i-th of them.
__host__ __device__ inline uint32_t xcd_blocks(uint32_t x, const XcdMap &m) {
    const uint32_t full = m.nbf / m.nx, rest = m.nb - m.nbf;
    return full + (rest > x ? (rest - x + m.nx - 1) / m.nx : 0u);
}
__host__ __device__ inline uint32_t xcd_block(uint32_t x, uint32_t i, const XcdMap &m) {
    const uint32_t full = m.nbf / m.nx;
    if (i < full) return m.G * (m.nx * (i / m.G) + x) + i % m.G;
    return m.nbf + x + m.nx * (i - full);
}
constexpr int kXcds = 8;
constexpr int kXcdGroupMin = 16, kXcdGroupMax = 64;   // blocks per group (16: 256 columns, any tile width)

// Launch shape of the sweep: C columns per wavefront tile, wpb wavefronts
// per block, `blocks` blocks, `lds` bytes of LDS per block.
struct SweepGeometry {
    int C, wpb;
    int64_t tiles, blocks;
    size_t lds;
};

// Point-parallel passes over (k, column) in point order p = k*ncol + c.
struct PointArgs {
    SweepArgs s;
    int mode;                      // POINT_COUNT, POINT_DUMP, POINT_SURR
    uint64_t seed;
    double keep;
    int64_t max_out;
    int64_t *block_counts;         // one per 256-point block
    const int64_t *block_offsets;
    float *feat, *rates;
    uint16_t *gates;
    int32_t *idx_map;              // surrogate / compacted: slot per point
    unsigned long long *counter;   // surrogate / compacted: slot counters, see kSlotRegions
    int64_t rcap;                  // slots per region
    double *cstate;                // compacted: post-adjustment state [13][cmp_ld]
};

// Slot space of the surrogate and compacted steps: point-pass block b takes
// its slots from region b % kSlotRegions, whose counter sits alone on a
// 128-byte line at counter[r * kCounterStride].  A single counter for the
// whole grid serialises millions of wavefront atomics on one L2 line.
// Region r holds slots [r * rcap, r * rcap + count_r), with rcap =
// ceil(blocks / kSlotRegions) * 256, so no region can overflow.
constexpr int kSlotRegions = 1024;
constexpr int kCounterStride = 16;
enum { POINT_COUNT = 0, POINT_DUMP = 1, POINT_SURR = 2, POINT_CSTATE = 3 };

// Post-adjustment state of a compacted point, the inputs of the rate block:
// T, p, rho, qv, qc, nc, qr, nr, qi, ni, qs, qg and the liquid saturation
// pressure at T.
constexpr int kCmpState = 13;

// Launchers (casim_sweep.hip).  `fast` selects the kernels compiled with
// kDefaultParams.  Return the launch's hipError_t.
hipError_t launch_sweep(const DevParams &P, bool fast, const SweepArgs &a, hipStream_t stream);
// Launch shape of the sweep for ncol columns, nslots carry slots and nlev
// levels (hipErrorInvalidValue when the carries and the layer thicknesses do
// not fit the LDS).
hipError_t sweep_geometry(int64_t ncol, int32_t nslots, int32_t nlev, int mode, SweepGeometry *geo);
// Tile launch order from the previous step's per-tile activity, separately
// for the wavefront positions each XCD runs (see virtual_block): busy tiles
// and most clear ones in index order, the XCD's last `reserve` clear tiles
// in its last positions.
hipError_t launch_tile_order(const int32_t *busy, const SweepGeometry &geo, int32_t nxcd, int32_t group,
                             int64_t reserve, int32_t *order, hipStream_t stream);
hipError_t launch_apply(const SweepArgs &a, double dt, hipStream_t stream);
hipError_t launch_math(const double *x, int64_t n, double *e, double *l, hipStream_t stream);
hipError_t launch_points(const DevParams &P, bool fast, const PointArgs &pa, hipStream_t stream);
// Rates of the filled slots of every region of the compacted state into
// rates[12][ld] (ld = kSlotRegions * rcap).
hipError_t launch_dense_rates(const DevParams &P, bool fast, bool warm, const double *cstate, int64_t ld,
                              const unsigned long long *counters, int64_t rcap, double *rates, hipStream_t stream);
hipError_t launch_zero_u64(unsigned long long *p, int64_t n, hipStream_t stream);
hipError_t launch_scan(const int64_t *counts, int64_t n, int64_t *offsets, int64_t *total, hipStream_t stream);

}  // namespace casim
