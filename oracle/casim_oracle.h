/*
 * casim_oracle.h -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
 *
 * Plain, slow, FP64 CPU definition of the per-column bulk-microphysics step
 * (saturation adjustment, warm-rain and ice process rates, sedimentation) of
 * the CASIM port study (arXiv 2010.14823, Sec. II: columns are independent,
 * processes run in sub-timesteps; Sec. III-B: the scheme writes a source term
 * per prognostic field).  The paper prints no process formulas; this oracle
 * follows the named published parametrisations listed in casim_oracle.c.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this library.  It shares no code, header or table with the GPU path.
 *
 * Array contract (same as the product's step): every field is float64,
 * laid out [k][ld] with the column index fastest, k = 0 at the surface.
 *   in[14]  : T, p, rho, qv, qc, nc, qr, nr, qi, ni, qs, ns, qg, ng
 *   tend[12]: dT, dqv, dqc, dnc, dqr, dnr, dqi, dni, dqs, dns, dqg, dng (per s)
 *   sfc[8]  : surface mass of r, i, s, g (kg m-2 over dt), then number of
 *             r, i, s, g (m-2 over dt), one value per column.
 */
#ifndef CASIM_ORACLE_H
#define CASIM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* stage bits of oracle_opts.stages */
#define ORACLE_ST_ADJUST 1   /* clean-up and instant phase changes */
#define ORACLE_ST_SATADJ 2   /* liquid saturation adjustment      */
#define ORACLE_ST_RATES  4   /* 12 process rates, limiter, apply   */
#define ORACLE_ST_SED    8   /* sedimentation                      */
#define ORACLE_ST_ALL    15

typedef struct oracle_opts {
    int32_t stages;        /* ORACLE_ST_* bits                         */
    int32_t newton_iters;  /* saturation-adjustment Newton iterations  */
    int32_t nthreads;      /* OpenMP threads over columns (<=0: default) */
    int32_t warm;          /* 1: warm configuration, ice processes off  */
} oracle_opts;

/* Default options: all stages, 5 Newton iterations, cold configuration. */
void oracle_default_opts(oracle_opts *o);

/* One step over ncol columns.  Returns 0, or -1 on bad arguments.
 * newton_fail (may be NULL) receives the number of adjusted points whose
 * final relative residual exceeded 1e-10. */
int oracle_step(const double *const in[14], const double *dz, int64_t ncol,
                int64_t ld, int32_t nlev, double dt,
                double *const tend[12], double *const sfc[8],
                const oracle_opts *o, int64_t *newton_fail);

/* Point-level pieces, exported for the closed-form pins. */
double oracle_esat_liquid(double T);
double oracle_esat_ice(double T);
double oracle_qsat_liquid(double T, double p);
double oracle_qsat_ice(double T, double p);

/* The 12 rates (kg/kg/s), order AUTO ACCR REVP DEPI DEPS IAUT SACI SACW GACW
 * FRZR SMLT GMLT, for one point state (q[6] = v c r i s g, n[6] with n[0]
 * unused). */
void oracle_point_rates(double T, double p, double rho, const double q[6],
                        const double n[6], int32_t warm, double rates[12]);

/* Saturation adjustment of one point: in/out T, qv, qc, nc. Returns the
 * number of Newton iterations run (0 if the point was not adjusted). */
int oracle_saturation_adjust(double *T, double p, double *qv, double *qc,
                             double *nc, int32_t newton_iters);

/* Clean-up, phase changes and saturation adjustment of one point (14 input
 * values in the field order above); returns the adjusted state (T, qv, qc,
 * nc, qr, nr, qi, ni, qs, ns, qg, ng) and the 12 rates on it. */
void oracle_point_process(const double in14[14], int32_t warm, int32_t newton_iters,
                          double state12[12], double rates[12]);

/* Clean-up, phase changes and saturation adjustment of one point, then the
 * limiter and apply step with the supplied 12 rates (a surrogate's rates)
 * instead of the point's own; tend12 receives its 12 tendencies. */
void oracle_point_apply(const double in14[14], const double rates[12], double dt, int32_t warm,
                        int32_t newton_iters, double tend12[12]);

/* Number of sedimentation substeps per category r, i, s, g. */
void oracle_nsub(const double *dz, int32_t nlev, double dt, int32_t nsub[4]);

#ifdef __cplusplus
}
#endif
#endif
