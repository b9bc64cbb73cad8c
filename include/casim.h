/*
 * casim.h -- C ABI of the MI355X (gfx950) bulk-microphysics column step.
 *
 * The library plays the role the CASIM port study (arXiv 2010.14823) gives the
 * microphysics: a sub-model that a parent atmospheric model calls once per
 * timestep for every grid column (Sec. I, Sec. II-A), which works on each
 * column independently (Sec. II) and returns a source term (tendency) for
 * each prognostic moisture field (Sec. III-B).  As in the paper's offload
 * (Sec. III-A, Sec. III-B), the whole scheme -- saturation adjustment, the
 * warm-rain and ice process rates with their conditionals, and sedimentation
 * in sub-timesteps -- runs on the device in one pass per step, constants are
 * copied to the device once at initialisation, and each step is ordered on a
 * caller-supplied queue (here a HIP stream).
 *
 * Conventions for every entry point:
 *  - Return value: CASIM_OK (0) or a negative CASIM_E* code; nothing throws.
 *    Arguments are validated on the host before anything is enqueued; a
 *    rejected call enqueues nothing.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Calls that take a stream return after enqueueing; their outputs are valid
 *    once the stream reaches that point.
 *  - One process-wide context (like the scheme's module globals, Sec. III-B).
 *    It is not thread-safe; at most one call may be in flight at a time.
 *  - Field layout: every 3-D field is float64 on the device, laid out
 *    [k][ld] with the column index fastest (element (k, c) at k*ld + c),
 *    k = 0 the lowest level.  The caller owns all field memory; the library
 *    never frees it and reads/writes it only inside enqueued work.
 *  - Citations: each declaration names the passage of the paper that defines
 *    what it does; "[proposal]" marks an entry point the paper does not
 *    describe (diagnostics, error text, the learned surrogate), whose form
 *    is this library's own choice.
 */
#ifndef CASIM_H
#define CASIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CASIM_ABI_VERSION 1

/* ---- error codes ------------------------------------------------------- */
#define CASIM_OK            0
#define CASIM_EINVAL       -1   /* bad argument (NULL, size, dt, ld, mode) */
#define CASIM_ENOINIT      -2   /* casim_init has not succeeded            */
#define CASIM_ECAPACITY    -3   /* request exceeds a configured capacity   */
#define CASIM_EHIP         -4   /* HIP runtime error (text: casim_strerror)*/
#define CASIM_ENOSURROGATE -5   /* surrogate mode without loaded weights   */

/* ---- modes and stage switches (casim_constants.mode / .stages) ---------- */
#define CASIM_MODE_FP64      0  /* plain path, all arithmetic in binary64  */
#define CASIM_MODE_FP32MIX   1  /* process rates and fall speeds in
                                   binary32; saturation adjustment, fluxes,
                                   level updates and surface sums binary64 */
#define CASIM_MODE_SURROGATE 2  /* process rates from the learned MLP      */
#define CASIM_MODE_FP64_COMPACT 3  /* binary64 like CASIM_MODE_FP64, with the
                                   12 rates evaluated by a separate kernel
                                   over a dense list of the points whose
                                   rate gates are open (ballot and prefix
                                   compaction; the post-adjustment state
                                   and the rates are staged through device
                                   memory).  Same results as CASIM_MODE_FP64
                                   to rounding; it trades HBM traffic for
                                   full wavefronts in the rate evaluation. */

#define CASIM_STAGE_ADJUST 1    /* clean-up + instant phase changes        */
#define CASIM_STAGE_SATADJ 2    /* liquid saturation adjustment            */
#define CASIM_STAGE_RATES  4    /* 12 process rates, limiter, apply        */
#define CASIM_STAGE_SED    8    /* sedimentation of rain, ice, snow, graupel */
#define CASIM_STAGE_ALL    15

/* casim_constants.flags: use the kernel that reads every constant at run time
 * even when the constants equal the defaults (the defaults are otherwise
 * compiled into a specialised kernel). */
#define CASIM_FLAG_GENERIC 1

#define CASIM_MAX_NLEV     512  /* largest number of levels per column     */
#define CASIM_NIN          14
#define CASIM_NTEND        12
#define CASIM_NSFC         8
#define CASIM_NRATE        12

/* Physical constants and parameters of the scheme.  casim_default_constants
 * fills the published values named beside each group; callers may change
 * them before casim_init. */
typedef struct casim_constants {
    int32_t mode;                  /* CASIM_MODE_*                          */
    int32_t stages;                /* CASIM_STAGE_* bits                    */
    int32_t warm;                  /* 1: warm configuration (no ice), Sec. II */
    int32_t flags;                 /* CASIM_FLAG_* bits                     */
    /* gas and phase change */
    double R_d, R_v, cp, L_v, L_s;               /* J kg-1 K-1, J kg-1      */
    double T_0, g;                                /* K, m s-2                */
    /* densities, kg m-3 */
    double rho_w, rho_i, rho_s, rho_g, rho_0;
    /* transport: K_a (W m-1 K-1), D_v = Dv0 (T/T_0)^Dv_exp (1e5/p)        */
    double K_a, Dv0, Dv_exp;
    /* saturation pressure a exp(b Tc/(Tc+c)): Bolton 1980 liquid, Buck 1981 ice */
    double esl_a, esl_b, esl_c, esi_a, esi_b, esi_c;
    /* Khairoutdinov & Kogan 2000: AUTO = a qc^e1 Nc^e2 (Nc cm-3), ACCR = a (qc qr)^e */
    double auto_a, auto_qc_exp, auto_nc_exp, accr_a, accr_exp;
    double m_r0;                   /* kg, mass of a new rain drop          */
    double m_s0;                   /* kg, mass of a new snow particle      */
    double m_i0;                   /* kg, mass of a nucleated crystal      */
    double n_act;                  /* kg-1, number given to new cloud      */
    /* Lin et al. 1983: IAUT = iaut_a exp(t_exp (T-T0)) (qi - q_i0); E_si = exp(t_exp (T-T0)) */
    double iaut_a, ice_t_exp;
    /* Bigg 1953 rain freezing: A' (K-1), B' (m-3 s-1) */
    double bigg_a, bigg_b;
    /* Cooper 1986 nucleation: n = min(a exp(b (T0-T)), max) per m3 */
    double cooper_a, cooper_b, cooper_max;
    /* snow and graupel intercepts, m-4 */
    double N0_s, N0_g;
    /* fall speed V(D) = a D^b (rho_0/rho)^1/2 for r, i, s, g; caps (m s-1) */
    double fall_a[4], fall_b[4], v_max[4];
    /* mean-diameter bounds 1/lambda, metres, for r, i, s, g */
    double d_min[4], d_max[4];
    int64_t capacity_points;       /* scratch sizing for compaction / surrogate */
} casim_constants;

/* Thresholds and solver controls. */
typedef struct casim_thresholds {
    double q_min;                  /* kg/kg: present if q >= q_min         */
    double T_hom;                  /* K: homogeneous freezing below        */
    double T_nuc;                  /* K: ice nucleation below              */
    double q_i0;                   /* kg/kg: ice autoconversion threshold  */
    int32_t newton_iters;          /* fixed Newton count of the adjustment */
    int32_t reserved0;
    double newton_rtol;            /* residual above which a point is flagged */
    /* learned surrogate gating */
    double sur_range_margin;       /* fraction of a feature's range added on each side */
    double sur_maha_max;           /* squared Mahalanobis distance limit (0: from training) */
    double sur_f_min;              /* limiter factor below which a point falls back */
} casim_thresholds;

/* One step's state.  All pointers except dz are device pointers.
 *   in[14]  : T (K), p (Pa), rho (kg m-3), qv, qc, nc, qr, nr, qi, ni, qs, ns,
 *             qg, ng (q in kg/kg, n in kg-1); read only.
 *   dz      : HOST pointer to nlev layer thicknesses (m), read during the
 *             call; the library keeps a device copy.
 *   ld      : leading dimension (>= ncol) of every 3-D field; columns
 *             ncol .. ld-1 of a row are never read or written.  Prefer the
 *             value casim_padded_ld recommends (a row stride that is a
 *             multiple of 4 KB is measurably slower).
 *   tend[12]: dT, dqv, dqc, dnc, dqr, dnr, dqi, dni, dqs, dns, dqg, dng, per
 *             second; written for every (k, c), c < ncol.
 *   sfc[8]  : per column, mass of r, i, s, g reaching the surface during dt
 *             (kg m-2), then their number (m-2); length >= ncol. */
typedef struct casim_state {
    const double *in[CASIM_NIN];
    const double *dz;
    int64_t ld;
    double *tend[CASIM_NTEND];
    double *sfc[CASIM_NSFC];
} casim_state;

/* Counters the step kernels raise on the device. */
typedef struct casim_step_status {
    int64_t newton_fail;    /* adjusted points with residual > newton_rtol */
    int64_t nonfinite;      /* points with a non-finite tendency          */
    int64_t fallback;       /* surrogate points that used the plain rates */
    int64_t inferred;       /* surrogate points that used the network     */
} casim_step_status;

/* [proposal] Fill *c / *t with the default published values named beside
 * each field (the paper prints no constants).  Never fails on non-NULL. */
int casim_default_constants(casim_constants *c);
int casim_default_thresholds(casim_thresholds *t);

/* Copy the constants to the device and allocate library scratch (Sec.
 * III-B: constants and globals are moved to the device once, at
 * initialisation).  May be called again to change constants or mode; it
 * synchronises the device first.  Errors: EINVAL (NULL, bad mode/stages,
 * non-positive physical constants), EHIP. */
int casim_init(const casim_constants *c, const casim_thresholds *t);

/* Enqueue one microphysics step over ncol columns of nlev levels on stream
 * (Sec. III-B: one offloaded pass over all columns writing a source term per
 * field).  Errors: ENOINIT, EINVAL (NULL pointer, ncol < 0, nlev outside
 * 1..CASIM_MAX_NLEV, ld < ncol, dt not finite or <= 0, dz not finite or
 * <= 0), ENOSURROGATE, ECAPACITY (the sedimentation substeps need more than
 * 64 carry slots: 2 x the sum of the four substep counts of casim_nsub,
 * e.g. 512 thin levels at dt = 2 s), EHIP.  All checks happen before
 * anything is enqueued.  ncol == 0 is a no-op. */
int casim_step(const casim_state *s, int64_t ncol, int32_t nlev, double dt, void *stream);

/* casim_step for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * same kernels and results as casim_step (bitwise), for modes CASIM_MODE_FP64
 * and CASIM_MODE_FP32MIX (others: EINVAL); the call itself allocates nothing.
 * Everything beyond the caller's inputs and outputs (the device copy of dz,
 * the step counters that casim_status reads, the per-tile activity record and
 * launch order) lives in one statically sized device array per GPU, set up by
 * casim_init on the GPU that is current then; a call on another GPU returns
 * ENOINIT.  Limit: at most 262,144 column tiles (4,194,304 columns at the
 * 16-column tiles of large domains; fewer on narrow tiles), else ECAPACITY.
 * All calls on one GPU share that array and it keeps the last call's
 * contents: calls whose execution overlaps on one GPU (other streams, other
 * host threads) race on it and must be ordered by the caller.  dz is a host
 * pointer, copied to the array with an asynchronous copy on `stream`: keep
 * it valid and unchanged until that copy has run (page-locked memory is read
 * when the stream reaches the copy; under graph capture the recorded copy
 * reads it again at every replay).
 * Errors: as casim_step. */
int casim_step_noalloc(const casim_state *s, int64_t ncol, int32_t nlev, double dt, void *stream);

/* Parent-model helper for multi-step runs (Sec. II-A: the parent model sums
 * the source terms its components return and integrates them into the
 * prognostic fields): X += dt * tend for the 12 prognostic fields of `s`
 * (in[] is written through a cast: it must be writable memory), q and n
 * clipped at 0.  Errors as casim_step. */
int casim_apply_tendencies(const casim_state *s, int64_t ncol, int32_t nlev, double dt, void *stream);

/* [proposal] Synchronise `stream`, copy the device counters into *out and
 * reset them (those of casim_step and of casim_step_noalloc on the current
 * GPU).  Errors: ENOINIT, EINVAL (NULL out), EHIP. */
int casim_status(void *stream, casim_step_status *out);

/* Shutdown (Sec. III-B: the finalisation routine closes the device data
 * region and releases the device memory it holds): frees library-owned
 * device memory, never caller memory.  Safe to call twice. */
int casim_finalize(void);

/* [proposal] Static text for a code; for CASIM_EHIP, the last HIP error seen. */
const char *casim_strerror(int code);

/* [proposal] Number of sedimentation substeps per category r, i, s, g that
 * casim_step uses for this grid and dt (sedimentation advances in
 * sub-timesteps, Sec. II; the static count max(1, ceil(v_max dt / min dz))
 * is this library's reading).  Host only. */
int casim_nsub(const double *dz_host, int32_t nlev, double dt, int32_t nsub_out[4]);

/* [proposal] A leading dimension for fields of ncol columns that the step
 * streams well: ncol rounded up to a multiple of 16 (with a 128-byte aligned
 * field base, every 16-column row segment a wavefront loads is then one
 * aligned 128-byte line), plus 256 when the rounded count is a multiple of
 * 512, i.e. when the row stride would be a multiple of 4 KB.  With such a
 * stride the rows of the 4 levels and 26 fields that one wavefront reads
 * together share all their low address bits; on 1024 x 1024 x 120 (row
 * stride 8 MiB) that layout made the binary64 step 7 % slower (6.53 against
 * 6.11 ms, median kernel time) and its streaming floor (casim_debug_stream)
 * 3-30 % slower, depending on where the buffers land.  Any
 * ld >= ncol stays valid; this is a recommendation for the caller's
 * allocation.  Returns the leading dimension (0 for ncol = 0), or
 * CASIM_EINVAL for ncol < 0 or ncol > 2^40.  Host only. */
int64_t casim_padded_ld(int64_t ncol);

/* ======================================================================
 * [proposal] Learned surrogate of the process-rate block (every entry point
 * of this section).  The paper has no learned component; this one replaces
 * the rate block of the scheme whose processes Sec. II lists.
 *
 * A multilayer perceptron maps a grid point's state after saturation
 * adjustment to its 12 process rates (AUTO ACCR REVP DEPI DEPS IAUT SACI SACW
 * GACW FRZR SMLT GMLT).  Features (float32, 12 per point): ln T, ln p,
 * ln rho, ln(q + 1e-12) for qv, qc, then ln(n + 1) for nc, and likewise
 * (q, n) for rain and ice, then ln(q + 1e-12) for snow and graupel (feature
 * order T, p, rho, qv, qc, nc, qr, nr, qi, ni, qs, qg).  Targets:
 * asinh(rate / 1e-12 kg kg-1 s-1), of |rate| for DEPI and DEPS (their sign is
 * the gate word's bit 12).  Gate word (uint16): bit j set when rate
 * j's condition holds (its categories present and its temperature side);
 * bit 12 set when the point is supersaturated over ice.  Closed gates are
 * exact zeros in the plain method and are masked out of training.
 *
 * Network: 12 -> 128 -> 128 -> 128 -> 12 with SiLU hidden activations on
 * standardised features and targets; parameters in one float32 vector of
 * CASIM_MLP_NPARAMS values, ordered W1 (12x128, row = input), b1, W2
 * (128x128), b2, W3, b3, W4 (128x12), b4.  Training (float32 forward,
 * backward and Adam) and inference (bfloat16 weights and activations on the
 * matrix cores, float32 accumulation) run in the library's kernels.
 * ==================================================================== */
#define CASIM_MLP_NIN     12
#define CASIM_MLP_NHID    128
#define CASIM_MLP_NOUT    12
#define CASIM_MLP_NPARAMS 36236
#define CASIM_MLP_MAX_BATCH 16384
#define CASIM_GATE_SUPERSAT_ICE (1u << 12)

/* Normalisation and trust-region statistics of a training set. */
typedef struct casim_mlp_stats {
    float x_mean[12], x_std[12];   /* features                               */
    float x_min[12], x_max[12];    /* training range of every feature        */
    float y_mean[12], y_std[12];   /* scaled targets over open gates         */
    float whiten[144];             /* W, row-major and lower-triangular (zeros
                                      above the diagonal; casim_mlp_set_stats
                                      rejects anything else with EINVAL), with
                                      W^T W = (C + 1e-9 I)^-1 for the covariance C of
                                      the standardised features (W = L^-1, L L^T the
                                      Cholesky factorisation): the squared
                                      Mahalanobis distance is |W z|^2, a sum of
                                      squares that float32 evaluates without the
                                      cancellation of z^T C^-1 z */
    float maha_q999;               /* 99.9th percentile of the squared Mahalanobis distance */
    float reserved[3];
} casim_mlp_stats;

/* Rate samples from the plain binary64 path: every point where anything can
 * happen is selected with probability keep_prob by a counter-based hash
 * (splitmix64) of (seed, point index k*ncol + c); the first max_samples
 * selected points in point order get their features, their 12 plain rates
 * (float32, kg/kg/s) and their gate word written.  *n_written (host)
 * receives the number written, *n_selected (host, may be NULL) the number
 * selected; max_samples = 0 only counts.  Synchronous.  Device buffers feat
 * and rates hold max_samples x 12 floats, gates max_samples words.  Errors as
 * casim_step, plus EINVAL for keep_prob outside (0, 1] or max_samples < 0. */
int casim_rates_dump(const casim_state *s, int64_t ncol, int32_t nlev, double dt, uint64_t seed,
                     double keep_prob, int64_t max_samples, float *feat, float *rates,
                     uint16_t *gates, int64_t *n_written, int64_t *n_selected, void *stream);

/* Compute the statistics of n training samples (device arrays as written by
 * casim_rates_dump), install them and copy them to *out (host).  Synchronous. */
int casim_mlp_fit_stats(const float *feat, const float *rates, const uint16_t *gates, int64_t n,
                        casim_mlp_stats *out, void *stream);
/* Install statistics from the host (e.g. from a checkpoint). */
int casim_mlp_set_stats(const casim_mlp_stats *st);

/* Standardised network inputs x (n x 12), targets y (n x 12) and loss mask
 * m (n x 12, 1 where the gate is open) from samples.  Needs statistics. */
int casim_mlp_prepare(const float *feat, const float *rates, const uint16_t *gates, int64_t n,
                      float *x, float *y, float *m, void *stream);

/* Initialise parameters (uniform in +-sqrt(6/(fan_in+fan_out)), drawn from a
 * counter-based hash of (seed, index)) and zero the Adam state. */
int casim_mlp_init(uint64_t seed);
/* Copy the float32 parameters to / from host memory (CASIM_MLP_NPARAMS). */
int casim_mlp_get_params(float *host_params);
int casim_mlp_set_params(const float *host_params);

/* Loss and gradient of the masked mean squared error over the batch rows
 * idx[0..batch) of (x, y, m) (idx NULL: rows 0..batch).  grad (device,
 * CASIM_MLP_NPARAMS) and loss (device, 1 float) are written; the parameters
 * are not changed.  batch in 1..CASIM_MLP_MAX_BATCH. */
int casim_mlp_grad(const float *x, const float *y, const float *m, const int32_t *idx, int32_t batch,
                   float *grad, float *loss, void *stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on that gradient; the
 * batch loss before the update goes to *loss (device, may be NULL). */
int casim_mlp_train_step(const float *x, const float *y, const float *m, const int32_t *idx,
                         int32_t batch, float lr, float *loss, void *stream);
/* float32 forward pass on n standardised inputs -> n x 12 standardised outputs. */
int casim_mlp_forward(const float *x, int64_t n, float *y, void *stream);

/* Serialise the trained state (format tag, statistics, float32 parameters,
 * Adam moments and step count) into blob; with blob NULL, *bytes receives the
 * size needed.  casim_mlp_load restores it (resuming training reproduces the
 * same parameters). */
int casim_mlp_save(void *blob, size_t *bytes);
int casim_mlp_load(const void *blob, size_t bytes);

/* Freeze the current parameters and statistics into the bfloat16 inference
 * set that CASIM_MODE_SURROGATE steps use.  Errors: ENOSURROGATE (no
 * parameters or statistics). */
int casim_surrogate_load(void);

/* Inference on n samples: rates (n x 12, kg/kg/s) from the bfloat16 network
 * with closed gates zeroed, rates kept non-negative (deposition rates keep
 * the sign of the ice supersaturation), and fallback[i] = 1 where a
 * standardised feature lies outside the standardised training range widened
 * by sur_range_margin of the range on each side, where the squared
 * Mahalanobis distance |W z|^2 exceeds the threshold (sur_maha_max, or the
 * training 99.9th percentile when that is 0), or where a rate comes out
 * non-finite.  feat (n x 12) and rates are device pointers aligned to 16
 * bytes (rows are read and written as 16-byte vectors); 0 <= n <= 2^36;
 * EINVAL otherwise. */
int casim_surrogate_infer(const float *feat, const uint16_t *gates, int64_t n, float *rates,
                          uint8_t *fallback, void *stream);

/* [proposal] The rates a CASIM_MODE_SURROGATE step would take from the network, per
 * point, through the step's own path (point pass -> slot -> network), for
 * inspection and testing: rates is a device array [12][nlev][ld] of float32
 * (kg/kg/s, gates and sign rules applied), flags a device array [nlev][ld]
 * of uint8: 0 = the network's rates (inside the trust region), 1 = outside
 * the trust region (the step uses the plain rates), 2 = no rate gate open
 * (rates 0).  The step additionally falls back where the limiter would scale
 * a category by less than sur_f_min; that test happens in the step itself.
 * Only the 14 input pointers, dz and ld of *s are used.  Works in any mode
 * of the current context.  Errors: ENOINIT, EINVAL (as casim_step),
 * ENOSURROGATE, ECAPACITY, EHIP. */
int casim_surrogate_rates(const casim_state *s, int64_t ncol, int32_t nlev, double dt, float *rates,
                          uint8_t *flags, void *stream);

/* ======================================================================
 * Host-resident state: copy in, step, copy out.
 *
 * The deployment of the scheme inside a parent model (Sec. II-A and III-B of
 * the CASIM port study): once per step the inputs are copied to the device
 * asynchronously, the parent model keeps computing its other components on
 * the CPU while the step runs, and then waits for the source terms, which
 * are copied back.  casim_step_host does this for a state held in host
 * memory.  The domain is cut into nblocks column blocks (0: 4); for each
 * block it enqueues the copy of the 14 input fields into library-owned
 * device buffers, the step on that block and the copy of its 12 tendencies
 * and 8 surface values back, on three internal streams with two buffer
 * sets, so that block b's step overlaps block b+1's inbound and block b-1's
 * outbound copies.  `stream` first orders the internal streams after its
 * own prior work and finally waits for the last outbound copy.  The call
 * returns after enqueueing; outputs are valid once `stream` has been
 * synchronised, and the inputs must not change before that.  Copies are
 * asynchronous only from page-locked memory (casim_host_alloc).
 *
 * Arguments and errors as casim_step; every pointer of casim_host_state is a
 * HOST pointer with the layout of casim_state.  The device buffers grow to
 * the largest block seen and are freed by casim_finalize. */
typedef struct casim_host_state {
    const double *in[CASIM_NIN];
    const double *dz;
    int64_t ld;
    double *tend[CASIM_NTEND];
    double *sfc[CASIM_NSFC];
} casim_host_state;

int casim_step_host(const casim_host_state *hs, int64_t ncol, int32_t nlev, double dt, int32_t nblocks,
                    void *stream);

/* Where the time of the last casim_step_host went (the split the paper
 * reports per step, Sec. III-C table of copy-on, kernel and copy-off times):
 * the summed durations of its inbound copies, its steps and its outbound
 * copies over all column blocks, in ms, from events on the three internal
 * streams (the three overlap in time, so their sum exceeds the call's wall
 * time).  Waits for those events.  *nblocks (may be NULL) receives the
 * number of blocks.  Zeros before any casim_step_host.  Errors: EINVAL (NULL
 * outputs), EHIP. */
int casim_host_times(double *h2d_ms, double *step_ms, double *d2h_ms, int32_t *nblocks);

/* [proposal] Page-locked host memory for casim_step_host (hipHostMalloc),
 * which the asynchronous copies of Sec. III-B need; *p is NULL on failure.
 * Errors: EINVAL (NULL p), EHIP. */
int casim_host_alloc(void **p, size_t bytes);
int casim_host_free(void *p);

/* [proposal] Diagnostics: the streaming floor of casim_step's own memory
 * traffic.  Runs the step's sweep with its tiles, launch order and activity
 * test and makes the loads the step makes (8 fields per point, the other 6
 * where a chunk is busy), then stores zeros as the 12 tendencies and
 * surface values -- no physics.  Its time is what the step's bytes cost in
 * the step's own access pattern; the outputs are meaningless.  Arguments
 * and errors as casim_step (the mode of the context is ignored). */
int casim_debug_stream(const casim_state *s, int64_t ncol, int32_t nlev, double dt, void *stream);

/* [proposal] Diagnostics: the device's streaming ceiling, from hand-written
 * kernels with non-temporal loads and stores of `width` (8 or 16) bytes per
 * lane and a grid-stride loop over `blocks` blocks of 256 threads.  kind 0
 * copies `bytes` from src to dst; kind 1 reads src and stores one XOR of
 * each block's words at the start of dst (the XOR of those values is the
 * XOR of all words of src); kind 2 writes zeros to dst (src unused, may be
 * NULL).  src and dst are device pointers aligned to `width`, dst holds
 * `bytes` bytes for every kind, bytes is a multiple of `width`, 1 <= blocks
 * <= 2^20.  Needs no casim_init.  Errors: EINVAL (kind, width, size, block
 * count, NULL or misaligned pointers), EHIP. */
int casim_debug_bandwidth(const void *src, void *dst, int64_t bytes, int32_t kind, int32_t width, int32_t blocks,
                          void *stream);

/* [proposal] Diagnostics: evaluate the binary64 exponential and logarithm that the
 * step kernels use internally, elementwise on n device values x (x > 0 for a
 * meaningful log), into device arrays exp_out and log_out (either may be
 * NULL).  Lets callers check their accuracy against a host library.
 * Errors: EINVAL (NULL x, n < 0), EHIP. */
int casim_debug_math(const double *x, int64_t n, double *exp_out, double *log_out, void *stream);

#ifdef __cplusplus
}
#endif
#endif
