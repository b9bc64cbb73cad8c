// Host side of libcasim: the process-wide context, argument validation,
// constant upload and kernel dispatch behind the C ABI of include/casim.h.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "casim_internal.h"
#include "casim_mlp_internal.h"

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
    // rate-dump scratch: per-block counts and offsets, total
    int64_t *d_counts = nullptr, *d_offsets = nullptr, *d_total = nullptr;
    int64_t dump_blocks = 0;
    // slot of every point and the slot counter (surrogate and compacted steps)
    int32_t *d_idx = nullptr;
    unsigned long long *d_count = nullptr;
    int64_t idx_cap = 0;
    // surrogate-step scratch, sized for sur_cap points
    float *d_feat = nullptr, *d_rates = nullptr;
    uint16_t *d_gates = nullptr;
    uint8_t *d_fb = nullptr;
    int64_t sur_cap = 0;
    // compacted-step scratch: post-adjustment state [13][cmp_cap], rates [12][cmp_cap]
    double *d_cstate = nullptr, *d_crates = nullptr;
    int64_t cmp_cap = 0;
    // tile launch order: per-tile activity of the last step and the order
    // derived from it; the activity is reused only for the same domain
    int32_t *d_busy = nullptr, *d_order = nullptr;
    int64_t tile_cap = 0;
    bool hist = false;                      // false: the tile history is void
    int reserve_tiles = 0;
    // host-state pipeline: streams, events and two device buffer sets, each
    // [14 + 12][pipe_lev][pipe_ld] fields and [8][pipe_ld] surface values
    bool pipe_ready = false;
    hipStream_t s_in = nullptr, s_comp = nullptr, s_out = nullptr;
    hipEvent_t ev_start = nullptr, ev_in[2] = {}, ev_comp[2] = {}, ev_free[2] = {};
    double *d_pipe[2] = {};
    int64_t pipe_ld = 0, pipe_lev = 0;
    // timing events of the last casim_step_host: per block, start and end of
    // its inbound copies, its step and its outbound copies
    std::vector<hipEvent_t> tev;
    int64_t tev_blocks = 0;
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
    if (c->mode < CASIM_MODE_FP64 || c->mode > CASIM_MODE_FP64_COMPACT) return CASIM_EINVAL;
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

// Slots per region of the slot space for a step over npts points (the point
// pass runs 256-point blocks; block b fills region b % kSlotRegions).
int64_t region_cap(int64_t npts) {
    const int64_t blocks = (npts + 255) / 256;
    return (blocks + kSlotRegions - 1) / kSlotRegions * 256;
}

// The grow functions below drain the device before freeing buffers a step
// in flight may use.  Slot indices are int32, so the slot space of a step
// (kSlotRegions * region_cap(npts) >= npts) holds at most 2^31-1 slots.
int ensure_idx(int64_t npts) {
    if (kSlotRegions * region_cap(npts) > INT32_MAX) return CASIM_ECAPACITY;
    if (!g.d_count) HIP_TRY(hipMalloc(&g.d_count, sizeof(unsigned long long) * kSlotRegions * kCounterStride));
    if (npts <= g.idx_cap) return CASIM_OK;
    HIP_TRY(hipDeviceSynchronize());
    hipFree(g.d_idx);
    g.d_idx = nullptr;
    g.idx_cap = 0;
    HIP_TRY(hipMalloc(&g.d_idx, sizeof(int32_t) * npts));
    g.idx_cap = npts;
    return CASIM_OK;
}

// Surrogate-step scratch for the slot space of npts points.
int ensure_sur(int64_t npts) {
    int rc = ensure_idx(npts);
    if (rc) return rc;
    npts = kSlotRegions * region_cap(npts);
    if (npts <= g.sur_cap) return CASIM_OK;
    HIP_TRY(hipDeviceSynchronize());
    hipFree(g.d_feat); hipFree(g.d_rates); hipFree(g.d_gates); hipFree(g.d_fb);
    g.d_feat = nullptr; g.d_rates = nullptr; g.d_gates = nullptr; g.d_fb = nullptr;
    g.sur_cap = 0;
    HIP_TRY(hipMalloc(&g.d_feat, sizeof(float) * 12 * npts));
    HIP_TRY(hipMalloc(&g.d_rates, sizeof(float) * 12 * npts));
    HIP_TRY(hipMalloc(&g.d_gates, sizeof(uint16_t) * npts));
    HIP_TRY(hipMalloc(&g.d_fb, npts));
    g.sur_cap = npts;
    return CASIM_OK;
}

// Compacted-step scratch for the slot space of npts points (room for every
// point to be slotted).
int ensure_cmp(int64_t npts) {
    int rc = ensure_idx(npts);
    if (rc) return rc;
    npts = kSlotRegions * region_cap(npts);
    if (npts <= g.cmp_cap) return CASIM_OK;
    HIP_TRY(hipDeviceSynchronize());
    hipFree(g.d_cstate); hipFree(g.d_crates);
    hipFree(g.d_busy); hipFree(g.d_order);
    g.d_busy = g.d_order = nullptr;
    g.tile_cap = 0;
    g.hist = false;
    g.reserve_tiles = 0;
    g.d_cstate = nullptr; g.d_crates = nullptr;
    g.cmp_cap = 0;
    HIP_TRY(hipMalloc(&g.d_cstate, sizeof(double) * kCmpState * npts));
    HIP_TRY(hipMalloc(&g.d_crates, sizeof(double) * 12 * npts));
    g.cmp_cap = npts;
    return CASIM_OK;
}

int ensure_dump(int64_t blocks) {
    if (blocks <= g.dump_blocks) return CASIM_OK;
    HIP_TRY(hipDeviceSynchronize());
    hipFree(g.d_counts); hipFree(g.d_offsets);
    g.d_counts = nullptr; g.d_offsets = nullptr; g.dump_blocks = 0;
    HIP_TRY(hipMalloc(&g.d_counts, sizeof(int64_t) * blocks));
    HIP_TRY(hipMalloc(&g.d_offsets, sizeof(int64_t) * blocks));
    if (!g.d_total) HIP_TRY(hipMalloc(&g.d_total, sizeof(int64_t)));
    g.dump_blocks = blocks;
    return CASIM_OK;
}

int pipe_create() {
    if (g.pipe_ready) return CASIM_OK;
    // default priority on every stream
    HIP_TRY(hipStreamCreateWithFlags(&g.s_in, hipStreamNonBlocking));
    HIP_TRY(hipStreamCreateWithFlags(&g.s_comp, hipStreamNonBlocking));
    HIP_TRY(hipStreamCreateWithFlags(&g.s_out, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&g.ev_start, hipEventDisableTiming));
    for (int j = 0; j < 2; ++j) {
        HIP_TRY(hipEventCreateWithFlags(&g.ev_in[j], hipEventDisableTiming));
        HIP_TRY(hipEventCreateWithFlags(&g.ev_comp[j], hipEventDisableTiming));
        HIP_TRY(hipEventCreateWithFlags(&g.ev_free[j], hipEventDisableTiming));
    }
    g.pipe_ready = true;
    return CASIM_OK;
}

void pipe_destroy() {
    if (!g.pipe_ready) return;
    hipDeviceSynchronize();
    for (hipEvent_t e : g.tev) hipEventDestroy(e);
    g.tev.clear();
    g.tev_blocks = 0;
    hipStreamDestroy(g.s_in); hipStreamDestroy(g.s_comp); hipStreamDestroy(g.s_out);
    hipEventDestroy(g.ev_start);
    for (int j = 0; j < 2; ++j) {
        hipEventDestroy(g.ev_in[j]); hipEventDestroy(g.ev_comp[j]); hipEventDestroy(g.ev_free[j]);
        hipFree(g.d_pipe[j]);
        g.d_pipe[j] = nullptr;
    }
    g.pipe_ld = g.pipe_lev = 0;
    g.pipe_ready = false;
}

// Six timing events per column block of casim_step_host.
int ensure_timing_events(int64_t nb) {
    while ((int64_t)g.tev.size() < 6 * nb) {
        hipEvent_t e;
        HIP_TRY(hipEventCreate(&e));
        g.tev.push_back(e);
    }
    return CASIM_OK;
}

// The leading dimension casim_padded_ld recommends: whole 128-byte rows, and
// no row stride that is a multiple of 4 KB (such a stride puts the rows a
// wavefront reads together at identical low address bits, measured slower).
int64_t padded_columns(int64_t ncol) {
    if (ncol == 0) return 0;
    const int64_t ld = (ncol + 15) / 16 * 16;
    return ld % 512 == 0 ? ld + 256 : ld;
}

// Room for blocks of `ld` columns and `nlev` levels in both buffer sets,
// whose own leading dimension is padded as casim_padded_ld recommends.
int ensure_pipe(int64_t ld, int64_t nlev) {
    if (ld <= g.pipe_ld && nlev <= g.pipe_lev) return CASIM_OK;
    HIP_TRY(hipDeviceSynchronize());
    const int64_t pl = padded_columns(ld);
    const int64_t L = pl > g.pipe_ld ? pl : g.pipe_ld, K = nlev > g.pipe_lev ? nlev : g.pipe_lev;
    for (int j = 0; j < 2; ++j) {
        hipFree(g.d_pipe[j]);
        g.d_pipe[j] = nullptr;
    }
    g.pipe_ld = g.pipe_lev = 0;
    const size_t bytes = sizeof(double) * ((size_t)(CASIM_NIN + CASIM_NTEND) * K * L + (size_t)CASIM_NSFC * L);
    for (int j = 0; j < 2; ++j) HIP_TRY(hipMalloc(&g.d_pipe[j], bytes));
    g.pipe_ld = L;
    g.pipe_lev = K;
    return CASIM_OK;
}

int ensure_tiles(int64_t ntiles) {
    if (ntiles <= g.tile_cap) return CASIM_OK;
    HIP_TRY(hipDeviceSynchronize());
    hipFree(g.d_busy); hipFree(g.d_order);
    g.d_busy = g.d_order = nullptr;
    g.tile_cap = 0;
    g.hist = false;
    HIP_TRY(hipMalloc(&g.d_busy, sizeof(int32_t) * ntiles));
    HIP_TRY(hipMalloc(&g.d_order, sizeof(int32_t) * ntiles));
    g.tile_cap = ntiles;
    return CASIM_OK;
}

// Launch shape of the sweep's blocks: the number of XCDs the block
// renumbering assumes, its group size in blocks, and the clear tiles kept for
// each XCD's last dispatch round.  CASIM_XCDS sets the XCD count (default 8,
// the XCDs of an MI355X; 1 turns the renumbering off), CASIM_XCD_GROUP forces
// the group size.
struct TilePlan {
    int nxcd = kXcds, group = kXcdGroupMin;
    int64_t reserve = 0;
};

int tile_plan(const SweepGeometry &geo, TilePlan &tp) {
    static const int nxcd = [] {
        const char *e = getenv("CASIM_XCDS");
        const int v = e ? atoi(e) : kXcds;
        return v >= 1 && v <= 64 ? v : kXcds;
    }();
    static const int forced_group = [] {
        const char *e = getenv("CASIM_XCD_GROUP");
        const int v = e ? atoi(e) : 0;
        return v >= 1 && v <= 4096 ? v : 0;
    }();
    // Groups of 16 to 64 blocks (256 to 1024 columns): the largest power of
    // two that still gives every XCD 16 groups, so that clustered cloud
    // spreads evenly over the XCDs (measured: 32 on 65,536 columns, 64 on
    // 1,048,576; smaller groups lose the streaming gain, larger ones the
    // balance).
    int group = forced_group;
    if (!group) {
        group = kXcdGroupMin;
        while (group < kXcdGroupMax && geo.blocks / ((int64_t)nxcd * 16) >= 2 * group) group *= 2;
    }
    if (!g.reserve_tiles) {
        int cus = 0;
        HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, g.device));
        g.reserve_tiles = 12 * (cus > 0 ? cus : 1);       // one dispatch round: 3 wavefronts x 4 SIMDs per CU
    }
    tp.nxcd = nxcd;
    tp.group = group;
    tp.reserve = (g.reserve_tiles + nxcd - 1) / nxcd;    // one dispatch round of one XCD's compute units
    return CASIM_OK;
}

bool tile_order_enabled() {
    static const int enabled = [] { const char *e = getenv("CASIM_TILE_ORDER"); return e ? atoi(e) : 1; }();
    return enabled != 0;
}

// What a step's per-tile activity record belongs to: the next step reuses it
// for its launch order only on the same domain, mode and configuration.
struct TileHistory {
    bool valid = false;
    const void *in0 = nullptr;
    int64_t ncol = 0, ld = 0, tiles = 0;
    int32_t nlev = 0, mode = -1, warm = -1;
    bool same(const casim_state *s, int64_t nc, int32_t nl, int64_t nt) const {
        return valid && in0 == (const void *)s->in[0] && ncol == nc && ld == s->ld && nlev == nl &&
               mode == g.c.mode && warm == g.c.warm && tiles == nt;
    }
    void record(const casim_state *s, int64_t nc, int32_t nl, int64_t nt) {
        valid = true; in0 = s->in[0]; ncol = nc; ld = s->ld; nlev = nl; mode = g.c.mode; warm = g.c.warm;
        tiles = nt;
    }
};

// Tile order for this step (from the last step's activity when it ran on the
// same domain) and activity recording for the next, with the per-tile
// buffers busy / order (ntiles entries each) and their history hist.
int plan_tiles_with(const casim_state *s, int64_t ncol, int32_t nlev, SweepArgs &a, int32_t *busy, int32_t *order,
                    TileHistory &hist, hipStream_t st) {
    SweepGeometry geo;
    HIP_TRY(sweep_geometry(ncol, a.nslots, nlev, a.mode, &geo));
    TilePlan tp;
    int rc = tile_plan(geo, tp);
    if (rc) return rc;
    a.nxcd = tp.nxcd;
    a.xcd_group = tp.group;
    a.ntiles = geo.tiles;
    a.tile_busy = busy;
    a.order = nullptr;
    if (hist.same(s, ncol, nlev, geo.tiles) && tile_order_enabled()) {
        HIP_TRY(launch_tile_order(busy, geo, tp.nxcd, tp.group, tp.reserve, order, st));
        a.order = order;
    }
    hist.record(s, ncol, nlev, geo.tiles);
    return CASIM_OK;
}

TileHistory g_hist;        // history of the library-owned tile buffers

// ---- scratch of the allocation-free step ---------------------------------
// One statically allocated device array per GPU holds everything
// casim_step_noalloc needs beyond the caller's inputs and outputs: the
// device copy of dz, the step's four counters, and the per-tile activity
// record and launch order.  In host code `scratch` names a host-side stand-in
// of the symbol, never device memory: its device address on each GPU comes
// from hipGetSymbolAddress at initialisation and is kept in g_scratch[device].
constexpr int kNoAllocMaxTiles = 1 << 18;      // 4,194,304 columns at 16-column tiles
constexpr size_t kScrDz = 0;                                       // CASIM_MAX_NLEV doubles
constexpr size_t kScrStatus = kScrDz + sizeof(double) * CASIM_MAX_NLEV;     // 4 counters
constexpr size_t kScrBusy = kScrStatus + 256;                      // int32 [kNoAllocMaxTiles]
constexpr size_t kScrOrder = kScrBusy + sizeof(int32_t) * kNoAllocMaxTiles; // int32 [kNoAllocMaxTiles]
constexpr size_t kScratchBytes = kScrOrder + sizeof(int32_t) * kNoAllocMaxTiles;
constexpr int kMaxDevices = 64;
static_assert(kScrStatus % 256 == 0 && kScrBusy % 256 == 0 && kScrOrder % 256 == 0, "scratch layout");

__device__ __align__(256) unsigned char scratch[kScratchBytes];

unsigned char *g_scratch[kMaxDevices] = {};   // device address of `scratch` on each GPU
TileHistory g_scratch_hist[kMaxDevices];

// Called with device `dev` current (from casim_init).
int scratch_setup(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return CASIM_ECAPACITY;
    if (g_scratch[dev]) return CASIM_OK;
    void *p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return CASIM_EHIP;
    g_scratch[dev] = static_cast<unsigned char *>(p);
    g_scratch_hist[dev].valid = false;
    return CASIM_OK;
}

int plan_tiles(const casim_state *s, int64_t ncol, int32_t nlev, SweepArgs &a, hipStream_t st) {
    SweepGeometry geo;
    HIP_TRY(sweep_geometry(ncol, a.nslots, nlev, a.mode, &geo));
    int rc = ensure_tiles(geo.tiles);
    if (rc) return rc;
    if (!g.hist) g_hist.valid = false;
    rc = plan_tiles_with(s, ncol, nlev, a, g.d_busy, g.d_order, g_hist, st);
    g.hist = true;
    return rc;
}

// The surrogate step's rate path: features and gates of every point that
// can react go to a slot (point pass), the network turns each slot into 12
// rates and a trust-region flag.  Leaves the point -> slot map in d_idx.
int surrogate_front(const SweepArgs &a, hipStream_t st) {
    const int64_t npts = (int64_t)a.nlev * a.ncol;
    int rc = ensure_sur(npts);
    if (rc) return rc;
    HIP_TRY(launch_zero_u64(g.d_count, (int64_t)kSlotRegions * kCounterStride, st));
    PointArgs pa{};
    pa.s = a;
    pa.mode = POINT_SURR;
    pa.feat = g.d_feat;
    pa.gates = g.d_gates;
    pa.idx_map = g.d_idx;
    pa.counter = g.d_count;
    pa.rcap = region_cap(npts);
    HIP_TRY(launch_points(g.P, g.fast, pa, st));
    HIP_TRY(launch_surrogate_infer(surrogate_dev((float)g.t.sur_range_margin, (float)g.t.sur_maha_max), g.d_feat,
                                   g.d_gates, npts, g.d_count, pa.rcap, g.d_rates, g.d_fb, st));
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
    a.sur_idx = nullptr;
    a.sur_rates = nullptr;
    a.sur_fallback = nullptr;
    a.sur_f_min = g.t.sur_f_min;
    a.cmp_rates = nullptr;
    a.cmp_ld = 0;
    a.order = nullptr;
    a.tile_busy = nullptr;
    a.ntiles = 0;
    return CASIM_OK;
}

}  // namespace

const casim_thresholds *casim_current_thresholds() { return g.init ? &g.t : nullptr; }

int casim_record_hip_error(int code, const char *msg) {
    snprintf(g.last_hip, sizeof g.last_hip, "HIP error %d: %s", code, msg);
    return CASIM_EHIP;
}

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
    if ((rc = scratch_setup(dev))) return rc;
    for (auto &h : g_scratch_hist) h.valid = false;     // new constants or mode: index order first
    g.c = *c;
    g.t = *t;
    g.P = derive(*c, *t, gamma_table(*c));
    g.fast = defaults_apply(*c, *t);
    g.hist = false;                         // the next step runs in index order
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

int64_t casim_padded_ld(int64_t ncol) {
    if (ncol < 0 || ncol > ((int64_t)1 << 40)) return CASIM_EINVAL;
    return padded_columns(ncol);
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
    if (g.c.mode == CASIM_MODE_SURROGATE && !surrogate_ready()) return CASIM_ENOSURROGATE;
    SweepArgs a{};
    fill_args(s, ncol, nlev, dt, a);
    nsub_of(g.c, s->dz, nlev, dt, a.nsub);
    for (int j = 0; j < 4; ++j) a.dts[j] = dt / a.nsub[j];
    int slot = 0;
    for (int j = 0; j < 4; ++j) {
        a.slot0[j] = slot;
        slot += 2 * a.nsub[j];
    }
    a.nslots = slot;
    if (slot > kMaxCarrySlots) return CASIM_ECAPACITY;
    rc = upload_dz(s->dz, nlev);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (g.c.mode == CASIM_MODE_SURROGATE) {
        if ((rc = surrogate_front(a, st))) return rc;
        a.sur_idx = g.d_idx;
        a.sur_rates = g.d_rates;
        a.sur_fallback = g.d_fb;
    } else if (g.c.mode == CASIM_MODE_FP64_COMPACT) {
        // post-adjustment state of every point with an open rate gate -> dense
        // binary64 rates -> sweep
        const int64_t npts = (int64_t)nlev * ncol;
        if ((rc = ensure_cmp(npts))) return rc;
        HIP_TRY(launch_zero_u64(g.d_count, (int64_t)kSlotRegions * kCounterStride, st));
        PointArgs pa{};
        pa.s = a;
        pa.s.cmp_ld = g.cmp_cap;
        pa.mode = POINT_CSTATE;
        pa.idx_map = g.d_idx;
        pa.counter = g.d_count;
        pa.rcap = region_cap(npts);
        pa.cstate = g.d_cstate;
        HIP_TRY(launch_points(g.P, g.fast, pa, st));
        HIP_TRY(launch_dense_rates(g.P, g.fast, a.warm != 0, g.d_cstate, g.cmp_cap, g.d_count, pa.rcap, g.d_crates,
                                   st));
        a.sur_idx = g.d_idx;
        a.cmp_rates = g.d_crates;
        a.cmp_ld = g.cmp_cap;
    }
    if ((rc = plan_tiles(s, ncol, nlev, a, st))) return rc;
    HIP_TRY(launch_sweep(g.P, g.fast, a, st));
    return CASIM_OK;
}

int casim_step_noalloc(const casim_state *s, int64_t ncol, int32_t nlev, double dt, void *stream) {
    int rc = check_state(s, ncol, nlev, dt);
    if (rc) return rc;
    if (g.c.mode != CASIM_MODE_FP64 && g.c.mode != CASIM_MODE_FP32MIX) return CASIM_EINVAL;
    if (ncol == 0) return CASIM_OK;
    if (!s->dz) return CASIM_EINVAL;
    for (int f = 0; f < CASIM_NSFC; ++f)
        if (!s->sfc[f]) return CASIM_EINVAL;
    for (int k = 0; k < nlev; ++k)
        if (!pos_finite(s->dz[k])) return CASIM_EINVAL;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices || !g_scratch[dev]) return CASIM_ENOINIT;   // casim_init ran on another GPU
    unsigned char *scr = g_scratch[dev];
    SweepArgs a{};
    fill_args(s, ncol, nlev, dt, a);
    nsub_of(g.c, s->dz, nlev, dt, a.nsub);
    for (int j = 0; j < 4; ++j) a.dts[j] = dt / a.nsub[j];
    int slot = 0;
    for (int j = 0; j < 4; ++j) {
        a.slot0[j] = slot;
        slot += 2 * a.nsub[j];
    }
    a.nslots = slot;
    if (slot > kMaxCarrySlots) return CASIM_ECAPACITY;
    SweepGeometry geo;
    HIP_TRY(sweep_geometry(ncol, a.nslots, nlev, a.mode, &geo));
    if (geo.tiles > kNoAllocMaxTiles) return CASIM_ECAPACITY;
    hipStream_t st = (hipStream_t)stream;
    // the vertical grid goes into the scratch with the step (4 KB at most)
    double *dz_d = reinterpret_cast<double *>(scr + kScrDz);
    HIP_TRY(hipMemcpyAsync(dz_d, s->dz, sizeof(double) * nlev, hipMemcpyHostToDevice, st));
    a.dz = dz_d;
    a.status = reinterpret_cast<unsigned long long *>(scr + kScrStatus);
    rc = plan_tiles_with(s, ncol, nlev, a, reinterpret_cast<int32_t *>(scr + kScrBusy),
                         reinterpret_cast<int32_t *>(scr + kScrOrder), g_scratch_hist[dev], st);
    if (rc) return rc;
    HIP_TRY(launch_sweep(g.P, g.fast, a, st));
    return CASIM_OK;
}

int casim_step_host(const casim_host_state *hs, int64_t ncol, int32_t nlev, double dt, int32_t nblocks,
                    void *stream) {
    if (!g.init) return CASIM_ENOINIT;
    if (!hs || nblocks < 0) return CASIM_EINVAL;
    if (ncol < 0 || nlev < 1 || nlev > CASIM_MAX_NLEV || hs->ld < ncol || !isfinite(dt) || !(dt > 0.0))
        return CASIM_EINVAL;
    if (ncol == 0) return CASIM_OK;
    if (!hs->dz) return CASIM_EINVAL;
    for (int f = 0; f < CASIM_NIN; ++f)
        if (!hs->in[f]) return CASIM_EINVAL;
    for (int f = 0; f < CASIM_NTEND; ++f)
        if (!hs->tend[f]) return CASIM_EINVAL;
    for (int f = 0; f < CASIM_NSFC; ++f)
        if (!hs->sfc[f]) return CASIM_EINVAL;
    for (int k = 0; k < nlev; ++k)
        if (!pos_finite(hs->dz[k])) return CASIM_EINVAL;
    if (nblocks == 0) nblocks = 4;
    // block width: a multiple of 64 columns
    int64_t bw = (ncol + nblocks - 1) / nblocks;
    bw = (bw + 63) / 64 * 64;
    const int64_t nb = (ncol + bw - 1) / bw;
    // the checks casim_step makes on every block, made once before anything
    // is enqueued, so that a rejected call leaves no copy behind
    {
        int32_t ns[4];
        nsub_of(g.c, hs->dz, nlev, dt, ns);
        if (2 * (ns[0] + ns[1] + ns[2] + ns[3]) > kMaxCarrySlots) return CASIM_ECAPACITY;
        if (g.c.mode == CASIM_MODE_SURROGATE && !surrogate_ready()) return CASIM_ENOSURROGATE;
        if ((g.c.mode == CASIM_MODE_SURROGATE || g.c.mode == CASIM_MODE_FP64_COMPACT) &&
            kSlotRegions * region_cap((int64_t)nlev * bw) > INT32_MAX)
            return CASIM_ECAPACITY;
    }
    int rc = pipe_create();
    if (rc) return rc;
    if ((rc = ensure_pipe(bw, nlev))) return rc;
    if ((rc = ensure_timing_events(nb))) return rc;
    g.tev_blocks = 0;
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(hipEventRecord(g.ev_start, st));
    HIP_TRY(hipStreamWaitEvent(g.s_in, g.ev_start, 0));
    const size_t hp = sizeof(double) * hs->ld, dp = sizeof(double) * g.pipe_ld;
    const int64_t fld = g.pipe_lev * g.pipe_ld;      // elements per device field
    for (int64_t b = 0; b < nb; ++b) {
        const int j = (int)(b & 1);
        const int64_t c0 = b * bw, nc = ncol - c0 < bw ? ncol - c0 : bw;
        double *base = g.d_pipe[j];
        casim_state ds{};
        for (int f = 0; f < CASIM_NIN; ++f) ds.in[f] = base + f * fld;
        for (int f = 0; f < CASIM_NTEND; ++f) ds.tend[f] = base + (CASIM_NIN + f) * fld;
        for (int f = 0; f < CASIM_NSFC; ++f) ds.sfc[f] = base + (CASIM_NIN + CASIM_NTEND) * fld + f * g.pipe_ld;
        ds.dz = hs->dz;
        ds.ld = g.pipe_ld;
        // inbound: buffer set j is free once block b-2's outbound copies are done
        hipEvent_t *te = &g.tev[6 * b];
        if (b >= 2) HIP_TRY(hipStreamWaitEvent(g.s_in, g.ev_free[j], 0));
        HIP_TRY(hipEventRecord(te[0], g.s_in));
        for (int f = 0; f < CASIM_NIN; ++f)
            HIP_TRY(hipMemcpy2DAsync(const_cast<double *>(ds.in[f]), dp, hs->in[f] + c0, hp, sizeof(double) * nc,
                                     nlev, hipMemcpyHostToDevice, g.s_in));
        HIP_TRY(hipEventRecord(te[1], g.s_in));
        HIP_TRY(hipEventRecord(g.ev_in[j], g.s_in));
        // step
        HIP_TRY(hipStreamWaitEvent(g.s_comp, g.ev_in[j], 0));
        HIP_TRY(hipEventRecord(te[2], g.s_comp));
        if ((rc = casim_step(&ds, nc, nlev, dt, g.s_comp))) return rc;
        HIP_TRY(hipEventRecord(te[3], g.s_comp));
        HIP_TRY(hipEventRecord(g.ev_comp[j], g.s_comp));
        // outbound
        HIP_TRY(hipStreamWaitEvent(g.s_out, g.ev_comp[j], 0));
        HIP_TRY(hipEventRecord(te[4], g.s_out));
        for (int f = 0; f < CASIM_NTEND; ++f)
            HIP_TRY(hipMemcpy2DAsync(hs->tend[f] + c0, hp, ds.tend[f], dp, sizeof(double) * nc, nlev,
                                     hipMemcpyDeviceToHost, g.s_out));
        for (int f = 0; f < CASIM_NSFC; ++f)
            HIP_TRY(hipMemcpyAsync(hs->sfc[f] + c0, ds.sfc[f], sizeof(double) * nc, hipMemcpyDeviceToHost, g.s_out));
        HIP_TRY(hipEventRecord(te[5], g.s_out));
        HIP_TRY(hipEventRecord(g.ev_free[j], g.s_out));
        g.tev_blocks = b + 1;
    }
    // the outbound stream is in order, so its last event covers every block
    HIP_TRY(hipStreamWaitEvent(st, g.ev_free[(nb - 1) & 1], 0));
    return CASIM_OK;
}

int casim_host_times(double *h2d_ms, double *step_ms, double *d2h_ms, int32_t *nblocks) {
    if (!h2d_ms || !step_ms || !d2h_ms) return CASIM_EINVAL;
    *h2d_ms = *step_ms = *d2h_ms = 0.0;
    if (nblocks) *nblocks = (int32_t)g.tev_blocks;
    if (!g.pipe_ready || g.tev_blocks == 0) return CASIM_OK;
    double sum[3] = {0.0, 0.0, 0.0};
    for (int64_t b = 0; b < g.tev_blocks; ++b) {
        for (int k = 0; k < 3; ++k) {
            HIP_TRY(hipEventSynchronize(g.tev[6 * b + 2 * k + 1]));
            float ms = 0.0f;
            HIP_TRY(hipEventElapsedTime(&ms, g.tev[6 * b + 2 * k], g.tev[6 * b + 2 * k + 1]));
            sum[k] += ms;
        }
    }
    *h2d_ms = sum[0];
    *step_ms = sum[1];
    *d2h_ms = sum[2];
    return CASIM_OK;
}

int casim_host_alloc(void **p, size_t bytes) {
    if (!p) return CASIM_EINVAL;
    *p = nullptr;
    HIP_TRY(hipHostMalloc(p, bytes, hipHostMallocDefault));
    return CASIM_OK;
}

int casim_host_free(void *p) {
    if (p) HIP_TRY(hipHostFree(p));
    return CASIM_OK;
}

int casim_rates_dump(const casim_state *s, int64_t ncol, int32_t nlev, double dt, uint64_t seed, double keep_prob,
                     int64_t max_samples, float *feat, float *rates, uint16_t *gates, int64_t *n_written,
                     int64_t *n_selected, void *stream) {
    int rc = check_state(s, ncol, nlev, dt);
    if (rc) return rc;
    if (!n_written || !(keep_prob > 0.0 && keep_prob <= 1.0) || max_samples < 0) return CASIM_EINVAL;
    if (max_samples > 0 && (!feat || !rates || !gates)) return CASIM_EINVAL;
    *n_written = 0;
    if (n_selected) *n_selected = 0;
    if (ncol == 0) return CASIM_OK;
    const int64_t npts = (int64_t)nlev * ncol;
    const int64_t blocks = (npts + 255) / 256;
    if ((rc = ensure_dump(blocks))) return rc;
    hipStream_t st = (hipStream_t)stream;
    PointArgs pa{};
    fill_args(s, ncol, nlev, dt, pa.s);
    pa.s.dz = nullptr;
    pa.seed = seed;
    pa.keep = keep_prob;
    pa.max_out = max_samples;
    pa.block_counts = g.d_counts;
    pa.block_offsets = g.d_offsets;
    pa.feat = feat;
    pa.rates = rates;
    pa.gates = gates;
    pa.mode = POINT_COUNT;
    HIP_TRY(launch_points(g.P, g.fast, pa, st));
    HIP_TRY(launch_scan(g.d_counts, blocks, g.d_offsets, g.d_total, st));
    if (max_samples > 0) {
        pa.mode = POINT_DUMP;
        HIP_TRY(launch_points(g.P, g.fast, pa, st));
    }
    int64_t total = 0;
    HIP_TRY(hipMemcpyAsync(&total, g.d_total, sizeof total, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    *n_written = total < max_samples ? total : max_samples;
    if (n_selected) *n_selected = total;
    return CASIM_OK;
}

int casim_surrogate_rates(const casim_state *s, int64_t ncol, int32_t nlev, double dt, float *rates,
                          uint8_t *flags, void *stream) {
    if (!g.init) return CASIM_ENOINIT;
    if (!s || !rates || !flags) return CASIM_EINVAL;
    if (ncol < 0 || nlev < 1 || nlev > CASIM_MAX_NLEV || s->ld < ncol || !isfinite(dt) || !(dt > 0.0))
        return CASIM_EINVAL;
    if (ncol == 0) return CASIM_OK;
    for (int f = 0; f < CASIM_NIN; ++f)
        if (!s->in[f]) return CASIM_EINVAL;
    if ((int64_t)nlev * s->ld > (int64_t)1 << 40) return CASIM_EINVAL;
    if (!surrogate_ready()) return CASIM_ENOSURROGATE;
    if (kSlotRegions * region_cap((int64_t)nlev * ncol) > INT32_MAX) return CASIM_ECAPACITY;
    SweepArgs a{};
    for (int f = 0; f < CASIM_NIN; ++f) a.in[f] = s->in[f];
    a.ld = s->ld;
    a.ncol = ncol;
    a.nlev = nlev;
    a.dt = dt;
    a.status = g.d_status;
    a.stages = g.c.stages;
    a.warm = g.c.warm ? 1 : 0;
    a.newton_iters = g.t.newton_iters;
    a.mode = g.c.mode;
    hipStream_t st = (hipStream_t)stream;
    int rc = surrogate_front(a, st);
    if (rc) return rc;
    HIP_TRY(launch_slot_scatter(g.d_idx, ncol, nlev, s->ld, g.d_rates, g.d_fb, rates, flags, st));
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
    unsigned long long h[4], hs[4] = {0, 0, 0, 0};
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    HIP_TRY(hipMemcpy(h, g.d_status, sizeof h, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemset(g.d_status, 0, sizeof h));
    // and the counters of the allocation-free step on the current device
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev >= 0 && dev < kMaxDevices && g_scratch[dev]) {
        HIP_TRY(hipMemcpy(hs, g_scratch[dev] + kScrStatus, sizeof hs, hipMemcpyDeviceToHost));
        HIP_TRY(hipMemset(g_scratch[dev] + kScrStatus, 0, sizeof hs));
        for (int j = 0; j < 4; ++j) h[j] += hs[j];
    }
    out->newton_fail = (int64_t)h[0];
    out->nonfinite = (int64_t)h[1];
    out->fallback = (int64_t)h[2];
    out->inferred = (int64_t)h[3];
    return CASIM_OK;
}

int casim_finalize(void) {
    pipe_destroy();
    if (g.d_dz || g.d_status) hipDeviceSynchronize();
    if (g.d_dz) hipFree(g.d_dz);
    if (g.d_status) hipFree(g.d_status);
    g.d_dz = nullptr;
    g.d_status = nullptr;
    hipFree(g.d_counts); hipFree(g.d_offsets); hipFree(g.d_total);
    g.d_counts = g.d_offsets = g.d_total = nullptr;
    g.dump_blocks = 0;
    hipFree(g.d_idx); hipFree(g.d_feat); hipFree(g.d_rates); hipFree(g.d_gates); hipFree(g.d_fb); hipFree(g.d_count);
    hipFree(g.d_cstate); hipFree(g.d_crates);
    hipFree(g.d_busy); hipFree(g.d_order);
    g.d_busy = g.d_order = nullptr;
    g.tile_cap = 0;
    g.hist = false;
    g.reserve_tiles = 0;
    g.d_idx = nullptr; g.d_feat = nullptr; g.d_rates = nullptr; g.d_gates = nullptr; g.d_fb = nullptr;
    g.d_count = nullptr; g.d_cstate = nullptr; g.d_crates = nullptr;
    g.idx_cap = g.sur_cap = g.cmp_cap = 0;
    g.h_dz.clear();
    g.init = false;
    g.device = -1;
    return CASIM_OK;
}

int casim_debug_stream(const casim_state *s, int64_t ncol, int32_t nlev, double dt, void *stream) {
    int rc = check_state(s, ncol, nlev, dt);
    if (rc) return rc;
    if (ncol == 0) return CASIM_OK;
    if (!s->dz) return CASIM_EINVAL;
    for (int f = 0; f < CASIM_NSFC; ++f)
        if (!s->sfc[f]) return CASIM_EINVAL;
    for (int k = 0; k < nlev; ++k)
        if (!pos_finite(s->dz[k])) return CASIM_EINVAL;
    SweepArgs a{};
    fill_args(s, ncol, nlev, dt, a);
    nsub_of(g.c, s->dz, nlev, dt, a.nsub);
    for (int j = 0; j < 4; ++j) a.dts[j] = dt / a.nsub[j];
    int slot = 0;
    for (int j = 0; j < 4; ++j) {
        a.slot0[j] = slot;
        slot += 2 * a.nsub[j];
    }
    a.nslots = slot;
    if (slot > kMaxCarrySlots) return CASIM_ECAPACITY;
    if ((rc = upload_dz(s->dz, nlev))) return rc;
    hipStream_t st = (hipStream_t)stream;
    a.mode = kModeStream;
    if ((rc = plan_tiles(s, ncol, nlev, a, st))) return rc;
    HIP_TRY(launch_sweep(g.P, true, a, st));
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
