"""Parity of the surrogate's GPU path with the oracle (oracle/surrogate.py,
oracle/mlp.py): statistics, the rate samples' features and gate words, the
surrogate step's own rate path (point pass -> slot -> matrix-core network ->
gates and signs, through casim_surrogate_rates), its trust-region flags, and
the step's use of the rates, on c0, on grid rows of c1 and on sampled
columns of the full 1024 x 1024 x 120 inference domain.

Every statistic and sample the oracle uses comes from the oracle itself; the
GPU receives the oracle's statistics through casim_mlp_set_stats.

Tolerances.  Features: the GPU takes the float32 hardware logarithm of the
binary64 state (error a few float32 ulps), so |df| <= 4e-6 max(1, |f|).
Network output, compared in the scaled target space asinh(rate / 1e-12):
the GPU and the emulation round the same float32 pre-activations to
bfloat16, but their float32 sums run in different orders, and the features
differ by the logarithm's rounding, so a pre-activation that lies within a
float32 rounding of a bfloat16 rounding boundary can round the other way
(one bfloat16 ulp, 2^-8 relative, in one activation); with 384 activations
per point such flips reach a few per cent of points.  One flip moves an
output by at most |w| * 2^-8 * |a| through the following layers.  Measured
on c0 and c1 rows: 99.9th percentile 0.0014, maximum 0.014 in asinh units;
the bounds below, 0.006 and 0.05, are 4 and 3.5 times that.  Trust-region flags agree exactly except for
points whose squared Mahalanobis distance lies within 1e-4 (relative) of the
limit or whose standardised feature lies within 1e-4 of a range bound.
"""
import numpy as np
import pytest

from oracle import mlp as omlp
from oracle import surrogate as osur
from paper_2010_14823_amd import synth
from util import config_state

pytestmark = pytest.mark.gpu

ASINH_Q999, ASINH_MAX = 0.006, 0.05


def oracle_samples(oracle_lib, st, warm=False):
    """Per point (point order k * ncol + c): adjusted state, rates, features,
    gate word, all from the oracle."""
    pts = st.transpose(1, 2, 0).reshape(-1, 14)
    n = len(pts)
    state = np.zeros((n, 12))
    rates = np.zeros((n, 12))
    for i, x in enumerate(pts):
        state[i], rates[i] = oracle_lib.point_process(x, warm=warm)
    feat = osur.features(state, pts[:, 1], pts[:, 2])
    gates = osur.gate_word(state, pts[:, 1], oracle_lib.qsat_liquid, oracle_lib.qsat_ice, warm=warm)
    return pts, state, rates, feat, gates


def to_mlpstats(st):
    from paper_2010_14823_amd import casim
    m = casim.MlpStats()
    for k in ("x_mean", "x_std", "x_min", "x_max", "y_mean", "y_std"):
        getattr(m, k)[:] = [float(v) for v in np.asarray(st[k], dtype=np.float32)]
    m.whiten[:] = [float(v) for v in np.asarray(st["whiten"], dtype=np.float32).ravel()]
    m.maha_q999 = float(np.float32(st["maha_q999"]))
    return m


def installed(st):
    """The statistics as the GPU holds them (float32 everywhere)."""
    out = {k: np.asarray(st[k], dtype=np.float32) for k in ("x_mean", "x_std", "x_min", "x_max", "y_mean", "y_std")}
    out["whiten"] = np.asarray(st["whiten"], dtype=np.float32).astype(np.float64)
    out["maha_q999"] = float(np.float32(st["maha_q999"]))
    return out


def random_theta(seed=9, scale=0.1):
    return np.random.default_rng(seed).normal(0, scale, omlp.N_PARAMS).astype(np.float32)


def setup_network(casim, oracle_lib, stats_source_st, theta):
    """Oracle statistics of the oracle's samples of stats_source_st installed
    on the GPU with parameters theta; returns the installed statistics."""
    _, _, rates, feat, gates = oracle_samples(oracle_lib, stats_source_st)
    keep = (gates & 0xFFF) != 0
    st = osur.fit_stats(feat[keep].astype(np.float32), rates[keep], gates[keep])
    casim.init()
    casim.mlp_set_stats(to_mlpstats(st))
    casim.mlp_set_params(theta)
    casim.surrogate_load()
    return installed(st)


def gpu_surrogate_rates(casim, st_np, dz, dt, ncol=None):
    import torch
    dev = torch.from_numpy(st_np).cuda()
    nlev, n = st_np.shape[1], st_np.shape[2]
    rates = torch.full((12, nlev, n), -1.0, dtype=torch.float32, device="cuda")
    flags = torch.full((nlev, n), 7, dtype=torch.uint8, device="cuda")
    casim.surrogate_rates(dev, dz, dt, rates, flags, ncol=ncol)
    torch.cuda.synchronize()
    return rates.cpu().numpy(), flags.cpu().numpy()


def near_boundary(z, st, margin):
    d2 = osur.maha2_whitened(z, st["whiten"])
    near = np.abs(d2 - st["maha_q999"]) <= 1e-4 * st["maha_q999"]
    lo = st["x_min"].astype(np.float64) - margin * (st["x_max"].astype(np.float64) - st["x_min"].astype(np.float64))
    hi = st["x_max"].astype(np.float64) + margin * (st["x_max"].astype(np.float64) - st["x_min"].astype(np.float64))
    zlo, zhi = osur.standardise(lo, st), osur.standardise(hi, st)
    near |= (np.minimum(np.abs(z - zlo), np.abs(z - zhi)) <= 1e-4 * np.maximum(1.0, np.abs(z))).any(axis=1)
    return near


def compare_rate_path(casim, oracle_lib, st_np, dz, dt, theta, stats, tag, margin=None):
    """GPU step-path rates and flags of every point against the oracle."""
    thr = casim.default_thresholds()
    margin = thr.sur_range_margin if margin is None else margin
    r_gpu, fl_gpu = gpu_surrogate_rates(casim, st_np, dz, dt)
    r_gpu = r_gpu.reshape(12, -1).T            # (points, 12) in point order
    fl_gpu = fl_gpu.reshape(-1)
    pts, state, _, feat, gates = oracle_samples(oracle_lib, st_np)
    slotted = (gates & 0xFFF) != 0
    assert np.array_equal(fl_gpu == 2, ~slotted), "slots differ from the open gates"
    assert np.all(r_gpu[~slotted] == 0.0)
    f32 = feat[slotted].astype(np.float32)
    r_or, fb_or = osur.infer(theta, stats, f32, gates[slotted], margin, stats["maha_q999"])
    fb_gpu = fl_gpu[slotted] == 1
    near = near_boundary(osur.standardise(f32, stats), stats, margin)
    mism = (fb_gpu != fb_or) & ~near
    assert not mism.any(), "%d trust-region flags differ away from the boundary" % mism.sum()
    # closed gates and signs agree exactly
    g = gates[slotted].astype(np.uint32)
    open_ = ((g[:, None] >> np.arange(12)) & 1) == 1
    assert np.all(r_gpu[slotted][~open_] == 0.0)
    assert np.all(np.sign(r_gpu[slotted][:, 3:5]) == np.sign(r_or[:, 3:5]))
    dy = np.abs(np.arcsinh(r_gpu[slotted].astype(np.float64) / 1e-12) - np.arcsinh(r_or / 1e-12))[open_]
    q999, mx = float(np.quantile(dy, 0.999)), float(dy.max())
    print("%s: %d slotted points, %d outside the trust region, |d asinh| 99.9%% %.3g max %.3g, "
          "flags near the boundary %d" % (tag, slotted.sum(), fb_gpu.sum(), q999, mx, near.sum()), flush=True)
    assert q999 < ASINH_Q999 and mx < ASINH_MAX
    return pts, state, r_or, fb_or, slotted


def test_fit_stats_matches_oracle(oracle_lib):
    """casim_mlp_fit_stats on oracle samples of c0 and c1 rows against the
    oracle's statistics of the same samples."""
    import torch
    from paper_2010_14823_amd import casim
    _, st0, _, _ = config_state("c0")
    _, st1, _, _ = config_state("c1", rows=[60, 61])
    feats, ratess, gatess = [], [], []
    for st in (st0, st1):
        _, _, rates, feat, gates = oracle_samples(oracle_lib, st)
        keep = (gates & 0xFFF) != 0
        feats.append(feat[keep]); ratess.append(rates[keep]); gatess.append(gates[keep])
    feat = np.concatenate(feats).astype(np.float32)
    rates = np.concatenate(ratess).astype(np.float32)
    gates = np.concatenate(gatess)
    n = len(feat)
    want = osur.fit_stats(feat, rates.astype(np.float64), gates)
    casim.init()
    got = casim.mlp_fit_stats(torch.from_numpy(feat).cuda(), torch.from_numpy(rates).cuda(),
                              torch.from_numpy(gates.astype(np.int16)).cuda(), n)
    g = {k: np.array(getattr(got, k)) for k in ("x_mean", "x_std", "x_min", "x_max", "y_mean", "y_std")}
    print("fit_stats on %d samples; maha q999 gpu %.6g oracle %.6g" % (n, got.maha_q999, want["maha_q999"]))
    assert np.allclose(g["x_mean"], want["x_mean"], rtol=2e-7, atol=1e-6)
    assert np.allclose(g["x_std"], want["x_std"], rtol=1e-5)
    assert np.array_equal(g["x_min"], want["x_min"]) and np.array_equal(g["x_max"], want["x_max"])
    assert np.allclose(g["y_mean"], want["y_mean"], rtol=1e-6, atol=1e-6)
    assert np.allclose(g["y_std"], want["y_std"], rtol=1e-5)
    w = np.array(got.whiten).reshape(12, 12)
    assert np.all(np.triu(w, 1) == 0.0)
    assert np.max(np.abs(w - want["whiten"])) <= 1e-5 * np.max(np.abs(want["whiten"]))
    # the GPU's percentile is the upper edge of its histogram bin (log10 bins of 12/4096)
    assert want["maha_q999"] <= got.maha_q999 * (1 + 1e-6) <= want["maha_q999"] * 10 ** (12 / 4096) * (1 + 1e-6)


def test_dump_features_and_gates_match_oracle(oracle_lib):
    """Every feature and gate word of casim_rates_dump against the oracle."""
    import torch
    from paper_2010_14823_amd import casim
    cfg, st, dz, _ = config_state("c0")
    dev = torch.from_numpy(st).cuda()
    nlev, ncol = st.shape[1], st.shape[2]
    cap = nlev * ncol
    tend = torch.empty((12, nlev, ncol), dtype=torch.float64, device="cuda")
    sfc = torch.empty((8, ncol), dtype=torch.float64, device="cuda")
    feat = torch.zeros((cap, 12), dtype=torch.float32, device="cuda")
    rates = torch.zeros((cap, 12), dtype=torch.float32, device="cuda")
    gates = torch.zeros((cap,), dtype=torch.int16, device="cuda")
    casim.init()
    n, _ = casim.rates_dump(dev, dz, cfg.dt, 3, 1.0, cap, feat, rates, gates, tend, sfc)
    f = feat[:n].cpu().numpy().astype(np.float64)
    g = gates[:n].cpu().numpy().astype(np.uint16)
    pts, state, r_or, f_or, g_or = oracle_samples(oracle_lib, st)
    # the dump holds every point where anything can happen, in point order
    qsl = np.array([oracle_lib.qsat_liquid(T, p) for T, p in pts[:, :2]])
    qsi = np.array([oracle_lib.qsat_ice(T, p) for T, p in pts[:, :2]])
    act = (pts[:, [4, 6, 8, 10, 12]] > 0).any(axis=1) | (pts[:, 3] > qsl) | ((pts[:, 0] < 268.15) & (pts[:, 3] > qsi))
    idx = np.nonzero(act)[0]
    assert len(idx) == n
    err = np.abs(f - f_or[idx]) / np.maximum(1.0, np.abs(f_or[idx]))
    print("dump: %d samples, worst feature error %.3g (feature %d)" % (n, err.max(), err.max(axis=0).argmax()))
    assert err.max() <= 4e-6
    assert np.array_equal(g, g_or[idx])


def test_plain_rows_inference_matches_emulation(oracle_lib):
    """casim_surrogate_infer on the oracle's own float32 features (no feature
    rounding between the two sides): rates and trust-region flags against the
    bfloat16 emulation."""
    import torch
    from paper_2010_14823_amd import casim
    _, st, _, _ = config_state("c0")
    theta = random_theta(9, 0.1)
    stats = setup_network(casim, oracle_lib, st, theta)
    _, _, _, feat, gates = oracle_samples(oracle_lib, config_state("c1", rows=[7])[1])
    keep = (gates & 0xFFF) != 0
    f32, g = feat[keep].astype(np.float32), gates[keep]
    n = len(f32)
    out = torch.empty((n, 12), dtype=torch.float32, device="cuda")
    fb = torch.empty((n,), dtype=torch.uint8, device="cuda")
    f_dev, g_dev = torch.from_numpy(f32).cuda(), torch.from_numpy(g.astype(np.int16)).cuda()
    casim.surrogate_infer(f_dev, g_dev, n, out, fb)
    r_gpu = out.cpu().numpy().astype(np.float64)
    # a batch smaller than one point tile gives the same rows bit for bit
    # (each point is its own column of every product)
    m = 7
    out_m = torch.empty((m, 12), dtype=torch.float32, device="cuda")
    fb_m = torch.empty((m,), dtype=torch.uint8, device="cuda")
    casim.surrogate_infer(f_dev[:m], g_dev[:m], m, out_m, fb_m)
    assert np.array_equal(out_m.cpu().numpy(), out.cpu().numpy()[:m])
    assert np.array_equal(fb_m.cpu().numpy(), fb.cpu().numpy()[:m])
    thr = casim.default_thresholds()
    r_or, fb_or = osur.infer(theta, stats, f32, g, thr.sur_range_margin, stats["maha_q999"])
    near = near_boundary(osur.standardise(f32, stats), stats, thr.sur_range_margin)
    assert not ((fb.cpu().numpy() == 1) != fb_or)[~near].any()
    open_ = ((g.astype(np.uint32)[:, None] >> np.arange(12)) & 1) == 1
    assert np.all(r_gpu[~open_] == 0.0)
    dy = np.abs(np.arcsinh(r_gpu / 1e-12) - np.arcsinh(r_or / 1e-12))[open_]
    print("plain rows: %d points, |d asinh| 99.9%% %.3g max %.3g" % (n, np.quantile(dy, 0.999), dy.max()))
    assert np.quantile(dy, 0.999) < ASINH_Q999 and dy.max() < ASINH_MAX


def test_step_path_rates_c0(oracle_lib):
    from paper_2010_14823_amd import casim
    cfg, st, dz, _ = config_state("c0")
    theta = random_theta()
    stats = setup_network(casim, oracle_lib, st, theta)
    compare_rate_path(casim, oracle_lib, st, dz, cfg.dt, theta, stats, "c0")
    # a narrow trust region sends many points to the plain rates: flags still agree
    casim.init(casim.default_constants(), casim.default_thresholds(sur_range_margin=-0.3))
    compare_rate_path(casim, oracle_lib, st, dz, cfg.dt, theta, stats, "c0 margin -0.3", margin=-0.3)


def test_step_path_rates_c1_rows(oracle_lib):
    from paper_2010_14823_amd import casim
    cfg, st, dz, _ = config_state("c1", rows=[100, 101, 170])
    theta = random_theta(21, 0.12)
    stats = setup_network(casim, oracle_lib, config_state("c1", rows=[40, 41])[1], theta)
    compare_rate_path(casim, oracle_lib, st, dz, cfg.dt, theta, stats, "c1 rows")


def test_surrogate_step_applies_the_network_rates(oracle_lib):
    """Surrogate step without sedimentation against the oracle's apply step
    with the oracle-emulated network rates where the point uses them (slot,
    inside the trust region, limiter factor >= sur_f_min) and the plain
    oracle elsewhere.  The rates differ by the emulation tolerance, which the
    tendency bound carries."""
    import torch
    from paper_2010_14823_amd import casim
    cfg, st, dz, _ = config_state("c0")
    theta = random_theta(5, 0.1)
    stats = setup_network(casim, oracle_lib, st, theta)
    thr = casim.default_thresholds()
    pts, state, r_or, fb_or, slotted = compare_rate_path(casim, oracle_lib, st, dz, cfg.dt, theta, stats, "c0")
    casim.init(casim.default_constants(mode=casim.MODE_SURROGATE, stages=7), thr)
    casim.status()
    dev = torch.from_numpy(st).cuda()
    tend = torch.empty((12,) + st.shape[1:], dtype=torch.float64, device="cuda")
    sfc = torch.empty((8, st.shape[2]), dtype=torch.float64, device="cuda")
    casim.step(dev, dz, cfg.dt, tend, sfc)
    s = casim.status()
    tg = tend.cpu().numpy().reshape(12, -1).T
    expect = np.zeros_like(tg)
    use = np.zeros(len(pts), dtype=bool)
    si = np.nonzero(slotted)[0]
    f = osur.limiter_min_f(state[si], r_or, cfg.dt)
    use[si] = ~fb_or & (f >= thr.sur_f_min)
    for i in range(len(pts)):
        if use[i]:
            expect[i] = oracle_lib.point_apply(pts[i], r_or[np.searchsorted(si, i)], cfg.dt)
        else:
            to, _ = oracle_lib.step(pts[i].reshape(14, 1, 1).copy(), np.array([500.0]), cfg.dt, stages=7)
            expect[i] = to[:, 0, 0]
    print("step: inferred %d (oracle %d), fallback %d" % (s["inferred"], use.sum(), s["fallback"]))
    assert abs(s["inferred"] - use.sum()) <= max(2, 0.002 * use.sum())
    den = np.abs(expect).max(axis=0)
    rel = np.abs(tg - expect) / np.where(den > 0, den, 1.0)
    print("step: normwise max %.3g, 99th percentile of the per-point worst field %.3g"
          % (rel.max(), np.quantile(rel.max(axis=1), 0.99)))
    # a wrong slot, gate or limiter decision gives O(1) errors
    assert rel.max() <= 0.1 and np.quantile(rel.max(axis=1), 0.99) <= 0.01
    if s["inferred"] == use.sum():
        # the points on the plain rates match the oracle to the binary64 bound
        assert rel[~use].max() <= 1e-12


def test_full_c4_sampled_columns(oracle_lib):
    """The step path on the whole 1024 x 1024 x 120 inference domain (the
    benchmark's launch configuration and padded field layout); sampled
    columns against the oracle."""
    import torch
    from paper_2010_14823_amd import casim
    cfg = synth.CONFIGS["c4"]
    f, dz, _ = synth.generate(cfg)
    st = synth.stack(f)
    del f
    ncol = st.shape[2]
    rng = np.random.default_rng(4)
    idx = np.unique(np.concatenate([np.arange(64), np.arange(ncol - 64, ncol), rng.choice(ncol, 768, replace=False)]))
    theta = random_theta(31, 0.1)
    stats = setup_network(casim, oracle_lib, np.ascontiguousarray(st[:, :, rng.choice(ncol, 256, replace=False)]),
                          theta)
    sub = np.ascontiguousarray(st[:, :, idx])
    dev = casim.empty_fields(14, cfg.nlev, ncol)
    dev.copy_(torch.from_numpy(st))
    del st
    ld = casim.padded_ld(ncol)
    rates = torch.full((12, cfg.nlev, ld), -1.0, dtype=torch.float32, device="cuda")
    flags = torch.full((cfg.nlev, ld), 7, dtype=torch.uint8, device="cuda")
    casim.surrogate_rates(dev, dz, cfg.dt, rates, flags)
    torch.cuda.synchronize()
    it = torch.from_numpy(idx).cuda()
    r_s = rates.index_select(2, it).cpu().numpy()
    fl_s = flags.index_select(1, it).cpu().numpy()
    del dev, rates, flags
    torch.cuda.empty_cache()
    pts, state, _, feat, gates = oracle_samples(oracle_lib, sub)
    r_gpu = r_s.reshape(12, -1).T
    fl = fl_s.reshape(-1)
    slotted = (gates & 0xFFF) != 0
    assert np.array_equal(fl == 2, ~slotted)
    thr = casim.default_thresholds()
    f32 = feat[slotted].astype(np.float32)
    r_or, fb_or = osur.infer(theta, stats, f32, gates[slotted], thr.sur_range_margin, stats["maha_q999"])
    near = near_boundary(osur.standardise(f32, stats), stats, thr.sur_range_margin)
    assert not ((fl[slotted] == 1) != fb_or)[~near].any()
    g = gates[slotted].astype(np.uint32)
    open_ = ((g[:, None] >> np.arange(12)) & 1) == 1
    dy = np.abs(np.arcsinh(r_gpu[slotted].astype(np.float64) / 1e-12) - np.arcsinh(r_or / 1e-12))[open_]
    print("c4 full: %d sampled columns, %d slotted points, |d asinh| 99.9%% %.3g max %.3g"
          % (idx.size, slotted.sum(), np.quantile(dy, 0.999), dy.max()), flush=True)
    assert np.quantile(dy, 0.999) < ASINH_Q999 and dy.max() < ASINH_MAX
