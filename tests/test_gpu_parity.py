"""Parity of the HIP path (through the C ABI) with the CPU oracle.

FP64 contract: for each of the 12 tendency fields and the 8 surface fields,
max|gpu - oracle| / max|oracle| <= 1e-12 (normwise; pointwise relative error
is ill-conditioned where q_v - q_sat cancels).  Clear subsaturated columns
must come out as exact zeros.
"""
import numpy as np
import pytest

from paper_2010_14823_amd import synth
from util import SFC, TEND, config_state, field_errors, oracle_steps, oracle_ulp_floor, run_gpu

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _assert_parity(oracle_lib, st, dz, dt, tol=TOL, tag="", **kw):
    okw = {k: v for k, v in kw.items() if k in ("stages", "warm", "newton_iters")}
    if "constants" in kw:
        okw["warm"] = bool(kw["constants"].warm)
        okw["stages"] = kw["constants"].stages
    tg, sg, status, _ = run_gpu(st, dz, dt, **kw)
    ncol = kw.get("ncol") or st.shape[2]
    to, so, fails = oracle_lib.step(st[:, :, :ncol], dz, dt, return_fails=True, **okw)
    errs = field_errors(tg[:, :, :ncol], sg[:, :ncol], to, so)
    print(tag, {k: float("%.3g" % v) for k, v in errs.items()}, status, "oracle newton fails", fails, flush=True)
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, bad
    assert status["nonfinite"] == 0
    assert status["newton_fail"] == fails
    return tg, sg, to, so


def test_c0_full(oracle_lib):
    cfg, st, dz, _ = config_state("c0")
    _assert_parity(oracle_lib, st, dz, cfg.dt, tag="c0")


def test_c1_full_and_clear_columns_zero(oracle_lib):
    cfg, st, dz, cols = config_state("c1")
    tg, sg, to, so = _assert_parity(oracle_lib, st, dz, cfg.dt, tag="c1")
    clear = ~synth.cloud_mask(cfg)[cols]
    assert clear.sum() > 1000
    assert np.all(tg[:, :, clear] == 0.0)
    assert np.all(sg[:, clear] == 0.0)


@pytest.mark.parametrize("key", ["c2", "c3", "c4"])
def test_large_config_row_subset(oracle_lib, key):
    # columns are independent: a subset of grid rows is the full computation
    cfg = synth.CONFIGS[key]
    rows = list(range(0, cfg.ny, cfg.ny // 24))[:24]
    cfg, st, dz, cols = config_state(key, rows)
    _assert_parity(oracle_lib, st, dz, cfg.dt, tag=key)


def test_ragged_tail_and_padding(oracle_lib):
    cfg, st, dz, _ = config_state("c0")
    # 50 columns in a leading dimension of 77: padding holds NaN and must stay unread/unwritten
    tg, sg, status, _ = run_gpu(st, dz, cfg.dt, ncol=50, ld=77)
    to, so = oracle_lib.step(st[:, :, :50], dz, cfg.dt)
    errs = field_errors(tg[:, :, :50], sg[:, :50], to, so)
    assert max(errs.values()) <= TOL, errs
    assert np.all(tg[:, :, 50:] == -7.0) and np.all(sg[:, 50:] == -7.0)
    assert status["nonfinite"] == 0


@pytest.mark.parametrize("ncol", [1, 63, 65, 129])
def test_odd_column_counts(oracle_lib, ncol):
    cfg = synth.Config("odd", 16, 9, 60, 21, 0.5)
    f, dz, _ = synth.generate(cfg)
    st = synth.stack(f)[:, :, :ncol].copy()
    _assert_parity(oracle_lib, st, dz, 2.0, tag="ncol%d" % ncol)


def test_single_level_and_zero_columns(oracle_lib):
    cfg, st, dz, _ = config_state("c0")
    one = st[:, 30:31, :].copy()
    _assert_parity(oracle_lib, one, dz[30:31], 2.0, tag="nlev1")
    import torch
    from paper_2010_14823_amd import casim
    casim.init()
    dev = torch.zeros((14, 3, 4), dtype=torch.float64, device="cuda")
    tend = torch.full((12, 3, 4), -1.0, dtype=torch.float64, device="cuda")
    sfc = torch.full((8, 4), -1.0, dtype=torch.float64, device="cuda")
    casim.step(dev, [10.0, 10.0, 10.0], 2.0, tend, sfc, ncol=0)
    torch.cuda.synchronize()
    assert torch.all(tend == -1.0)


@pytest.mark.parametrize("dt", [0.5, 10.0])
def test_many_substeps(oracle_lib, dt):
    cfg = synth.Config("deep120", 32, 4, 120, 5, 0.5, deep=True)
    f, dz, _ = synth.generate(cfg)
    st = synth.stack(f)
    ns = oracle_lib.nsub(dz, dt)
    print("nsub", ns)
    _assert_parity(oracle_lib, st, dz, dt, tag="dt%g" % dt)


@pytest.mark.parametrize("stages", [1, 2, 3, 4, 8, 7, 12])
def test_stage_subsets(oracle_lib, stages):
    cfg, st, dz, _ = config_state("c0")
    _assert_parity(oracle_lib, st, dz, cfg.dt, stages=stages, tag="stages%d" % stages)


def test_warm_configuration(oracle_lib):
    cfg, st, dz, _ = config_state("c0")
    tg, sg, to, so = _assert_parity(oracle_lib, st, dz, cfg.dt, warm=1, tag="warm")
    for j in range(6, 12):
        assert np.all(tg[j] == 0.0)


def test_warm_configuration_c1_sixteen_column_tiles(oracle_lib):
    """The compiled-in warm kernel at the tile width the benchmark uses on the
    large domains: the whole 256 x 256 x 100 domain (65,536 columns select
    16-column tiles), two steps on the same state so that the second runs in
    the activity-derived launch order."""
    import torch
    from paper_2010_14823_amd import casim
    cfg, st, dz, _ = config_state("c1")
    assert st.shape[2] // 16 >= 2048           # the library picks 16-column tiles
    dev = torch.from_numpy(st).cuda()
    casim.init(casim.default_constants(warm=1))
    casim.status()
    outs = []
    for _ in range(2):
        tend = torch.full((12,) + st.shape[1:], -7.0, dtype=torch.float64, device="cuda")
        sfc = torch.full((8, st.shape[2]), -7.0, dtype=torch.float64, device="cuda")
        casim.step(dev, dz, cfg.dt, tend, sfc)
        torch.cuda.synchronize()
        outs.append((tend.cpu().numpy(), sfc.cpu().numpy()))
    status = casim.status()
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    tg, sg = outs[1]
    to, so, fails = oracle_lib.step(st, dz, cfg.dt, warm=True, return_fails=True)
    errs = field_errors(tg, sg, to, so)
    print("warm c1", {k: float("%.3g" % v) for k, v in errs.items()}, status)
    assert max(errs.values()) <= TOL, errs
    assert status["newton_fail"] == 2 * fails and status["nonfinite"] == 0
    for j in range(6, 12):
        assert np.all(tg[j] == 0.0)


@pytest.mark.parametrize("cols_per_wave", [16, 32])
def test_warm_configuration_forced_tiles(oracle_lib, cols_per_wave, monkeypatch):
    monkeypatch.setenv("CASIM_COLS_PER_WAVE", str(cols_per_wave))
    cfg = synth.Config("warmtiles", 37, 11, 100, 23, 0.5)
    f, dz, _ = synth.generate(cfg)
    _assert_parity(oracle_lib, synth.stack(f), dz, 2.0, warm=1, tag="warm C%d" % cols_per_wave)


def test_newton_failure_flag(oracle_lib):
    cfg, st, dz, _ = config_state("c0")
    tg, sg, status, _ = run_gpu(st, dz, cfg.dt, newton_iters=1)
    to, so, fails = oracle_lib.step(st, dz, cfg.dt, newton_iters=1, return_fails=True)
    assert fails > 0
    assert status["newton_fail"] == fails
    errs = field_errors(tg, sg, to, so)
    assert max(errs.values()) <= TOL, errs


def test_deterministic(oracle_lib):
    cfg, st, dz, _ = config_state("c0")
    a = run_gpu(st, dz, cfg.dt)
    b = run_gpu(st, dz, cfg.dt)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_nonfinite_input_counted(oracle_lib):
    cfg, st, dz, _ = config_state("c0")
    bad = st.copy()
    bad[4, 10, 3] = np.inf          # one infinite cloud mass
    tg, sg, status, _ = run_gpu(bad, dz, cfg.dt)
    assert status["nonfinite"] >= 1


def test_multistep_apply_matches_oracle(oracle_lib):
    """Four coupled steps.  Per field the bound is 1e-12 or ten times the
    oracle's own sensitivity to one-ulp perturbations of the states it steps
    from, whichever is larger: after a step the cloud sits at saturation and
    the next adjustment's increment is a cancelling difference of q_v and
    q_sat, which two correctly rounded binary64 evaluations do not share."""
    cfg, st, dz, _ = config_state("c0")
    tg, sg, status, state_after = run_gpu(st, dz, cfg.dt, steps=4)
    to, so = oracle_steps(oracle_lib, st, dz, cfg.dt, steps=4)
    errs = field_errors(tg, sg, to, so)
    floor, _ = oracle_ulp_floor(oracle_lib, st, dz, cfg.dt, 4)
    print("4 steps", {k: "%.2g (floor %.2g)" % (v, floor[k]) for k, v in errs.items()})
    bad = {k: (v, floor[k]) for k, v in errs.items() if not v <= max(TOL, 10 * floor[k])}
    assert not bad, bad
    # non-negativity of every q and n after the parent-model update
    assert np.all(state_after[3:] >= 0.0)


def test_argument_errors_on_device():
    import torch
    from paper_2010_14823_amd import casim
    casim.init()
    dev = torch.zeros((14, 3, 8), dtype=torch.float64, device="cuda")
    tend = torch.zeros((12, 3, 8), dtype=torch.float64, device="cuda")
    sfc = torch.zeros((8, 8), dtype=torch.float64, device="cuda")
    dz = [10.0, 10.0, 10.0]
    for kw in ({"dt": 0.0}, {"dt": float("nan")}, {"dz": [10.0, 0.0, 10.0]}, {"dz": [10.0, float("inf"), 1.0]}):
        a = {"dt": 2.0, "dz": dz}; a.update(kw)
        with pytest.raises(casim.CasimError) as e:
            casim.step(dev, a["dz"], a["dt"], tend, sfc)
        assert e.value.code == -1
    st = casim.make_state(dev, dz, tend, sfc, ld=4)      # ld < ncol
    assert casim.lib().casim_step(st, 8, 3, 2.0, None) == -1
    assert casim.lib().casim_step(st, 2, 600, 2.0, None) == -1


@pytest.mark.parametrize("cols_per_wave", [4, 8, 16, 32, 64])
@pytest.mark.parametrize("generic", [False, True])
def test_tile_widths_and_runtime_constants(oracle_lib, cols_per_wave, generic, monkeypatch):
    """Every wavefront tile (C columns x 64/C levels) and both the compiled-in
    and the run-time constant kernels, on a ragged domain with a partial last
    chunk (nlev not a multiple of 64/C) and several substeps."""
    from paper_2010_14823_amd import casim
    monkeypatch.setenv("CASIM_COLS_PER_WAVE", str(cols_per_wave))
    cfg = synth.Config("tiles", 13, 7, 101, 17, 0.5, deep=True)
    f, dz, _ = synth.generate(cfg)
    st = synth.stack(f)
    c = casim.default_constants(flags=casim.FLAG_GENERIC if generic else 0)
    for dt in (2.0, 7.0):
        _assert_parity(oracle_lib, st, dz, dt, constants=c,
                       tag="C%d generic=%d dt=%g" % (cols_per_wave, generic, dt))


@pytest.mark.parametrize("cols_per_wave", [16, 64])
def test_fp32mix_tiles_agree(oracle_lib, cols_per_wave, monkeypatch):
    """The mixed-precision path gives the same answer at every tile width (to
    binary32 rounding) and stays close to the binary64 oracle."""
    from paper_2010_14823_amd import casim
    monkeypatch.setenv("CASIM_COLS_PER_WAVE", str(cols_per_wave))
    cfg, st, dz, _ = config_state("c0")
    tg, sg, status, _ = run_gpu(st, dz, cfg.dt, mode=casim.MODE_FP32MIX)
    to, so = oracle_lib.step(st, dz, cfg.dt)
    errs = field_errors(tg, sg, to, so)
    print("fp32mix C=%d" % cols_per_wave, {k: float("%.3g" % v) for k, v in errs.items()})
    assert max(errs.values()) < 6e-5, errs        # measured 5.7e-6 (dng)


@pytest.mark.parametrize("mode", [0, 1])
def test_tile_order_is_a_pure_schedule(oracle_lib, mode):
    """The second step on a state launches the tiles in the order derived
    from the first step's activity (busy tiles never in the last dispatch
    round) and the blocks renumbered so that each XCD runs groups of
    neighbouring tiles; every tile is still processed exactly once, so all
    steps give bitwise the same tendencies, for the full domain and ragged
    ones with 16-, 8- and 4-column tiles (1, 2 and 4 wavefronts per block)."""
    import torch
    from paper_2010_14823_amd import casim
    cfg, st, dz, _ = config_state("c1")
    for ncol in (st.shape[2], 60001, 20001, 5001):
        dev = torch.from_numpy(np.ascontiguousarray(st[:, :, :ncol])).cuda()
        outs = []
        casim.init(casim.default_constants(mode=mode))
        for _ in range(3):
            tend = torch.full((12, cfg.nlev, ncol), -7.0, dtype=torch.float64, device="cuda")
            sfc = torch.full((8, ncol), -7.0, dtype=torch.float64, device="cuda")
            casim.step(dev, dz, cfg.dt, tend, sfc)
            torch.cuda.synchronize()
            outs.append((tend.cpu().numpy(), sfc.cpu().numpy()))
        for t, s in outs[1:]:
            assert np.array_equal(t, outs[0][0]) and np.array_equal(s, outs[0][1])
        assert not np.any(outs[0][0] == -7.0)


def test_streaming_floor_diagnostic_runs_and_stores_zeros():
    """casim_debug_stream (the step's traffic without physics) writes every
    tendency and surface value of the domain, all zero for finite inputs."""
    import torch
    from paper_2010_14823_amd import casim
    cfg, st, dz, _ = config_state("c1", rows=list(range(0, 256, 8)))
    dev = torch.from_numpy(st).cuda()
    tend = torch.full((12,) + st.shape[1:], -7.0, dtype=torch.float64, device="cuda")
    sfc = torch.full((8, st.shape[2]), -7.0, dtype=torch.float64, device="cuda")
    casim.init()
    for _ in range(2):
        casim.debug_stream(dev, dz, cfg.dt, tend, sfc)
    torch.cuda.synchronize()
    assert bool((tend == 0.0).all()) and bool((sfc == 0.0).all())


def test_padded_view_layout_matches_contiguous():
    """Fields passed as the columns view of padded storage (level stride
    casim_padded_ld, as `bench.py` allocates them) give the same bits as
    contiguous fields, on a ragged column count; the padding columns are
    neither read (NaN there stays out of every result) nor written; the
    binding refuses views the ABI cannot express."""
    import torch
    from paper_2010_14823_amd import casim
    cfg, st, dz, _ = config_state("c1", rows=list(range(0, 256, 8)))
    ncol = 8190
    st = np.ascontiguousarray(st[:, :, :ncol])
    tg, sg, _, _ = run_gpu(st, dz, cfg.dt)
    ld = casim.padded_ld(ncol)
    assert ld == 8192 + 256
    nlev = st.shape[1]
    sbuf = torch.full((14, nlev, ld), float("nan"), dtype=torch.float64, device="cuda")
    dev = sbuf[:, :, :ncol]
    dev.copy_(torch.from_numpy(st))
    tbuf = torch.full((12, nlev, ld), -7.0, dtype=torch.float64, device="cuda")
    tend = tbuf[:, :, :ncol]
    sfc = torch.full((8, ncol), -7.0, dtype=torch.float64, device="cuda")
    casim.init()
    casim.status()
    casim.step(dev, dz, cfg.dt, tend, sfc)
    torch.cuda.synchronize()
    assert np.array_equal(tend.cpu().numpy(), tg) and np.array_equal(sfc.cpu().numpy(), sg)
    assert bool((tbuf[:, :, ncol:] == -7.0).all())
    # the parent-model update on the view equals the one on contiguous fields
    ref = torch.from_numpy(st).cuda()
    rt, rs = tend.contiguous(), sfc.clone()
    casim.apply_tendencies(dev, dz, cfg.dt, tend, sfc)
    casim.apply_tendencies(ref, dz, cfg.dt, rt, rs)
    torch.cuda.synchronize()
    assert torch.equal(dev, ref) and bool(torch.isnan(sbuf[:, :, ncol:]).all())
    assert casim.status()["nonfinite"] == 0
    e = casim.empty_fields(12, nlev, ncol)
    assert tuple(e.shape) == (12, nlev, ncol) and e.stride(1) == ld
    with pytest.raises(ValueError):       # column stride 2
        casim.step(sbuf[:, :, 0:ncol:2], dz, cfg.dt, tbuf[:, :, 0:ncol:2], sfc)
    with pytest.raises(ValueError):       # tendencies with another leading dimension
        casim.step(dev, dz, cfg.dt, tend.contiguous(), sfc)
    with pytest.raises(ValueError):       # more columns than the view holds
        casim.step(dev, dz, cfg.dt, tend, sfc.new_zeros((8, ncol + 1)), ncol=ncol + 1)
