"""The compacted binary64 mode (rates evaluated by a separate kernel over a
dense list of the points whose rate gates are open) against the CPU oracle,
to the same 1e-12 normwise bound as the fused path, and against the fused
path itself on the GPU."""
import numpy as np
import pytest

from paper_2010_14823_amd import synth
from util import config_state, field_errors, run_gpu

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _compact(**kw):
    from paper_2010_14823_amd import casim
    return dict(mode=casim.MODE_FP64_COMPACT, **kw)


def _check(oracle_lib, st, dz, dt, tag, **kw):
    okw = {k: v for k, v in kw.items() if k in ("stages", "warm", "newton_iters")}
    if "constants" in kw:
        okw["warm"] = bool(kw["constants"].warm)
        okw["stages"] = kw["constants"].stages
    tg, sg, status, _ = run_gpu(st, dz, dt, **kw)
    ncol = kw.get("ncol") or st.shape[2]
    to, so, fails = oracle_lib.step(st[:, :, :ncol], dz, dt, return_fails=True, **okw)
    errs = field_errors(tg[:, :, :ncol], sg[:, :ncol], to, so)
    print(tag, {k: float("%.3g" % v) for k, v in errs.items()}, status, flush=True)
    bad = {k: v for k, v in errs.items() if not v <= TOL}
    assert not bad, bad
    assert status["nonfinite"] == 0
    assert status["newton_fail"] == fails
    return tg, sg


def test_compact_c0(oracle_lib):
    cfg, st, dz, _ = config_state("c0")
    _check(oracle_lib, st, dz, cfg.dt, "compact c0", **_compact())


def test_compact_c1_and_clear_columns_zero(oracle_lib):
    cfg, st, dz, cols = config_state("c1")
    tg, sg = _check(oracle_lib, st, dz, cfg.dt, "compact c1", **_compact())
    clear = ~synth.cloud_mask(cfg)[cols]
    assert np.all(tg[:, :, clear] == 0.0) and np.all(sg[:, clear] == 0.0)


@pytest.mark.parametrize("key", ["c2", "c3"])
def test_compact_row_subsets(oracle_lib, key):
    cfg = synth.CONFIGS[key]
    rows = list(range(0, cfg.ny, cfg.ny // 16))[:16]
    cfg, st, dz, _ = config_state(key, rows)
    _check(oracle_lib, st, dz, cfg.dt, "compact " + key, **_compact())


def test_compact_warm_stages_and_generic(oracle_lib):
    from paper_2010_14823_amd import casim
    cfg, st, dz, _ = config_state("c0")
    _check(oracle_lib, st, dz, cfg.dt, "compact warm", **_compact(warm=1))
    for stages in (4, 7, 12):
        _check(oracle_lib, st, dz, cfg.dt, "compact stages%d" % stages, **_compact(stages=stages))
    c = casim.default_constants(mode=casim.MODE_FP64_COMPACT, flags=casim.FLAG_GENERIC)
    _check(oracle_lib, st, dz, cfg.dt, "compact generic", constants=c)


@pytest.mark.parametrize("cols_per_wave", [4, 16, 64])
def test_compact_ragged_tiles(oracle_lib, cols_per_wave, monkeypatch):
    monkeypatch.setenv("CASIM_COLS_PER_WAVE", str(cols_per_wave))
    cfg = synth.Config("tiles", 13, 7, 101, 17, 0.5, deep=True)
    f, dz, _ = synth.generate(cfg)
    st = synth.stack(f)
    for dt in (2.0, 7.0):
        _check(oracle_lib, st, dz, dt, "compact C%d dt=%g" % (cols_per_wave, dt), **_compact(ld=96))


def test_compact_matches_fused_and_reuses_scratch(oracle_lib):
    """Same answers as the fused binary64 sweep, also when a second, smaller
    domain reuses the slot scratch of the first."""
    from paper_2010_14823_amd import casim
    cfg, st, dz, _ = config_state("c1")
    ref_t, ref_s, _, _ = run_gpu(st, dz, cfg.dt)
    for ncol in (st.shape[2], 1000):
        tg, sg, status, _ = run_gpu(st, dz, cfg.dt, mode=casim.MODE_FP64_COMPACT, ncol=ncol)
        rt, rs, _, _ = run_gpu(st, dz, cfg.dt, ncol=ncol)
        errs = field_errors(tg[:, :, :ncol], sg[:, :ncol], rt[:, :, :ncol], rs[:, :ncol])
        same = np.array_equal(tg[:, :, :ncol], rt[:, :, :ncol]) and np.array_equal(sg[:, :ncol], rs[:, :ncol])
        print("compact vs fused ncol=%d bitwise=%s" % (ncol, same), {k: float("%.3g" % v) for k, v in errs.items()})
        assert max(errs.values()) <= 1e-13, errs
    assert np.array_equal(ref_t[:, :, :1000], rt[:, :, :1000])
