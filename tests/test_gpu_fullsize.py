"""Parity at the benchmark's full sizes and launch configuration, and at the
largest level count the library accepts.

The 1024 x 1024 x 120 domains run whole on the GPU, as `bench.py` times them
(fields stored with the padded leading dimension casim_padded_ld gives,
16-column tiles in binary64 and 32 in FP32-mixed, XCD groups of 64 blocks,
and from the second step on the launch order built from the previous
step's activity); columns are independent, so the oracle checks a sample of
them one by one: every tenth tile's first column, the first and last 64
columns and 1024 random ones.
"""
import numpy as np
import pytest

from paper_2010_14823_amd import synth
from util import field_errors

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _sample(ncol, rng):
    idx = np.concatenate([np.arange(64), np.arange(ncol - 64, ncol), np.arange(0, ncol, 160),
                          rng.choice(ncol, 1024, replace=False)])
    return np.unique(idx)


@pytest.mark.parametrize("key,mode", [("c3", 0), ("c2", 0), ("c3", 1)])
def test_full_domain_sampled_columns(oracle_lib, key, mode):
    """mode 0: binary64, bound 1e-12; mode 1: FP32-mixed (rates and fall
    speeds in float32), bound 2e-4 as for its ten-step test."""
    import torch
    from paper_2010_14823_amd import casim
    cfg = synth.CONFIGS[key]
    f, dz, _ = synth.generate(cfg)
    st = synth.stack(f)
    del f
    ncol = st.shape[2]
    ld = casim.padded_ld(ncol)
    assert ld == ncol + 256
    dev = casim.empty_fields(14, cfg.nlev, ncol)
    dev.copy_(torch.from_numpy(st))
    tbuf = torch.full((12, cfg.nlev, ld), -7.0, dtype=torch.float64, device="cuda")
    tend = tbuf[:, :, :ncol]
    sfc = torch.full((8, ncol), -7.0, dtype=torch.float64, device="cuda")
    casim.init(casim.default_constants(mode=mode))
    casim.status()
    idx = _sample(ncol, np.random.default_rng(11))
    it = torch.from_numpy(idx).cuda()
    outs = []
    for _ in range(2):            # the second step runs in the activity-derived order
        casim.step(dev, dz, cfg.dt, tend, sfc)
        torch.cuda.synchronize()
        outs.append((tend.index_select(2, it).cpu().numpy(), sfc.index_select(1, it).cpu().numpy()))
        assert not bool((tend == -7.0).any()) and not bool((sfc == -7.0).any())
    # the padding columns of the leading dimension are never written
    assert bool((tbuf[:, :, ncol:] == -7.0).all())
    status = casim.status()
    del dev, tend, tbuf, sfc
    torch.cuda.empty_cache()
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    to, so = oracle_lib.step(np.ascontiguousarray(st[:, :, idx]), dz, cfg.dt)
    errs = field_errors(outs[1][0], outs[1][1], to, so)
    print(key, "mode", mode, "sampled columns", idx.size, {k: float("%.3g" % v) for k, v in errs.items()}, status,
          flush=True)
    bad = {k: v for k, v in errs.items() if not v <= (TOL if mode == 0 else 2e-4)}
    assert not bad, bad
    assert status["nonfinite"] == 0


def test_largest_level_count(oracle_lib):
    """512 levels (CASIM_MAX_NLEV): parity where the carry slots fit (dt = 1 s,
    44 slots) and a capacity error, before anything is enqueued, where they
    do not (dt = 2 s: 88 slots)."""
    import torch
    from paper_2010_14823_amd import casim
    cfg = synth.Config("levels512", 16, 12, 512, 7, 0.5)
    f, dz, _ = synth.generate(cfg)
    st = synth.stack(f)
    dev = torch.from_numpy(st).cuda()
    tend = torch.full((12, 512, cfg.ncol), -7.0, dtype=torch.float64, device="cuda")
    sfc = torch.full((8, cfg.ncol), -7.0, dtype=torch.float64, device="cuda")
    casim.init()
    casim.status()
    casim.step(dev, dz, 1.0, tend, sfc)
    torch.cuda.synchronize()
    to, so, fails = oracle_lib.step(st, dz, 1.0, return_fails=True)
    errs = field_errors(tend.cpu().numpy(), sfc.cpu().numpy(), to, so)
    status = casim.status()
    print("512 levels", {k: float("%.3g" % v) for k, v in errs.items()}, status, flush=True)
    assert max(errs.values()) <= TOL, errs
    assert status["newton_fail"] == fails and status["nonfinite"] == 0
    tend.fill_(-7.0)
    with pytest.raises(casim.CasimError) as e:
        casim.step(dev, dz, 2.0, tend, sfc)
    assert e.value.code == -3             # CASIM_ECAPACITY
    torch.cuda.synchronize()
    assert bool((tend == -7.0).all())


def test_fp32mix_wide_tiles_ragged_domain(oracle_lib, monkeypatch):
    """The FP32-mixed kernel picks 32-column tiles on domains of 262,144
    columns or more; on 521 x 509 columns x 21 levels (a ragged last tile,
    a half-filled last chunk of 2 levels) its output
    matches the oracle on the sampled columns (last tile included) to the
    FP32-mixed bound, and equals the 16-column tiling bit for bit (a point's
    arithmetic does not depend on the tile shape: the flux from the level
    above arrives by a lane shuffle or from the carry in LDS, the same
    value either way)."""
    import torch
    from paper_2010_14823_amd import casim
    cfg = synth.Config("wide_ragged", 521, 509, 21, 21, 0.5)
    f, dz, _ = synth.generate(cfg)
    st = synth.stack(f)
    del f
    ncol = st.shape[2]
    assert ncol % 32 != 0 and ncol // 32 >= 8192
    dev = torch.from_numpy(st).cuda()
    idx = _sample(ncol, np.random.default_rng(5))
    it = torch.from_numpy(idx).cuda()
    outs = {}
    for tiles in ("auto", "16"):
        if tiles == "16":
            monkeypatch.setenv("CASIM_COLS_PER_WAVE", "16")
        tend = torch.full((12, cfg.nlev, ncol), -7.0, dtype=torch.float64, device="cuda")
        sfc = torch.full((8, ncol), -7.0, dtype=torch.float64, device="cuda")
        casim.init(casim.default_constants(mode=1))
        casim.step(dev, dz, cfg.dt, tend, sfc)
        torch.cuda.synchronize()
        assert not bool((tend == -7.0).any()) and not bool((sfc == -7.0).any())
        outs[tiles] = (tend.index_select(2, it).cpu().numpy(), sfc.index_select(1, it).cpu().numpy())
        del tend, sfc
    to, so = oracle_lib.step(np.ascontiguousarray(st[:, :, idx]), dz, cfg.dt)
    errs = field_errors(outs["auto"][0], outs["auto"][1], to, so)
    cross = field_errors(outs["auto"][0], outs["auto"][1], outs["16"][0], outs["16"][1])
    print("wide ragged fp32mix: vs oracle", max(errs.values()), "32 vs 16 columns", max(cross.values()), flush=True)
    assert max(errs.values()) <= 2e-4, errs
    assert np.array_equal(outs["auto"][0], outs["16"][0]) and np.array_equal(outs["auto"][1], outs["16"][1]), cross
