"""The host-state entry point (copy in, step, copy out over column blocks on
three streams) against the device-resident step and the CPU oracle."""
import numpy as np
import pytest

from paper_2010_14823_amd import synth
from util import config_state, field_errors, run_gpu

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _host_step(st, dz, dt, ncol, ld, nblocks, pinned=True):
    import torch
    from paper_2010_14823_amd import casim
    nlev = st.shape[1]
    if pinned:
        hin, hout, hsfc = (casim.HostArray((14, nlev, ld)), casim.HostArray((12, nlev, ld)),
                           casim.HostArray((8, ld)))
        a_in, a_out, a_sfc = hin.array, hout.array, hsfc.array
    else:
        a_in, a_out, a_sfc = np.empty((14, nlev, ld)), np.empty((12, nlev, ld)), np.empty((8, ld))
    a_in[:] = np.nan
    a_in[:, :, :ncol] = st[:, :, :ncol]
    a_out[:] = -7.0
    a_sfc[:] = -7.0
    casim.step_host(a_in, dz, dt, a_out, a_sfc, ncol=ncol, nblocks=nblocks)
    torch.cuda.synchronize()
    status = casim.status()
    out = a_out.copy(), a_sfc.copy()
    if pinned:
        for h in (hin, hout, hsfc):
            h.free()
    return out[0], out[1], status


@pytest.mark.parametrize("nblocks", [1, 3, 0])
def test_host_pipeline_c1_matches_device_path_and_oracle(oracle_lib, nblocks):
    from paper_2010_14823_amd import casim
    casim.init()
    cfg, st, dz, _ = config_state("c1")
    ncol = st.shape[2]
    tg, sg, status = _host_step(st, dz, cfg.dt, ncol, ncol, nblocks)
    rt, rs, _, _ = run_gpu(st, dz, cfg.dt)
    dev = field_errors(tg, sg, rt, rs)
    print("host pipeline nblocks=%d vs device path" % nblocks, {k: float("%.3g" % v) for k, v in dev.items()})
    assert max(dev.values()) <= 1e-13, dev
    to, so = oracle_lib.step(st, dz, cfg.dt)
    errs = field_errors(tg, sg, to, so)
    assert max(errs.values()) <= TOL, errs
    assert status["nonfinite"] == 0


def test_host_pipeline_ragged_blocks_and_padding(oracle_lib):
    from paper_2010_14823_amd import casim
    casim.init()
    cfg = synth.Config("ragged", 25, 40, 73, 5, 0.5)
    f, dz, _ = synth.generate(cfg)
    st = synth.stack(f)
    ncol, ld = 1000, 1037
    for nblocks, pinned in ((3, True), (7, False)):
        tg, sg, _ = _host_step(st, dz, cfg.dt, ncol, ld, nblocks, pinned=pinned)
        # padding columns are neither read nor written
        assert np.all(tg[:, :, ncol:] == -7.0) and np.all(sg[:, ncol:] == -7.0)
        to, so = oracle_lib.step(st[:, :, :ncol], dz, cfg.dt)
        errs = field_errors(tg[:, :, :ncol], sg[:, :ncol], to, so)
        print("ragged nblocks=%d pinned=%s" % (nblocks, pinned), max(errs.values()))
        assert max(errs.values()) <= TOL, errs


def test_host_pipeline_argument_errors():
    import ctypes
    from paper_2010_14823_amd import casim
    casim.init()
    hs = casim.HostState()
    assert casim.lib().casim_step_host(ctypes.byref(hs), 8, 3, 2.0, 0, None) == -1   # NULL fields
    assert casim.lib().casim_step_host(None, 8, 3, 2.0, 0, None) == -1
    p = ctypes.c_void_p()
    assert casim.lib().casim_host_alloc(None, 8) == -1
    assert casim.lib().casim_host_alloc(ctypes.byref(p), 64) == 0 and p.value
    assert casim.lib().casim_host_free(p) == 0


def test_rejected_call_enqueues_nothing():
    """A request casim_step would reject (more carry slots than the sweep
    holds: 512 thin levels at dt = 2 s) fails before any copy is enqueued:
    the host outputs keep their values."""
    import torch
    from paper_2010_14823_amd import casim
    cfg = synth.Config("levels512", 8, 8, 512, 7, 0.5)
    f, dz, _ = synth.generate(cfg)
    st = synth.stack(f)
    casim.init()
    hin, hout, hsfc = casim.HostArray(st.shape), casim.HostArray((12, 512, 64)), casim.HostArray((8, 64))
    hin.array[:] = st
    hout.array[:] = -7.0
    hsfc.array[:] = -7.0
    with pytest.raises(casim.CasimError) as e:
        casim.step_host(hin.array, dz, 2.0, hout.array, hsfc.array)
    assert e.value.code == -3
    torch.cuda.synchronize()
    assert np.all(hout.array == -7.0) and np.all(hsfc.array == -7.0)
    for h in (hin, hout, hsfc):
        h.free()
