"""The allocation-free step (casim_step_noalloc) against casim_step, through
the C ABI: bitwise the same tendencies and surface sums on two calls in a
row, the second on a smaller domain, then again on that domain (launch
order from the activity record in the static scratch), in both binary64 and
FP32-mixed modes; binary64 also against the oracle; its counters reach
casim_status; modes it does not serve and domains beyond its tile limit are
rejected before anything is enqueued."""
import numpy as np
import pytest

from paper_2010_14823_amd import synth
from util import config_state, field_errors

pytestmark = pytest.mark.gpu


def _run(casim, fn, dev, dz, dt, ncol=None):
    import torch
    nlev, ld = dev.shape[1], dev.shape[2]
    tend = torch.full((12, nlev, ld), -7.0, dtype=torch.float64, device="cuda")
    sfc = torch.full((8, ld), -7.0, dtype=torch.float64, device="cuda")
    fn(dev, dz, dt, tend, sfc, ncol=ncol)
    torch.cuda.synchronize()
    return tend.cpu().numpy(), sfc.cpu().numpy()


@pytest.mark.parametrize("mode", [0, 1])
def test_noalloc_matches_step(oracle_lib, mode):
    import torch
    from paper_2010_14823_amd import casim
    big_cfg, big, dz_b, _ = config_state("c1", rows=list(range(0, 256, 2)))      # 32,768 columns x 100
    small_cfg, small, dz_s, _ = config_state("c0")                               # 64 columns x 60
    casim.init(casim.default_constants(mode=mode))
    casim.status()
    for tag, st, dz, dt in (("large", big, dz_b, big_cfg.dt), ("small", small, dz_s, small_cfg.dt),
                            ("small again", small, dz_s, small_cfg.dt)):
        dev = torch.from_numpy(st).cuda()
        t_ref, s_ref = _run(casim, casim.step, dev, dz, dt)
        st_ref = casim.status()
        t_na, s_na = _run(casim, casim.step_noalloc, dev, dz, dt)
        st_na = casim.status()
        assert not np.any(t_na == -7.0) and not np.any(s_na == -7.0)
        assert np.array_equal(t_na, t_ref) and np.array_equal(s_na, s_ref), tag
        assert st_na == st_ref, (tag, st_na, st_ref)
        if mode == 0:
            to, so = oracle_lib.step(st, dz, dt)
            errs = field_errors(t_na, s_na, to, so)
            print(tag, "worst normwise error vs oracle %.3g" % max(errs.values()))
            assert max(errs.values()) <= 1e-12
        del dev


def test_noalloc_rejections():
    import torch
    from paper_2010_14823_amd import casim
    cfg, st, dz, _ = config_state("c0")
    dev = torch.from_numpy(st).cuda()
    tend = torch.full((12,) + st.shape[1:], -7.0, dtype=torch.float64, device="cuda")
    sfc = torch.full((8, st.shape[2]), -7.0, dtype=torch.float64, device="cuda")
    casim.init(casim.default_constants(mode=casim.MODE_FP64_COMPACT))
    with pytest.raises(casim.CasimError) as e:
        casim.step_noalloc(dev, dz, cfg.dt, tend, sfc)
    assert e.value.code == -1
    # beyond the tile limit: 262,145 tiles of 16 columns, one level
    casim.init()
    ncol = 16 * (1 << 18) + 16
    big = torch.zeros((14, 1, ncol), dtype=torch.float64, device="cuda")
    big[0].fill_(280.0); big[1].fill_(9e4); big[2].fill_(1.1)
    bt = torch.full((12, 1, ncol), -7.0, dtype=torch.float64, device="cuda")
    bs = torch.full((8, ncol), -7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(casim.CasimError) as e:
        casim.step_noalloc(big, [100.0], 2.0, bt, bs)
    assert e.value.code == -3
    torch.cuda.synchronize()
    assert bool((bt == -7.0).all()) and bool((tend == -7.0).all())
    # at the limit it runs (262,144 tiles)
    n2 = 16 * (1 << 18)
    casim.step_noalloc(big, [100.0], 2.0, bt, bs, ncol=n2)
    torch.cuda.synchronize()
    assert bool((bt[:, :, :n2] == 0.0).all()) and bool((bt[:, :, n2:] == -7.0).all())
