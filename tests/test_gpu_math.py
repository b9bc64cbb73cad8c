"""Accuracy of the binary64 exp and log the step kernels use, against the
host C library through numpy (both claim a few ulp at most)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_exp_log_accuracy():
    import torch
    from paper_2010_14823_amd import casim
    rng = np.random.default_rng(3)
    xe = np.concatenate([rng.uniform(-80, 80, 200000), rng.uniform(-1, 1, 100000),
                         [0.0, 1e-300, -700.0, 700.0, 0.5 * np.log(2), -0.5 * np.log(2)]])
    xl = np.concatenate([10 ** rng.uniform(-30, 12, 200000), rng.uniform(0.5, 2.0, 100000),
                         [1.0, 2.0, 0.5, 1e-300, 1e300, np.sqrt(0.5), np.sqrt(2.0)]])
    e, _ = casim.debug_math(torch.from_numpy(xe).cuda())
    _, l = casim.debug_math(torch.from_numpy(xl).cuda())
    torch.cuda.synchronize()
    e = e.cpu().numpy(); l = l.cpu().numpy()
    ref_e = np.exp(xe); ref_l = np.log(xl)
    rel_e = np.abs(e - ref_e) / ref_e
    # log near 1 is compared in absolute terms scaled by the argument's distance
    rel_l = np.abs(l - ref_l) / np.maximum(np.abs(ref_l), 1e-300)
    ulp = np.finfo(float).eps
    print("exp max rel err %.3g ulp, log max rel err %.3g ulp" % (rel_e.max() / ulp, rel_l[ref_l != 0].max() / ulp))
    assert rel_e.max() < 4 * ulp
    assert rel_l[ref_l != 0].max() < 4 * ulp
    assert l[xl == 1.0][0] == 0.0
    _, l0 = casim.debug_math(torch.zeros(3, dtype=torch.float64, device="cuda"))
    assert torch.all(torch.isinf(l0)) and torch.all(l0 < 0)
