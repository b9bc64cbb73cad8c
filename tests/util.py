"""Shared helpers of the test-suite: run the GPU path and the oracle on the
same seeded inputs and compare them field by field."""
import numpy as np

from paper_2010_14823_amd import synth

TEND = ("dT", "dqv", "dqc", "dnc", "dqr", "dnr", "dqi", "dni", "dqs", "dns", "dqg", "dng")
SFC = ("Pr", "Pi", "Ps", "Pg", "Nr", "Ni", "Ns", "Ng")


def normwise(g, o):
    """max |g - o| / max |o| (0 when both are identically zero)."""
    g = np.asarray(g); o = np.asarray(o)
    den = np.max(np.abs(o)) if o.size else 0.0
    num = np.max(np.abs(g - o)) if o.size else 0.0
    if den == 0.0:
        return 0.0 if num == 0.0 else np.inf
    return num / den


def field_errors(tg, sg, to, so):
    errs = {}
    for j, n in enumerate(TEND):
        errs[n] = normwise(tg[j], to[j])
    for j, n in enumerate(SFC):
        errs[n] = normwise(sg[j], so[j])
    return errs


def config_state(key, rows=None):
    cfg = synth.CONFIGS[key]
    f, dz, cols = synth.generate(cfg, rows)
    return cfg, synth.stack(f), dz, cols


def run_gpu(state_np, dz, dt, *, ncol=None, ld=None, mode=0, stages=15, warm=0,
            newton_iters=5, pad_value=np.nan, steps=1, constants=None):
    """Upload, run ``steps`` casim steps (applying tendencies between them) and
    return (tend, sfc, status) as numpy arrays over the first ncol columns."""
    import torch
    from paper_2010_14823_amd import casim
    nf, nlev, n = state_np.shape
    ncol = n if ncol is None else ncol
    ld = ncol if ld is None else ld
    host = np.full((nf, nlev, ld), pad_value)
    host[:, :, :ncol] = state_np[:, :, :ncol]
    dev = torch.from_numpy(host).cuda()
    tend = torch.full((12, nlev, ld), -7.0, dtype=torch.float64, device="cuda")
    sfc = torch.full((8, ld), -7.0, dtype=torch.float64, device="cuda")
    c = constants if constants is not None else casim.default_constants(mode=mode, stages=stages, warm=warm)
    t = casim.default_thresholds(newton_iters=newton_iters)
    casim.init(c, t)
    casim.status()
    for s in range(steps):
        casim.step(dev, dz, dt, tend, sfc, ncol=ncol)
        if s + 1 < steps:
            casim.apply_tendencies(dev, dz, dt, tend, sfc, ncol=ncol)
    st = casim.status()
    torch.cuda.synchronize()
    out_t = tend.cpu().numpy()
    out_s = sfc.cpu().numpy()
    return out_t, out_s, st, dev.cpu().numpy()


def oracle_steps(oracle, state_np, dz, dt, steps=1, **kw):
    """The oracle's multi-step run with the same parent-model update
    (X += dt * tend, q and n clipped at 0)."""
    st = state_np.copy()
    for s in range(steps):
        tend, sfc = oracle.step(st, dz, dt, **kw)
        if s + 1 < steps:
            st[0] = st[0] + dt * tend[0]
            for f in range(1, 12):
                v = st[f + 2] + dt * tend[f]
                st[f + 2] = np.where(v > 0.0, v, 0.0)
    return tend, sfc


def oracle_ulp_floor(oracle, state_np, dz, dt, steps, seed=0, **kw):
    """How far the oracle's own multi-step answer moves when every state it
    steps from is perturbed by one unit in the last place (relative 2^-52,
    random sign, T and the 12 prognostic fields): per tendency/surface field
    the normwise change of the last step's outputs, and per state field the
    change of the state after steps - 1 updates.  Two correct binary64
    implementations that round differently differ by about this much: near
    saturation the adjustment's increment is a small difference of q_v and
    q_sat, so after a few coupled steps a one-ulp change of q_v moves the
    tendencies by far more than one ulp of their own size."""
    rng = np.random.default_rng(seed)

    def run(perturb):
        st = state_np.copy()
        for s in range(steps):
            if perturb:
                for f in [0] + list(range(3, 14)):
                    st[f] = st[f] * (1.0 + rng.choice([-1.0, 1.0], size=st[f].shape) * 2.0 ** -52)
            tend, sfc = oracle.step(st, dz, dt, **kw)
            if s + 1 < steps:
                st[0] = st[0] + dt * tend[0]
                for f in range(1, 12):
                    v = st[f + 2] + dt * tend[f]
                    st[f + 2] = np.where(v > 0.0, v, 0.0)
        return tend, sfc, st
    t0, s0, x0 = run(False)
    t1, s1, x1 = run(True)
    errs = field_errors(t1, s1, t0, s0)
    idx = [0] + list(range(3, 14))
    state_errs = {f: normwise(x1[f], x0[f]) for f in idx}
    return errs, state_errs
