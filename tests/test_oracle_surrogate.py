"""Pins of the surrogate's front and back end in the oracle (oracle/surrogate.py)
against facts that do not come from that module: the plain oracle's own
rate conditions, closed forms of the statistics on designed data, the
library's order statistic, exact round trips and the limiter's effect in the
oracle's step."""
import math

import numpy as np
import pytest

from oracle import surrogate as osur
from paper_2010_14823_amd import synth


def _c0_points(oracle_lib):
    f, dz, _ = synth.generate(synth.CONFIGS["c0"])
    st = synth.stack(f)
    return st.transpose(1, 2, 0).reshape(-1, 14)


def _random_states(oracle_lib, n=3000, seed=0):
    """Point inputs spread over both temperature sides, sub- and supersaturated,
    each category present, absent or just around the presence threshold."""
    rng = np.random.default_rng(seed)
    out = np.zeros((n, 14))
    T = rng.uniform(225.0, 295.0, n)
    p = rng.uniform(2e4, 1e5, n)
    out[:, 0], out[:, 1], out[:, 2] = T, p, p / (287.04 * T)
    qsl = np.array([oracle_lib.qsat_liquid(a, b) for a, b in zip(T, p)])
    out[:, 3] = qsl * rng.uniform(0.5, 1.06, n)
    for j, (q0, n0) in enumerate([(3e-4, 1e8), (1e-4, 1e4), (5e-5, 1e5), (5e-5, 1e5), (5e-5, 1e5)]):
        pick = rng.uniform(size=n)
        q = np.where(pick < 0.4, 0.0, q0 * np.exp(0.8 * rng.standard_normal(n)))
        q = np.where((pick > 0.9) & (pick < 0.95), rng.uniform(0.5e-12, 2e-12, n), q)
        out[:, 4 + 2 * j] = q
        out[:, 5 + 2 * j] = np.where(q > 0, n0, 0.0)
    return out


def test_gate_word_is_the_oracle_rate_pattern(oracle_lib):
    """Bit j is set exactly where the oracle's rate j is non-zero; bit 12
    exactly where deposition (onto ice or snow) is positive."""
    pts = np.concatenate([_c0_points(oracle_lib), _random_states(oracle_lib)])
    seen = np.zeros(13, dtype=int)
    for warm in (False, True):
        for x in pts:
            state, r = oracle_lib.point_process(x, warm=warm)
            g = int(osur.gate_word(state[None], x[1], oracle_lib.qsat_liquid, oracle_lib.qsat_ice, warm=warm)[0])
            for j in range(12):
                assert bool((g >> j) & 1) == (r[j] != 0.0), (x, j, r)
                seen[j] += (g >> j) & 1
            dep = max(r[3], r[4]) > 0
            assert bool(g & osur.GATE_SUPERSAT_ICE) == dep, (x, r)
            seen[12] += dep
    assert np.all(seen > 0), seen          # every bit occurs


def test_features_at_a_hand_point():
    state = np.array([[math.exp(5.5), 1e-3 - 1e-12, 0.0, math.exp(18.0) - 1.0, 2e-4 - 1e-12, 0.0,
                       5e-5 - 1e-12, math.exp(11.0) - 1.0, 0.0, 7.0, 3e-6 - 1e-12, 0.0]])
    f = osur.features(state, np.array([6e4]), np.array([0.75]))[0]
    # order: T p rho qv qc nc qr nr qi ni qs qg
    want = [5.5, math.log(6e4), math.log(0.75), math.log(1e-3), math.log(1e-12), 18.0,
            math.log(2e-4), 0.0, math.log(5e-5), 11.0, math.log(1e-12), math.log(3e-6)]
    assert np.allclose(f, want, rtol=0, atol=1e-12)


def _designed_features(n=2000, seed=3):
    """Features whose standardised covariance is exactly the identity:
    orthonormal columns (QR of a centred random matrix) scaled to unit
    population variance, then shifted and scaled per feature."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((n, 12))
    a -= a.mean(axis=0)
    q, _ = np.linalg.qr(a)
    z = q * math.sqrt(n)            # population variance 1, mean 0, orthogonal
    mean = rng.uniform(-10, 10, 12)
    std = rng.uniform(0.1, 5.0, 12)
    return z * std + mean, mean, std


def test_statistics_of_designed_data():
    x, mean, std = _designed_features()
    n = len(x)
    rates = np.zeros((n, 12))
    gates = np.zeros(n, dtype=np.uint16)
    # target 0: open on the first half, values whose asinh is +-1 alternating
    rates[: n // 2, 0] = 1e-12 * math.sinh(1.0) * np.where(np.arange(n // 2) % 2 == 0, 1.0, -1.0)
    gates[: n // 2] = 1
    st = osur.fit_stats(x.astype(np.float32), rates, gates)
    assert np.allclose(st["x_mean"], mean, rtol=0, atol=2e-5 * np.abs(mean).max())
    assert np.allclose(st["x_std"], std, rtol=1e-5)
    assert np.array_equal(st["x_min"], x.astype(np.float32).min(axis=0))
    assert st["y_mean"][0] == pytest.approx(0.0, abs=1e-7) and st["y_std"][0] == pytest.approx(1.0, rel=1e-7)
    assert np.all(st["y_mean"][1:] == 0.0) and np.all(st["y_std"][1:] == 1.0)     # never open: 0 and 1
    # the standardised covariance is the identity (up to the float32 stats),
    # with divisor n - 1
    assert np.allclose(st["cov"], np.eye(12) * n / (n - 1), atol=2e-5)
    assert np.allclose(st["cov_inv"] @ (st["cov"] + 1e-9 * np.eye(12)), np.eye(12), atol=1e-12)
    # the whitening factor is lower triangular and W^T W is the inverse
    assert np.all(np.triu(st["whiten"], 1) == 0.0)
    assert np.allclose(st["whiten"].T @ st["whiten"], st["cov_inv"], rtol=0, atol=1e-12)
    z = osur.standardise(x.astype(np.float32), st)
    d2 = osur.maha2(z, st["cov_inv"])
    assert np.allclose(d2, (z ** 2).sum(axis=1) * (n - 1) / n, rtol=1e-4)
    assert np.allclose(osur.maha2_whitened(z, st["whiten"]), d2, rtol=1e-12)
    # the mean has distance 0
    assert osur.maha2(np.zeros((1, 12)), st["cov_inv"])[0] == 0.0
    # the 99.9th percentile is the ceil(0.999 n)-th order statistic
    assert st["maha_q999"] == np.quantile(d2, 0.999, method="inverted_cdf")


def test_whitened_distance_with_dependent_features():
    """ln rho = ln p - ln T - ln R_d holds exactly in the inputs, so the
    covariance of (ln T, ln p, ln rho, ...) is singular but for the ridge; the
    whitened float32 distance stays close to the binary64 one, while the
    quadratic form with the inverse in float32 does not."""
    rng = np.random.default_rng(8)
    n = 5000
    T = rng.uniform(220, 300, n); p = rng.uniform(2e4, 1e5, n)
    x = np.column_stack([np.log(T), np.log(p), np.log(p / (287.04 * T))] +
                        [rng.standard_normal(n) for _ in range(9)]).astype(np.float32)
    st = osur.fit_stats(x, np.zeros((n, 12)), np.zeros(n, np.uint16))
    z = osur.standardise(x, st)
    exact = osur.maha2(z, st["cov_inv"])
    z32 = z.astype(np.float32)
    w32 = st["whiten"].astype(np.float32)
    via_w = ((z32 @ w32.T) ** 2).sum(axis=1, dtype=np.float32)
    ci32 = st["cov_inv"].astype(np.float32)
    via_inv = np.einsum("ni,ij,nj->n", z32, ci32, z32, dtype=np.float32)
    err_w = np.max(np.abs(via_w - exact) / exact)
    err_inv = np.max(np.abs(via_inv - exact) / exact)
    assert err_w < 1e-3 and err_inv > 100 * err_w, (err_w, err_inv)


def test_trust_region():
    x, mean, std = _designed_features(500)
    st = osur.fit_stats(x.astype(np.float32), np.zeros((500, 12)), np.zeros(500, np.uint16))
    z = osur.standardise(x.astype(np.float32), st)
    assert not osur.out_of_range(z, st, 0.0).any()                       # the training set is inside
    span = (st["x_max"] - st["x_min"]).astype(np.float64)
    for j in (0, 7, 11):
        for side, sign in (("x_max", 1.0), ("x_min", -1.0)):
            xo = x[:1].copy()
            xo[0, j] = st[side][j] + sign * 0.05 * span[j]
            zo = osur.standardise(xo, st)
            assert osur.out_of_range(zo, st, 0.0)[0] and osur.out_of_range(zo, st, 0.04)[0]
            assert not osur.out_of_range(zo, st, 0.06)[0]
    lim = st["maha_q999"]
    fb = osur.fallback(z, st, 0.1, lim)
    # at most the points above the 99.9th percentile (the percentile point
    # itself may land either side in the whitened form's rounding)
    assert fb.sum() == (osur.maha2_whitened(z, st["whiten"]) > lim).sum() <= math.ceil(0.001 * 500) + 1


def test_detransform_round_trip_gates_and_signs():
    rng = np.random.default_rng(4)
    n = 400
    rates = np.abs(rng.lognormal(-18, 3, (n, 12)))
    gates = rng.integers(0, 1 << 13, n).astype(np.uint16)
    sup = (gates & osur.GATE_SUPERSAT_ICE) != 0
    rates[:, 3] *= np.where(sup, 1.0, -1.0)
    rates[:, 4] *= np.where(sup, 1.0, -1.0)
    st = {"y_mean": np.float32(rng.uniform(-5, 5, 12)), "y_std": np.float32(rng.uniform(0.5, 8, 12))}
    y = (osur.scaled_targets(rates) - st["y_mean"]) / st["y_std"]
    back = osur.detransform(y, st, gates)
    open_ = ((gates[:, None] >> np.arange(12)) & 1) == 1
    assert np.allclose(back[open_], rates[open_], rtol=1e-12, atol=0)
    assert np.all(back[~open_] == 0.0)
    # signs: negative predictions of a non-deposition rate are clipped at 0,
    # deposition takes the sign of bit 12 whatever the network says
    neg = osur.detransform(-np.abs(y) - 3.0, {"y_mean": np.zeros(12, np.float32), "y_std": np.ones(12, np.float32)},
                           gates | 0xFFF)
    assert np.all(neg[:, [0, 1, 2, 5, 6, 7, 8, 9, 10, 11]] == 0.0)
    assert np.all(np.sign(neg[:, 3]) == np.where(sup, 1.0, -1.0))


def test_limiter_factor_matches_the_oracle_step(oracle_lib):
    """A single cloud sink that would remove more than the cloud present: the
    factor is q_c / (R dt), and the oracle's apply step then moves exactly
    q_c to rain."""
    x = np.array([285.0, 9e4, 1.1, 0.9 * oracle_lib.qsat_liquid(285.0, 9e4), 0.0, 0.0, 0, 0, 0, 0, 0, 0, 0, 0])
    x[4], x[5] = 2e-4, 1e8
    state, r = oracle_lib.point_process(x)
    assert state[2] == 0.0          # subsaturated: all cloud evaporated -- use a saturated point instead
    T, p = 285.0, 9e4
    x[3] = oracle_lib.qsat_liquid(T, p)
    state, r = oracle_lib.point_process(x)
    qc = state[2]
    assert qc > 0
    rates = np.zeros(12)
    dt = 2.0
    rates[0] = 3.0 * qc / dt                       # AUTO three times too large
    f = osur.limiter_min_f(state[None], rates[None], dt)[0]
    assert f == pytest.approx(1.0 / 3.0, rel=1e-15)
    tend = oracle_lib.point_apply(x, rates, dt)
    adj, _ = oracle_lib.point_process(x)
    assert adj[2] + dt * tend[2] - (state[2] - qc) == pytest.approx(0.0, abs=1e-20)
    # rain gains exactly the limited cloud: tend_qr * dt == qc
    assert tend[4] * dt == pytest.approx(qc, rel=1e-14)
    # below the limit f = 1
    rates[0] = 0.5 * qc / dt
    assert osur.limiter_min_f(state[None], rates[None], dt)[0] == 1.0
