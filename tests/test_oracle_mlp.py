"""Pins of the FP64 surrogate-network oracle: central finite differences,
the closed form of the first Adam step, SiLU facts and bfloat16 rounding of
known bit patterns."""
import numpy as np
import pytest

from oracle import mlp


def _problem(seed=0, n=7):
    rng = np.random.default_rng(seed)
    theta = rng.normal(0.0, 0.3, mlp.N_PARAMS)
    X = rng.normal(size=(n, 12))
    T = rng.normal(size=(n, 12))
    M = (rng.uniform(size=(n, 12)) < 0.7).astype(float)
    return theta, X, T, M


def test_parameter_count():
    assert mlp.N_PARAMS == 36236


def test_silu_facts():
    z = np.linspace(-20, 20, 2001)
    assert mlp.silu(np.array([0.0]))[0] == 0.0
    assert np.allclose(mlp.silu(z), z * (1.0 / (1.0 + np.exp(-z))), rtol=1e-15, atol=0)
    h = 1e-6
    fd = (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - mlp.dsilu(z))) < 1e-8
    assert mlp.dsilu(np.array([0.0]))[0] == 0.5


def test_gradient_matches_central_differences():
    theta, X, T, M = _problem()
    L, g = mlp.loss_and_grad(theta, X, T, M)
    assert L == pytest.approx(mlp.loss(theta, X, T, M), rel=1e-15)
    rng = np.random.default_rng(1)
    idx = np.concatenate([rng.choice(mlp.N_PARAMS, 60, replace=False),
                          [0, 1535, 1536 + 127, 36236 - 1, 36236 - 12, 1664, 34687]])
    h = 1e-4

    def at(i, d):
        t = theta.copy(); t[i] += d
        return mlp.loss(t, X, T, M)
    for i in idx:
        # fourth-order central difference: error O(h^4)
        fd = (8 * (at(i, h) - at(i, -h)) - (at(i, 2 * h) - at(i, -2 * h))) / (12 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1e-3, abs(g[i])) + 1e-11, (i, fd, g[i])


def test_masked_entries_do_not_contribute():
    theta, X, T, M = _problem(2)
    L, g = mlp.loss_and_grad(theta, X, T, M)
    T2 = T + (1 - M) * 1e3          # change only masked-out targets
    L2, g2 = mlp.loss_and_grad(theta, X, T2, M)
    assert L == L2 and np.array_equal(g, g2)
    y, _ = mlp.forward(theta, X)
    assert mlp.loss(theta, X, y, M) == 0.0


def test_first_adam_step_closed_form():
    rng = np.random.default_rng(4)
    theta = rng.normal(size=100)
    g = rng.normal(size=100)
    lr = 1e-3
    t1, m, v = mlp.adam(theta, g, np.zeros(100), np.zeros(100), 1, lr)
    # bias-corrected moments equal g and g^2, so the step is lr * g / (|g| + eps)
    assert np.allclose(t1, theta - lr * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_bf16_rounding_known_patterns():
    one = np.float32(1.0)
    ulp = np.float32(2.0 ** -7)             # bfloat16 spacing at 1
    vals = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -8 + 2.0 ** -20,
                     -2.5, 3.0e38, 1e-40], dtype=np.float32)
    r = mlp.bf16_round(vals)
    assert r[0] == one
    assert r[1] == one                        # tie -> even (1.0)
    assert r[2] == one + 2 * ulp              # tie -> even (1 + 2^-6)
    assert r[3] == one + ulp                  # above the tie rounds up
    assert r[4] == np.float32(-2.5)
    u = r.view(np.uint32)
    assert np.all(u & 0xFFFF == 0)


def test_bf16_forward_close_to_fp64():
    theta, X, _, _ = _problem(5, 50)
    y64, _ = mlp.forward(theta, X)
    yb = mlp.forward_bf16(theta, X)
    scale = np.max(np.abs(y64))
    assert np.max(np.abs(yb - y64)) < 0.05 * scale
