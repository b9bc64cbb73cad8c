"""Front and back end of the process-rate surrogate -- TEST INFRASTRUCTURE.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
may import this module; the product never does and shares no code with it.
Plain numpy, float64 unless a step is defined in another precision.

The learned surrogate replaces the 12 process rates of the plain step (the
rate block of the scheme whose processes the paper lists in Sec. II) by a
network's output.  Around the network (oracle/mlp.py) this module defines:

* the 12 input features of a post-adjustment point: ln T, ln p, ln rho,
  ln(q + 1e-12) for vapour and cloud, ln(n + 1) for cloud number, then the
  (mass, number) pairs of rain and ice, then the masses of snow and graupel;
* the gate word: bit j set when rate j's condition holds (its categories
  present, its temperature side, and for rain evaporation no cloud and
  subsaturation over liquid), bit 12 when the point is supersaturated over
  ice with ice or snow present below 0 C;
* the training statistics: feature means and population standard deviations
  (floored at 1e-6), feature minima and maxima, means and population standard
  deviations (floored at 1e-3; 0 and 1 when a rate never occurs) of the scaled
  targets asinh(rate / 1e-12) over open gates (for the two deposition rates
  the magnitude's: their sign is the gate word's, so the network learns only
  how large they are), the covariance C of the
  features standardised with those (float32) statistics (divisor n - 1), the
  squared Mahalanobis distance z^T (C + 1e-9 I)^-1 z, and its 99.9th
  percentile, taken as the ceil(0.999 n)-th smallest value.  The statistics
  also carry the whitening factor W = L^-1 of the Cholesky factorisation
  L L^T = C + 1e-9 I, with which the distance is |W z|^2 (the form a float32
  evaluation needs: ln rho, ln p and ln T are nearly dependent, so C is close
  to singular and z^T C^-1 z would cancel);
* the trust region: a point falls back to the plain rates when a standardised
  feature lies outside the standardised training range widened by the margin
  on each side, or its squared Mahalanobis distance exceeds the limit;
* the de-transform: rate = 1e-12 sinh(y * y_std + y_mean); closed gates give
  0; deposition onto ice and snow (rates 3, 4) takes the sign of the ice
  supersaturation (bit 12), every other rate is clipped at 0.

Readings where the step's definition leaves freedom are stated at each
function; the range check is taken on the standardised feature so that the
network input and the check see the same number.
"""
from __future__ import annotations

import math

import numpy as np

from . import mlp

Q_FLOOR = 1e-12
RATE_SCALE = 1e-12
GATE_SUPERSAT_ICE = 1 << 12
T0, Q_MIN, Q_I0 = 273.15, 1e-12, 1e-4
AUTO, ACCR, REVP, DEPI, DEPS, IAUT, SACI, SACW, GACW, FRZR, SMLT, GMLT = range(12)


def features(state12, p, rho):
    """(n, 12) float64 features of post-adjustment states.

    state12: (n, 12) in the order T, qv, qc, nc, qr, nr, qi, ni, qs, ns, qg, ng
    (what the oracle's point processing returns); p, rho: (n,)."""
    s = np.atleast_2d(np.asarray(state12, dtype=np.float64))
    T, qv, qc, nc, qr, nr, qi, ni, qs, ns, qg, ng = s.T
    cols = [np.log(T), np.log(p), np.log(rho), np.log(qv + Q_FLOOR), np.log(qc + Q_FLOOR), np.log(nc + 1.0),
            np.log(qr + Q_FLOOR), np.log(nr + 1.0), np.log(qi + Q_FLOOR), np.log(ni + 1.0),
            np.log(qs + Q_FLOOR), np.log(qg + Q_FLOOR)]
    return np.stack([np.broadcast_to(c, T.shape) for c in cols], axis=-1)


def gate_word(state12, p, qsat_liquid, qsat_ice, warm=False):
    """uint16 gate words of post-adjustment states.  qsat_liquid, qsat_ice:
    callables (T, p) -> saturation mixing ratio."""
    s = np.atleast_2d(np.asarray(state12, dtype=np.float64))
    T, qv, qc, nc, qr, nr, qi, ni, qs, ns, qg, ng = s.T
    p = np.broadcast_to(np.asarray(p, dtype=np.float64), T.shape)
    cP, rP = qc >= Q_MIN, qr >= Q_MIN
    iP = (qi >= Q_MIN) & (not warm)
    sP = (qs >= Q_MIN) & (not warm)
    gP = (qg >= Q_MIN) & (not warm)
    cold = (T < T0) & (not warm)
    hot = (T > T0) & (not warm)
    qsl = np.array([qsat_liquid(a, b) for a, b in zip(T, p)])
    qsi = np.array([qsat_ice(a, b) for a, b in zip(T, p)])
    bits = [cP & (nc > 0), cP & rP, rP & (qc == 0.0) & (qv < qsl), iP & cold, sP & cold,
            iP & cold & (qi > Q_I0), sP & iP & cold, sP & cP & cold, gP & cP & cold, rP & cold,
            sP & hot, gP & hot]
    g = np.zeros(T.shape, dtype=np.uint32)
    for j, b in enumerate(bits):
        g |= b.astype(np.uint32) << j
    g |= ((cold & (iP | sP) & (qv > qsi)).astype(np.uint32)) << 12
    return g.astype(np.uint16)


def scaled_targets(rates):
    """Training targets asinh(rate / 1e-12); for deposition onto ice and snow
    (rates 3, 4) of the magnitude, whose sign the gate word carries."""
    r = np.array(rates, dtype=np.float64)
    r[..., DEPI] = np.abs(r[..., DEPI])
    r[..., DEPS] = np.abs(r[..., DEPS])
    return np.arcsinh(r / RATE_SCALE)


def fit_stats(feat, rates, gates):
    """Training statistics (dict of float32 arrays, plus q999) of n samples."""
    x = np.asarray(feat, dtype=np.float64)
    n = x.shape[0]
    mean = x.mean(axis=0)
    std = np.maximum(np.sqrt(((x - mean) ** 2).mean(axis=0)), 1e-6)
    st = {"x_mean": mean.astype(np.float32), "x_std": std.astype(np.float32),
          "x_min": x.min(axis=0).astype(np.float32), "x_max": x.max(axis=0).astype(np.float32)}
    t = scaled_targets(rates)
    g = np.asarray(gates).astype(np.uint32)
    ym, ys = np.zeros(12), np.ones(12)
    for j in range(12):
        sel = ((g >> j) & 1) == 1
        if sel.any():
            v = t[sel, j]
            ym[j] = v.mean()
            ys[j] = max(math.sqrt(((v - ym[j]) ** 2).mean()), 1e-3)
    st["y_mean"], st["y_std"] = ym.astype(np.float32), ys.astype(np.float32)
    z = standardise(x, st)
    cov = z.T @ z / max(n - 1, 1)
    st["cov"] = cov
    st["cov_inv"] = np.linalg.inv(cov + 1e-9 * np.eye(12))
    # W = L^-1 is lower triangular like L; np.tril keeps its zeros exact
    st["whiten"] = np.tril(np.linalg.inv(np.linalg.cholesky(cov + 1e-9 * np.eye(12))))
    d2 = maha2(z, st["cov_inv"])
    k = int(math.ceil(0.999 * n))
    st["maha_q999"] = float(np.sort(d2)[k - 1])
    return st


def standardise(feat, st):
    return (np.asarray(feat, dtype=np.float64) - st["x_mean"].astype(np.float64)) / st["x_std"].astype(np.float64)


def maha2(z, cov_inv):
    z = np.atleast_2d(z)
    return np.einsum("ni,ij,nj->n", z, np.asarray(cov_inv, dtype=np.float64), z)


def maha2_whitened(z, whiten):
    w = np.atleast_2d(z) @ np.asarray(whiten, dtype=np.float64).T
    return (w * w).sum(axis=1)


def out_of_range(z, st, margin):
    """Standardised features outside the standardised training range widened
    by margin * (max - min) on each side."""
    lo = st["x_min"].astype(np.float64) - margin * (st["x_max"].astype(np.float64) - st["x_min"].astype(np.float64))
    hi = st["x_max"].astype(np.float64) + margin * (st["x_max"].astype(np.float64) - st["x_min"].astype(np.float64))
    zlo, zhi = standardise(lo, st), standardise(hi, st)
    return ((z < zlo) | (z > zhi)).any(axis=1)


def fallback(z, st, margin, maha_limit):
    """True where the point leaves the trust region (distance from the
    whitening factor the statistics hold)."""
    return out_of_range(z, st, margin) | ~(maha2_whitened(z, st["whiten"]) <= maha_limit)


def detransform(y_std_units, st, gates):
    """Rates (n, 12) from standardised network outputs with the gate and sign rules."""
    y = np.asarray(y_std_units, dtype=np.float64) * st["y_std"].astype(np.float64) + st["y_mean"].astype(np.float64)
    r = RATE_SCALE * np.sinh(y)
    g = np.asarray(gates).astype(np.uint32)
    sup = (g & GATE_SUPERSAT_ICE) != 0
    out = np.empty_like(r)
    for j in range(12):
        if j in (DEPI, DEPS):
            v = np.where(sup, np.abs(r[:, j]), -np.abs(r[:, j]))
        else:
            v = np.maximum(r[:, j], 0.0)
        out[:, j] = np.where((g >> j) & 1, v, 0.0)
    return out


def limiter_min_f(state12, rates, dt):
    """Smallest limiter factor min_x min(1, q_x / (R_x dt)) over the source
    categories (vapour, cloud, rain, ice, snow, graupel) of the rates, with
    signed deposition drawing from vapour when positive and from the
    condensate when negative."""
    s = np.atleast_2d(np.asarray(state12, dtype=np.float64))
    r = np.atleast_2d(np.asarray(rates, dtype=np.float64))
    dep_v = np.maximum(r[:, DEPI], 0) + np.maximum(r[:, DEPS], 0)
    R = np.stack([dep_v, r[:, AUTO] + r[:, ACCR] + r[:, SACW] + r[:, GACW], r[:, REVP] + r[:, FRZR],
                  r[:, IAUT] + r[:, SACI] + np.maximum(-r[:, DEPI], 0), r[:, SMLT] + np.maximum(-r[:, DEPS], 0),
                  r[:, GMLT]], axis=1)
    q = s[:, [1, 2, 4, 6, 8, 10]]
    f = np.ones(len(s))
    for c in range(6):
        lim = R[:, c] * dt > q[:, c]
        with np.errstate(divide="ignore", invalid="ignore"):
            fc = np.where(lim, q[:, c] / (R[:, c] * dt), 1.0)
        f = np.minimum(f, fc)
    return f


def bf16_weights(theta):
    """The inference weight set: every weight rounded to bfloat16, biases kept
    in float32."""
    out = []
    for W, b in mlp.unpack(np.asarray(theta, dtype=np.float64)):
        out.append((mlp.bf16_round(W.astype(np.float32)), b.astype(np.float32)))
    return out


def infer(theta, st, feat, gates, margin, maha_limit):
    """Surrogate rates (n, 12) and fallback flags (n,) of float32 features:
    standardise, bfloat16 network with float32 accumulation
    (mlp.forward_bf16), de-transform with gates and signs, trust region."""
    z = standardise(feat, st)
    y = mlp.forward_bf16(theta, z.astype(np.float32))
    return detransform(y, st, gates), fallback(z, st, margin, maha_limit)
