"""Seeded synthetic column generator for the bulk-microphysics step.

This module is shared by the CPU oracle's tests and by the GPU path's tests
and benchmark.  It holds none of the microphysics: its saturation formula
(Tetens 1930 over liquid, Murray 1967 over ice) is a generator-only
convention for turning a drawn relative humidity into a vapour mixing ratio,
deliberately different from the Bolton/Buck formulas the step itself uses.

Shapes and distributions follow the synthetic stand-in for the paper's MONC
stratus test case (Sec. III-C runs 60-level columns; columns are independent,
Sec. II):

* interfaces z_{k+1/2} = 20 km * ((k+1)/nlev)**1.5 (stretched 0-20 km), k=0 at
  the surface;
* T = 300 K - 6.5 K/km up to 12 km, isothermal 222 K above;
* p dry-hydrostatic from 1000 hPa, rho = p / (R_d T);
* relative humidity: AR(1) Gaussian in k (lag-1 correlation 0.9) mapped
  through the normal CDF onto U(0.6, 1.05);
* cloud liquid q_c = 3e-4 * exp(0.8 N) kg/kg where RH > 0.98, n_c = 1e8 /kg;
  rain q_r = 1e-4 * exp(0.8 N) below the lowest cloud level, n_r = 1e4 /kg;
  ice, snow, graupel each 5e-5 * exp(0.8 N) where T < 0 C at or below the
  highest cloud level, numbers 1e5 /kg;
* a clustered cloud mask (periodic Gaussian filter, sigma = 8 columns, of
  white noise, thresholded to exactly round(f * ncol) cloudy columns);
* clear columns hold vapour at 0.3-0.9 of the lesser of liquid and ice
  saturation and no condensate;
* the "deep" variant sets RH ~ U(0.99, 1.02) i.i.d. between 1 and 14 km in
  cloudy columns and half of ice saturation above 14 km.

Every random draw for grid row ``y`` (``nx`` columns) comes from its own
stream, ``SeedSequence([seed, 1, y])``, so any subset of rows is reproduced
exactly without generating the whole domain.  The cloud mask uses
``SeedSequence([seed, 0])``.

Arrays are returned in the library's layout: one array per field of shape
``(nlev, ncol)`` (column index fastest), column index ``c = x + nx * y``.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

FIELDS = ("T", "p", "rho", "qv", "qc", "nc", "qr", "nr",
          "qi", "ni", "qs", "ns", "qg", "ng")

# generator-only physical constants
_RD = 287.04            # J/kg/K, dry air (for hydrostatic p and rho)
_G = 9.80665            # m/s^2
_EPS = 287.04 / 461.5   # R_d / R_v
_T0 = 273.15


@dataclasses.dataclass(frozen=True)
class Config:
    name: str
    nx: int
    ny: int
    nlev: int
    seed: int
    cloud_frac: float | None     # None: every column cloudy (no mask)
    deep: bool = False
    dt: float = 2.0

    @property
    def ncol(self) -> int:
        return self.nx * self.ny

    @property
    def points(self) -> int:
        return self.ncol * self.nlev


# The five workloads: small parity case, LES-like domain, sparse deep
# convection, the mixed-precision case and the surrogate inference case.
CONFIGS = {
    "c0": Config("c0_8x8x60", 8, 8, 60, 0, None),
    "c1": Config("c1_256x256x100", 256, 256, 100, 1, 0.5),
    "c2": Config("c2_1024x1024x120_deep10", 1024, 1024, 120, 2, 0.1, deep=True),
    "c3": Config("c3_1024x1024x120", 1024, 1024, 120, 3, 0.5),
    "c4": Config("c4_1024x1024x120", 1024, 1024, 120, 4, 0.5),
}


def tetens_es_liquid(T):
    """Generator-only liquid saturation pressure (Tetens 1930), Pa."""
    Tc = T - _T0
    return 610.78 * np.exp(17.27 * Tc / (Tc + 237.3))


def murray_es_ice(T):
    """Generator-only ice saturation pressure (Murray 1967), Pa."""
    Tc = T - _T0
    return 610.78 * np.exp(21.875 * Tc / (Tc + 265.5))


def _q_from_e(e, p):
    return _EPS * e / (p - (1.0 - _EPS) * e)


def vertical_grid(nlev: int):
    """Layer thicknesses dz (nlev,) and mid-level heights z (nlev,), metres."""
    zi = 20000.0 * (np.arange(1, nlev + 1, dtype=np.float64) / nlev) ** 1.5
    zlo = np.concatenate(([0.0], zi[:-1]))
    return zi - zlo, 0.5 * (zi + zlo)


def reference_profile(nlev: int):
    """T, p, rho (each (nlev,)) of the fixed background atmosphere."""
    _, z = vertical_grid(nlev)
    gamma = 6.5e-3
    T = np.where(z <= 12000.0, 300.0 - gamma * z, 222.0)
    p12 = 1.0e5 * (222.0 / 300.0) ** (_G / (_RD * gamma))
    p = np.where(z <= 12000.0,
                 1.0e5 * (T / 300.0) ** (_G / (_RD * gamma)),
                 p12 * np.exp(-_G * (z - 12000.0) / (_RD * 222.0)))
    rho = p / (_RD * T)
    return T, p, rho


def cloud_mask(cfg: Config) -> np.ndarray:
    """Boolean (ncol,) cloudy-column mask, exactly round(f*ncol) True."""
    if cfg.cloud_frac is None:
        return np.ones(cfg.ncol, dtype=bool)
    rng = np.random.default_rng(np.random.SeedSequence([cfg.seed, 0]))
    noise = rng.standard_normal((cfg.ny, cfg.nx))
    # periodic Gaussian filter, sigma = 8 columns, via FFT
    sigma = 8.0
    kx = np.fft.fftfreq(cfg.nx)
    ky = np.fft.fftfreq(cfg.ny)
    filt = np.exp(-2.0 * (math.pi * sigma) ** 2 * (ky[:, None] ** 2 + kx[None, :] ** 2))
    smooth = np.real(np.fft.ifft2(np.fft.fft2(noise) * filt)).ravel()
    ncloud = int(round(cfg.cloud_frac * cfg.ncol))
    mask = np.zeros(cfg.ncol, dtype=bool)
    if ncloud > 0:
        order = np.argsort(-smooth, kind="stable")
        mask[order[:ncloud]] = True
    return mask


def _ndtr(x):
    from scipy.special import ndtr
    return ndtr(x)


def _rows(cfg: Config, rows, mask):
    """Generate the fields of grid rows ``rows``; returns dict of (nlev, len(rows)*nx)."""
    nlev, nx = cfg.nlev, cfg.nx
    _, z = vertical_grid(nlev)
    T0p, p0p, rho0p = reference_profile(nlev)
    ncols = len(rows) * nx
    out = {f: np.zeros((nlev, ncols), dtype=np.float64) for f in FIELDS}
    esl = tetens_es_liquid(T0p)
    esi = murray_es_ice(T0p)
    qsl = _q_from_e(esl, p0p)
    qsi = _q_from_e(esi, p0p)
    qs_min = np.where(T0p < _T0, np.minimum(qsl, qsi), qsl)
    below0 = T0p < _T0
    for j, y in enumerate(rows):
        sl = slice(j * nx, (j + 1) * nx)
        rng = np.random.default_rng(np.random.SeedSequence([cfg.seed, 1, int(y)]))
        white = rng.standard_normal((nlev, nx))
        nc_ = rng.standard_normal((nlev, nx))
        nr_ = rng.standard_normal((nlev, nx))
        ni_ = rng.standard_normal((nlev, nx))
        ns_ = rng.standard_normal((nlev, nx))
        ng_ = rng.standard_normal((nlev, nx))
        ar = np.empty_like(white)
        ar[0] = white[0]
        a, b = 0.9, math.sqrt(1.0 - 0.81)
        for k in range(1, nlev):
            ar[k] = a * ar[k - 1] + b * white[k]
        u = _ndtr(ar)
        cloudy = mask[j * nx:(j + 1) * nx]
        rh = 0.6 + 0.45 * u
        if cfg.deep:
            ud = _ndtr(white)
            band = (z >= 1000.0) & (z <= 14000.0)
            rh = np.where(band[:, None], 0.99 + 0.03 * ud, rh)
        # a cloudy column without any RH > 0.98 level is saturated at its max-RH level
        has = (rh > 0.98).any(axis=0)
        fix = cloudy & ~has
        if fix.any():
            kmax = np.argmax(rh, axis=0)
            cols = np.nonzero(fix)[0]
            rh[kmax[cols], cols] = 1.0
        qv = rh * qsl[:, None]
        if cfg.deep:
            top = z > 14000.0
            qv = np.where(top[:, None], 0.5 * qsi[:, None], qv)
        incloud = (rh > 0.98) & cloudy[None, :]
        if cfg.deep:
            incloud &= ~(z > 14000.0)[:, None]
        anycl = incloud.any(axis=0)
        kidx = np.arange(nlev)[:, None]
        lowest = np.where(anycl, np.argmax(incloud, axis=0), -1)
        highest = np.where(anycl, nlev - 1 - np.argmax(incloud[::-1], axis=0), -1)
        qc = np.where(incloud, 3e-4 * np.exp(0.8 * nc_), 0.0)
        ncn = np.where(incloud, 1e8, 0.0)
        rain = anycl[None, :] & (kidx < lowest[None, :])
        qr = np.where(rain, 1e-4 * np.exp(0.8 * nr_), 0.0)
        nrn = np.where(rain, 1e4, 0.0)
        icy = anycl[None, :] & (kidx <= highest[None, :]) & below0[:, None]
        qi = np.where(icy, 5e-5 * np.exp(0.8 * ni_), 0.0)
        qs = np.where(icy, 5e-5 * np.exp(0.8 * ns_), 0.0)
        qg = np.where(icy, 5e-5 * np.exp(0.8 * ng_), 0.0)
        nin = np.where(icy, 1e5, 0.0)
        # clear columns: subsaturated vapour only
        qclear = (0.3 + 0.6 * u) * qs_min[:, None]
        qv = np.where(cloudy[None, :], qv, qclear)
        out["T"][:, sl] = T0p[:, None]
        out["p"][:, sl] = p0p[:, None]
        out["rho"][:, sl] = rho0p[:, None]
        out["qv"][:, sl] = qv
        out["qc"][:, sl] = qc
        out["nc"][:, sl] = ncn
        out["qr"][:, sl] = qr
        out["nr"][:, sl] = nrn
        out["qi"][:, sl] = qi
        out["ni"][:, sl] = nin
        out["qs"][:, sl] = qs
        out["ns"][:, sl] = nin
        out["qg"][:, sl] = qg
        out["ng"][:, sl] = nin
    return out


def generate(cfg: Config, rows=None, mask=None):
    """Synthetic state for ``cfg`` (all rows, or the listed grid rows).

    Returns ``(fields, dz, cols)``: ``fields`` maps each name in ``FIELDS`` to a
    float64 array of shape (nlev, ncols); ``dz`` is (nlev,); ``cols`` holds the
    global column indices of the generated columns.  ``mask`` may pass
    ``cloud_mask(cfg)`` in when it is already known.
    """
    if rows is None:
        rows = range(cfg.ny)
    rows = list(rows)
    mask_all = cloud_mask(cfg) if mask is None else mask
    sub = np.concatenate([mask_all[y * cfg.nx:(y + 1) * cfg.nx] for y in rows]) if rows else np.zeros(0, bool)
    fields = _rows(cfg, rows, sub)
    dz, _ = vertical_grid(cfg.nlev)
    cols = np.concatenate([np.arange(y * cfg.nx, (y + 1) * cfg.nx) for y in rows]) if rows else np.zeros(0, np.int64)
    return fields, dz, cols


def stack(fields) -> np.ndarray:
    """(14, nlev, ncol) contiguous array in FIELDS order."""
    return np.ascontiguousarray(np.stack([fields[f] for f in FIELDS]))


def generate_stacked(cfg: Config, workers: int = 8, rows_per_task: int = 16):
    """The whole (14, nlev, ncol) state of ``cfg`` in FIELDS order, filled by
    ``workers`` threads over blocks of grid rows (bitwise what
    ``stack(generate(cfg)[0])`` returns: every row draws from its own
    stream).  Returns ``(state, dz)``."""
    import concurrent.futures as cf
    mask = cloud_mask(cfg)
    out = np.empty((len(FIELDS), cfg.nlev, cfg.ncol), dtype=np.float64)

    def task(y0):
        rows = range(y0, min(cfg.ny, y0 + rows_per_task))
        f, _, cols = generate(cfg, rows, mask=mask)
        c0, c1 = cols[0], cols[-1] + 1
        for j, name in enumerate(FIELDS):
            out[j, :, c0:c1] = f[name]
        return None

    with cf.ThreadPoolExecutor(max_workers=max(1, workers)) as ex:
        list(ex.map(task, range(0, cfg.ny, rows_per_task)))
    dz, _ = vertical_grid(cfg.nlev)
    return out, dz
