"""CPU oracle of the bulk-microphysics column step -- TEST INFRASTRUCTURE.

This package is the plain FP64 definition the GPU path is checked against.
Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import it; the product (``paper_2010_14823_amd``) never does, and it shares
no code with it.  ``casim_oracle.c`` holds the step (built here with gcc,
``-O2 -fno-fast-math -ffp-contract=off -fopenmp``); ``mlp.py`` holds the FP64
multilayer-perceptron oracle for the learned rate surrogate.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "casim_oracle.c")
_LIB = os.environ.get("ORACLE_LIB_OVERRIDE") or os.path.join(_HERE, "liboracle.so")

ST_ADJUST, ST_SATADJ, ST_RATES, ST_SED, ST_ALL = 1, 2, 4, 8, 15
RATE_NAMES = ("AUTO", "ACCR", "REVP", "DEPI", "DEPS", "IAUT", "SACI",
              "SACW", "GACW", "FRZR", "SMLT", "GMLT")
TEND_NAMES = ("dT", "dqv", "dqc", "dnc", "dqr", "dnr", "dqi", "dni",
              "dqs", "dns", "dqg", "dng")
SFC_NAMES = ("Pr", "Pi", "Ps", "Pg", "Nr", "Ni", "Ns", "Ng")


def build(force: bool = True) -> str:
    """Compile liboracle.so from casim_oracle.c with gcc."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
               "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Opts(ctypes.Structure):
    _fields_ = [("stages", ctypes.c_int32), ("newton_iters", ctypes.c_int32),
                ("nthreads", ctypes.c_int32), ("warm", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        L.oracle_step.argtypes = [ctypes.POINTER(dp), dp, ctypes.c_int64, ctypes.c_int64,
                                  ctypes.c_int32, ctypes.c_double, ctypes.POINTER(dp),
                                  ctypes.POINTER(dp), ctypes.POINTER(_Opts),
                                  ctypes.POINTER(ctypes.c_int64)]
        L.oracle_step.restype = ctypes.c_int
        for name in ("oracle_esat_liquid", "oracle_esat_ice"):
            getattr(L, name).argtypes = [ctypes.c_double]
            getattr(L, name).restype = ctypes.c_double
        for name in ("oracle_qsat_liquid", "oracle_qsat_ice"):
            getattr(L, name).argtypes = [ctypes.c_double, ctypes.c_double]
            getattr(L, name).restype = ctypes.c_double
        L.oracle_point_rates.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                         dp, dp, ctypes.c_int32, dp]
        L.oracle_point_rates.restype = None
        L.oracle_saturation_adjust.argtypes = [dp, ctypes.c_double, dp, dp, dp, ctypes.c_int32]
        L.oracle_saturation_adjust.restype = ctypes.c_int
        L.oracle_nsub.argtypes = [dp, ctypes.c_int32, ctypes.c_double, ctypes.POINTER(ctypes.c_int32)]
        L.oracle_point_process.argtypes = [dp, ctypes.c_int32, ctypes.c_int32, dp, dp]
        L.oracle_point_process.restype = None
        L.oracle_nsub.restype = None
        L.oracle_point_apply.argtypes = [dp, dp, ctypes.c_double, ctypes.c_int32, ctypes.c_int32, dp]
        L.oracle_point_apply.restype = None
        _lib = L
    return _lib


def _dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def step(state: np.ndarray, dz: np.ndarray, dt: float, *, stages: int = ST_ALL,
         newton_iters: int = 5, nthreads: int = 0, warm: bool = False,
         return_fails: bool = False):
    """Run the oracle step.

    ``state``: float64 (14, nlev, ncol) in T, p, rho, qv, qc, nc, qr, nr, qi,
    ni, qs, ns, qg, ng order.  Returns ``(tend (12, nlev, ncol), sfc (8, ncol))``
    (plus the Newton-failure count if ``return_fails``).
    """
    state = np.ascontiguousarray(state, dtype=np.float64)
    dz = np.ascontiguousarray(dz, dtype=np.float64)
    _, nlev, ncol = state.shape
    tend = np.zeros((12, nlev, ncol))
    sfc = np.zeros((8, ncol))
    dp = ctypes.POINTER(ctypes.c_double)
    ins = (dp * 14)(*[_dptr(state[f]) for f in range(14)])
    outs = (dp * 12)(*[_dptr(tend[f]) for f in range(12)])
    sf = (dp * 8)(*[_dptr(sfc[f]) for f in range(8)])
    o = _Opts(stages, newton_iters, nthreads, 1 if warm else 0)
    fails = ctypes.c_int64(0)
    rc = lib().oracle_step(ins, _dptr(dz), ncol, ncol, nlev, float(dt), outs, sf,
                           ctypes.byref(o), ctypes.byref(fails))
    if rc != 0:
        raise ValueError("oracle_step rejected its arguments")
    if return_fails:
        return tend, sfc, fails.value
    return tend, sfc


def esat_liquid(T): return lib().oracle_esat_liquid(float(T))
def esat_ice(T): return lib().oracle_esat_ice(float(T))
def qsat_liquid(T, p): return lib().oracle_qsat_liquid(float(T), float(p))
def qsat_ice(T, p): return lib().oracle_qsat_ice(float(T), float(p))


def point_rates(T, p, rho, q6, n6, warm=False) -> np.ndarray:
    q = np.ascontiguousarray(q6, dtype=np.float64)
    n = np.ascontiguousarray(n6, dtype=np.float64)
    out = np.zeros(12)
    lib().oracle_point_rates(float(T), float(p), float(rho), _dptr(q), _dptr(n),
                             1 if warm else 0, _dptr(out))
    return out


def saturation_adjust(T, p, qv, qc, nc, newton_iters=5):
    a = np.array([T, qv, qc, nc], dtype=np.float64)
    vals = [ctypes.c_double(x) for x in a]
    it = lib().oracle_saturation_adjust(ctypes.byref(vals[0]), float(p), ctypes.byref(vals[1]),
                                        ctypes.byref(vals[2]), ctypes.byref(vals[3]), newton_iters)
    return vals[0].value, vals[1].value, vals[2].value, vals[3].value, it


def nsub(dz: np.ndarray, dt: float):
    dz = np.ascontiguousarray(dz, dtype=np.float64)
    out = (ctypes.c_int32 * 4)()
    lib().oracle_nsub(_dptr(dz), len(dz), float(dt), out)
    return list(out)


def point_process(in14, warm=False, newton_iters=5):
    """(adjusted state (12,), rates (12,)) of one point after clean-up, phase
    changes and saturation adjustment."""
    v = np.ascontiguousarray(in14, dtype=np.float64)
    st = np.zeros(12)
    r = np.zeros(12)
    lib().oracle_point_process(_dptr(v), 1 if warm else 0, newton_iters, _dptr(st), _dptr(r))
    return st, r


def point_apply(in14, rates12, dt, warm=False, newton_iters=5):
    """Tendencies (12,) of one point whose S4 rates are replaced by rates12."""
    v = np.ascontiguousarray(in14, dtype=np.float64)
    r = np.ascontiguousarray(rates12, dtype=np.float64)
    out = np.zeros(12)
    lib().oracle_point_apply(_dptr(v), _dptr(r), float(dt), 1 if warm else 0, newton_iters, _dptr(out))
    return out
