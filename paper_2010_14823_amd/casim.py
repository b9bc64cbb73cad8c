"""ctypes binding of libcasim (include/casim.h): argument marshalling only.

Every step of the microphysics runs in the HIP kernels of libcasim.so; this
module only builds the C structs, takes device pointers and the current HIP
stream from PyTorch tensors, and turns negative return codes into
``CasimError``.  If the shared library has not been built, loading fails
loudly: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcasim.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "casim.h")

MODE_FP64, MODE_FP32MIX, MODE_SURROGATE, MODE_FP64_COMPACT = 0, 1, 2, 3
STAGE_ADJUST, STAGE_SATADJ, STAGE_RATES, STAGE_SED, STAGE_ALL = 1, 2, 4, 8, 15
FLAG_GENERIC = 1
NIN, NTEND, NSFC = 14, 12, 8
IN_NAMES = ("T", "p", "rho", "qv", "qc", "nc", "qr", "nr", "qi", "ni", "qs", "ns", "qg", "ng")
TEND_NAMES = ("dT", "dqv", "dqc", "dnc", "dqr", "dnr", "dqi", "dni", "dqs", "dns", "dqg", "dng")
SFC_NAMES = ("Pr", "Pi", "Ps", "Pg", "Nr", "Ni", "Ns", "Ng")

_d4 = ctypes.c_double * 4


class Constants(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("stages", ctypes.c_int32), ("warm", ctypes.c_int32),
                ("flags", ctypes.c_int32)] + \
        [(n, ctypes.c_double) for n in (
            "R_d", "R_v", "cp", "L_v", "L_s", "T_0", "g", "rho_w", "rho_i", "rho_s", "rho_g",
            "rho_0", "K_a", "Dv0", "Dv_exp", "esl_a", "esl_b", "esl_c", "esi_a", "esi_b", "esi_c",
            "auto_a", "auto_qc_exp", "auto_nc_exp", "accr_a", "accr_exp", "m_r0", "m_s0", "m_i0",
            "n_act", "iaut_a", "ice_t_exp", "bigg_a", "bigg_b", "cooper_a", "cooper_b",
            "cooper_max", "N0_s", "N0_g")] + \
        [("fall_a", _d4), ("fall_b", _d4), ("v_max", _d4), ("d_min", _d4), ("d_max", _d4),
         ("capacity_points", ctypes.c_int64)]


class Thresholds(ctypes.Structure):
    _fields_ = [("q_min", ctypes.c_double), ("T_hom", ctypes.c_double), ("T_nuc", ctypes.c_double),
                ("q_i0", ctypes.c_double), ("newton_iters", ctypes.c_int32),
                ("reserved0", ctypes.c_int32), ("newton_rtol", ctypes.c_double),
                ("sur_range_margin", ctypes.c_double), ("sur_maha_max", ctypes.c_double),
                ("sur_f_min", ctypes.c_double)]


class State(ctypes.Structure):
    _fields_ = [("in_", ctypes.c_void_p * NIN), ("dz", ctypes.POINTER(ctypes.c_double)),
                ("ld", ctypes.c_int64), ("tend", ctypes.c_void_p * NTEND),
                ("sfc", ctypes.c_void_p * NSFC)]


class HostState(ctypes.Structure):
    _fields_ = [("in_", ctypes.c_void_p * NIN), ("dz", ctypes.POINTER(ctypes.c_double)),
                ("ld", ctypes.c_int64), ("tend", ctypes.c_void_p * NTEND),
                ("sfc", ctypes.c_void_p * NSFC)]


class StepStatus(ctypes.Structure):
    _fields_ = [("newton_fail", ctypes.c_int64), ("nonfinite", ctypes.c_int64),
                ("fallback", ctypes.c_int64), ("inferred", ctypes.c_int64)]


_f12 = ctypes.c_float * 12
MLP_NPARAMS = 36236
MLP_MAX_BATCH = 16384
GATE_SUPERSAT_ICE = 1 << 12
RATE_NAMES = ("AUTO", "ACCR", "REVP", "DEPI", "DEPS", "IAUT", "SACI", "SACW", "GACW", "FRZR", "SMLT", "GMLT")
FEATURE_NAMES = ("lnT", "lnp", "lnrho", "lnqv", "lnqc", "lnnc", "lnqr", "lnnr", "lnqi", "lnni", "lnqs", "lnqg")


class MlpStats(ctypes.Structure):
    _fields_ = [("x_mean", _f12), ("x_std", _f12), ("x_min", _f12), ("x_max", _f12),
                ("y_mean", _f12), ("y_std", _f12), ("whiten", ctypes.c_float * 144),
                ("maha_q999", ctypes.c_float), ("reserved", ctypes.c_float * 3)]


class CasimError(RuntimeError):
    def __init__(self, code, func):
        self.code = code
        super().__init__("%s failed: %s (%d)" % (func, strerror(code), code))


_lib = None


def lib():
    """The loaded libcasim.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # PyTorch ships its own HIP runtime under the same soname as ROCm's;
        # loading torch first makes libcasim bind to that one instance, so
        # torch's streams and device pointers belong to the library's runtime.
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libcasim.so is not built: run python -m paper_2010_14823_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        sigs = {
            "casim_default_constants": [ctypes.POINTER(Constants)],
            "casim_default_thresholds": [ctypes.POINTER(Thresholds)],
            "casim_init": [ctypes.POINTER(Constants), ctypes.POINTER(Thresholds)],
            "casim_step": [ctypes.POINTER(State), i64, i32, dbl, vp],
            "casim_step_noalloc": [ctypes.POINTER(State), i64, i32, dbl, vp],
            "casim_step_host": [ctypes.POINTER(HostState), i64, i32, dbl, i32, vp],
            "casim_host_alloc": [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t],
            "casim_host_free": [vp],
            "casim_apply_tendencies": [ctypes.POINTER(State), i64, i32, dbl, vp],
            "casim_status": [vp, ctypes.POINTER(StepStatus)],
            "casim_finalize": [],
            "casim_nsub": [ctypes.POINTER(ctypes.c_double), i32, dbl, ctypes.POINTER(ctypes.c_int32)],
            "casim_debug_math": [vp, i64, vp, vp, vp],
            "casim_debug_stream": [ctypes.POINTER(State), i64, i32, dbl, vp],
            "casim_debug_bandwidth": [vp, vp, i64, i32, i32, i32, vp],
            "casim_rates_dump": [ctypes.POINTER(State), i64, i32, dbl, ctypes.c_uint64, dbl, i64, vp, vp, vp,
                                 ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64), vp],
            "casim_mlp_fit_stats": [vp, vp, vp, i64, ctypes.POINTER(MlpStats), vp],
            "casim_mlp_set_stats": [ctypes.POINTER(MlpStats)],
            "casim_mlp_prepare": [vp, vp, vp, i64, vp, vp, vp, vp],
            "casim_mlp_init": [ctypes.c_uint64],
            "casim_mlp_get_params": [vp],
            "casim_mlp_set_params": [vp],
            "casim_mlp_grad": [vp, vp, vp, vp, i32, vp, vp, vp],
            "casim_mlp_train_step": [vp, vp, vp, vp, i32, ctypes.c_float, vp, vp],
            "casim_mlp_forward": [vp, i64, vp, vp],
            "casim_mlp_save": [vp, ctypes.POINTER(ctypes.c_size_t)],
            "casim_mlp_load": [vp, ctypes.c_size_t],
            "casim_surrogate_load": [],
            "casim_surrogate_infer": [vp, vp, i64, vp, vp, vp],
            "casim_surrogate_rates": [ctypes.POINTER(State), i64, i32, dbl, vp, vp, vp],
            "casim_host_times": [ctypes.POINTER(dbl), ctypes.POINTER(dbl), ctypes.POINTER(dbl),
                                 ctypes.POINTER(ctypes.c_int32)],
        }
        for name, args in sigs.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.casim_padded_ld.argtypes = [i64]
        L.casim_padded_ld.restype = ctypes.c_int64
        L.casim_strerror.argtypes = [ctypes.c_int]
        L.casim_strerror.restype = ctypes.c_char_p
        _lib = L
    return _lib


def header_functions(path: str = HEADER):
    """Names of the functions include/casim.h declares."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(casim_[a-z0-9_]+)\s*\(", text)))


def strerror(code: int) -> str:
    return lib().casim_strerror(int(code)).decode()


def _check(rc: int, func: str):
    if rc != 0:
        raise CasimError(rc, func)


def default_constants(**overrides) -> Constants:
    c = Constants()
    _check(lib().casim_default_constants(ctypes.byref(c)), "casim_default_constants")
    for k, v in overrides.items():
        setattr(c, k, v)
    return c


def default_thresholds(**overrides) -> Thresholds:
    t = Thresholds()
    _check(lib().casim_default_thresholds(ctypes.byref(t)), "casim_default_thresholds")
    for k, v in overrides.items():
        setattr(t, k, v)
    return t


def init(constants: Constants | None = None, thresholds: Thresholds | None = None):
    c = constants if constants is not None else default_constants()
    t = thresholds if thresholds is not None else default_thresholds()
    _check(lib().casim_init(ctypes.byref(c), ctypes.byref(t)), "casim_init")


def finalize():
    _check(lib().casim_finalize(), "casim_finalize")


def _stream_handle(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _dz_array(dz, nlev: int):
    """dz as a contiguous float64 host array of exactly nlev entries (the
    library reads nlev values through the pointer)."""
    import numpy as np
    dzh = np.ascontiguousarray(dz, dtype=np.float64)
    if dzh.shape != (int(nlev),):
        raise ValueError("dz must hold exactly nlev = %d layer thicknesses, got shape %s" % (nlev, dzh.shape))
    return dzh


def padded_ld(ncol: int) -> int:
    """casim_padded_ld: the leading dimension the library recommends for
    fields of ncol columns (whole 128-byte rows, and no row stride that is a
    multiple of 4 KB)."""
    ld = int(lib().casim_padded_ld(int(ncol)))
    if ld < 0:
        raise CasimError(ld, "casim_padded_ld")
    return ld


def empty_fields(nf: int, nlev: int, ncol: int, fill: float | None = None):
    """Device float64 fields (nf, nlev, ncol) stored with the leading
    dimension padded_ld(ncol): the columns view of an (nf, nlev, ld)
    allocation.  Every entry point that takes device fields accepts such a
    view as it is (its level stride is the leading dimension)."""
    import torch
    shape = (int(nf), int(nlev), padded_ld(ncol))
    if fill is None:
        buf = torch.empty(shape, dtype=torch.float64, device="cuda")
    else:
        buf = torch.full(shape, float(fill), dtype=torch.float64, device="cuda")
    return buf[:, :, :int(ncol)]


def _layout(state, ncol):
    """(nlev, ld, ncol) of device fields (nf, nlev, width): ld is the level
    stride (the width of a contiguous tensor, the padded leading dimension
    of a view such as empty_fields returns); ncol defaults to the width."""
    nlev, width = state.shape[1], state.shape[2]
    ld = max(state.stride(1), width) if nlev == 1 else state.stride(1)
    return nlev, ld, width if ncol is None else int(ncol)


def make_state(state, dz, tend, sfc, ld: int | None = None) -> State:
    """Build a casim_state from device tensors.

    ``state``: float64 cuda tensor (14, nlev, width) whose level stride is
    the leading dimension ld (a contiguous tensor, or a view of padded
    storage); ``tend``: (12, nlev, width) with the same ld; ``sfc``: (8, >=
    ncol); ``dz``: host sequence of nlev thicknesses (m).
    """
    import numpy as np
    st = State()
    for f in range(NIN):
        st.in_[f] = state[f].data_ptr()
    for f in range(NTEND):
        st.tend[f] = tend[f].data_ptr()
    for f in range(NSFC):
        st.sfc[f] = sfc[f].data_ptr()
    dzh = _dz_array(dz, state.shape[1])
    st._dz_keep = dzh
    st.dz = dzh.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    st.ld = int(ld if ld is not None else _layout(state, None)[1])
    return st


def _rows_ok(t, ld):
    """t (nf, rows, width) with unit column stride, row stride ld >= width and
    fields that do not overlap."""
    nf, rows, width = t.shape
    if width > 1 and t.stride(2) != 1:
        return False
    if rows > 1 and t.stride(1) != ld:
        return False
    return ld >= width and (nf <= 1 or t.stride(0) >= (rows - 1) * ld + width)


def _check_ncol(ncol, state):
    """The step covers columns 0 .. ncol-1 of the fields: no more than the
    tensor holds (the library would otherwise touch the columns past a view,
    which need not belong to its storage)."""
    if not 0 <= ncol <= state.shape[2]:
        raise ValueError("ncol = %d is outside the fields' %d columns" % (ncol, state.shape[2]))


def _check_tensors(state, tend, sfc, ncol):
    """Validate device fields; returns (nlev, ld, ncol) as _layout does."""
    import torch
    for name, t, lead, dims in (("state", state, NIN, 3), ("tend", tend, NTEND, 3), ("sfc", sfc, NSFC, 2)):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.dim() == dims):
            raise ValueError("%s must be a %d-D float64 cuda tensor" % (name, dims))
        if t.shape[0] != lead:
            raise ValueError("%s must have %d fields" % (name, lead))
    nlev, ld, ncol = _layout(state, ncol)
    _check_ncol(ncol, state)
    if state.shape[1:] != tend.shape[1:]:
        raise ValueError("state and tend must share (nlev, columns)")
    if not (_rows_ok(state, ld) and _rows_ok(tend, ld)):
        raise ValueError("state and tend need unit column stride and one level stride (the leading dimension)")
    if not _rows_ok(sfc.unsqueeze(1), sfc.shape[1]):
        raise ValueError("sfc needs unit column stride and non-overlapping rows")
    if sfc.shape[-1] < ncol:
        raise ValueError("sfc is shorter than ncol")
    return nlev, ld, ncol


def step(state, dz, dt: float, tend, sfc, ncol: int | None = None, stream=None):
    """Enqueue casim_step on the current (or given) stream."""
    nlev, ld, ncol = _check_tensors(state, tend, sfc, ncol)
    st = make_state(state, dz, tend, sfc, ld)
    _check(lib().casim_step(ctypes.byref(st), ncol, nlev, float(dt), _stream_handle(stream)),
           "casim_step")


def step_noalloc(state, dz, dt: float, tend, sfc, ncol: int | None = None, stream=None):
    """Enqueue casim_step_noalloc (no device allocation in the call)."""
    nlev, ld, ncol = _check_tensors(state, tend, sfc, ncol)
    st = make_state(state, dz, tend, sfc, ld)
    _check(lib().casim_step_noalloc(ctypes.byref(st), ncol, nlev, float(dt), _stream_handle(stream)),
           "casim_step_noalloc")


def apply_tendencies(state, dz, dt: float, tend, sfc, ncol: int | None = None, stream=None):
    nlev, ld, ncol = _check_tensors(state, tend, sfc, ncol)
    st = make_state(state, dz, tend, sfc, ld)
    _check(lib().casim_apply_tendencies(ctypes.byref(st), ncol, nlev, float(dt), _stream_handle(stream)),
           "casim_apply_tendencies")


def status(stream=None) -> dict:
    s = StepStatus()
    _check(lib().casim_status(_stream_handle(stream), ctypes.byref(s)), "casim_status")
    return {"newton_fail": s.newton_fail, "nonfinite": s.nonfinite,
            "fallback": s.fallback, "inferred": s.inferred}


def nsub(dz, dt: float):
    import numpy as np
    dzh = np.ascontiguousarray(dz, dtype=np.float64)
    if dzh.ndim != 1 or dzh.size < 1:
        raise ValueError("dz must be a 1-D sequence of layer thicknesses")
    out = (ctypes.c_int32 * 4)()
    _check(lib().casim_nsub(dzh.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(dzh),
                            float(dt), out), "casim_nsub")
    return list(out)


def debug_stream(state, dz, dt: float, tend, sfc, ncol: int | None = None, stream=None):
    """casim_debug_stream: the step's memory traffic without its physics."""
    nlev, ld, ncol = _check_tensors(state, tend, sfc, ncol)
    st = make_state(state, dz, tend, sfc, ld)
    _check(lib().casim_debug_stream(ctypes.byref(st), ncol, nlev, float(dt), _stream_handle(stream)),
           "casim_debug_stream")


def debug_bandwidth(src, dst, nbytes: int, kind: int, width: int = 16, blocks: int = 1024, stream=None):
    """casim_debug_bandwidth: 0 copy src -> dst, 1 read src (one XOR per block
    into dst), 2 write zeros to dst; device tensors aligned to width (8 or 16
    bytes per lane), grid of `blocks` 256-thread blocks."""
    _check(lib().casim_debug_bandwidth(_p(src), _p(dst), int(nbytes), int(kind), int(width), int(blocks),
                                       _stream_handle(stream)), "casim_debug_bandwidth")


def debug_math(x, stream=None):
    """(exp(x), log(x)) evaluated by the library's internal binary64 routines."""
    import torch
    e = torch.empty_like(x)
    l = torch.empty_like(x)
    _check(lib().casim_debug_math(ctypes.c_void_p(x.data_ptr()), x.numel(), ctypes.c_void_p(e.data_ptr()),
                                  ctypes.c_void_p(l.data_ptr()), _stream_handle(stream)), "casim_debug_math")
    return e, l


# ---- learned surrogate ------------------------------------------------------

def _p(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def rates_dump(state, dz, dt, seed, keep_prob, max_samples, feat, rates, gates, tend, sfc,
               ncol=None, stream=None):
    """casim_rates_dump into device tensors feat (>= max x 12 float32), rates,
    gates (int16).  Returns (written, selected)."""
    nlev, ld, ncol = _check_tensors(state, tend, sfc, ncol)
    st = make_state(state, dz, tend, sfc, ld)
    n = ctypes.c_int64(0)
    sel = ctypes.c_int64(0)
    _check(lib().casim_rates_dump(ctypes.byref(st), ncol, nlev, float(dt), int(seed), float(keep_prob),
                                  int(max_samples), _p(feat), _p(rates), _p(gates), ctypes.byref(n),
                                  ctypes.byref(sel), _stream_handle(stream)), "casim_rates_dump")
    return n.value, sel.value


def mlp_fit_stats(feat, rates, gates, n, stream=None) -> MlpStats:
    st = MlpStats()
    _check(lib().casim_mlp_fit_stats(_p(feat), _p(rates), _p(gates), int(n), ctypes.byref(st),
                                     _stream_handle(stream)), "casim_mlp_fit_stats")
    return st


def mlp_set_stats(st: MlpStats):
    _check(lib().casim_mlp_set_stats(ctypes.byref(st)), "casim_mlp_set_stats")


def mlp_prepare(feat, rates, gates, n, x, y, m, stream=None):
    _check(lib().casim_mlp_prepare(_p(feat), _p(rates), _p(gates), int(n), _p(x), _p(y), _p(m),
                                   _stream_handle(stream)), "casim_mlp_prepare")


def mlp_init(seed: int):
    _check(lib().casim_mlp_init(int(seed)), "casim_mlp_init")


def mlp_get_params():
    import numpy as np
    out = np.empty(MLP_NPARAMS, dtype=np.float32)
    _check(lib().casim_mlp_get_params(out.ctypes.data_as(ctypes.c_void_p)), "casim_mlp_get_params")
    return out


def mlp_set_params(theta):
    import numpy as np
    t = np.ascontiguousarray(theta, dtype=np.float32)
    assert t.size == MLP_NPARAMS
    _check(lib().casim_mlp_set_params(t.ctypes.data_as(ctypes.c_void_p)), "casim_mlp_set_params")


def mlp_grad(x, y, m, idx, batch, grad, loss, stream=None):
    _check(lib().casim_mlp_grad(_p(x), _p(y), _p(m), _p(idx), int(batch), _p(grad), _p(loss),
                                _stream_handle(stream)), "casim_mlp_grad")


def mlp_train_step(x, y, m, idx, batch, lr, loss=None, stream=None):
    _check(lib().casim_mlp_train_step(_p(x), _p(y), _p(m), _p(idx), int(batch), ctypes.c_float(lr),
                                      _p(loss), _stream_handle(stream)), "casim_mlp_train_step")


def mlp_forward(x, n, y, stream=None):
    _check(lib().casim_mlp_forward(_p(x), int(n), _p(y), _stream_handle(stream)), "casim_mlp_forward")


def mlp_save() -> bytes:
    size = ctypes.c_size_t(0)
    _check(lib().casim_mlp_save(None, ctypes.byref(size)), "casim_mlp_save")
    buf = ctypes.create_string_buffer(size.value)
    _check(lib().casim_mlp_save(ctypes.cast(buf, ctypes.c_void_p), ctypes.byref(size)), "casim_mlp_save")
    return buf.raw[:size.value]


def mlp_load(blob: bytes):
    buf = ctypes.create_string_buffer(blob, len(blob))
    _check(lib().casim_mlp_load(ctypes.cast(buf, ctypes.c_void_p), len(blob)), "casim_mlp_load")


def surrogate_load():
    _check(lib().casim_surrogate_load(), "casim_surrogate_load")


def surrogate_infer(feat, gates, n, rates, fallback, stream=None):
    _check(lib().casim_surrogate_infer(_p(feat), _p(gates), int(n), _p(rates), _p(fallback),
                                       _stream_handle(stream)), "casim_surrogate_infer")


def surrogate_rates(state, dz, dt, rates, flags, ncol=None, stream=None):
    """casim_surrogate_rates: per-point network rates (12, nlev, ld) float32 and
    trust-region flags (nlev, ld) uint8 of a surrogate step on ``state``."""
    import torch
    if not (isinstance(state, torch.Tensor) and state.is_cuda and state.dtype == torch.float64
            and state.dim() == 3 and state.shape[0] == NIN):
        raise ValueError("state must be a (14, nlev, columns) float64 cuda tensor")
    nlev, ld, ncol = _layout(state, ncol)
    _check_ncol(ncol, state)
    if not _rows_ok(state, ld):
        raise ValueError("state needs unit column stride and one level stride (the leading dimension)")
    if not (rates.is_cuda and rates.dtype == torch.float32 and rates.is_contiguous()
            and tuple(rates.shape) == (12, nlev, ld)):
        raise ValueError("rates must be a contiguous float32 cuda tensor (12, nlev, ld)")
    if not (flags.is_cuda and flags.dtype == torch.uint8 and flags.is_contiguous()
            and tuple(flags.shape) == (nlev, ld)):
        raise ValueError("flags must be a contiguous uint8 cuda tensor (nlev, ld)")
    st = make_state(state, dz, rates, rates, ld)
    _check(lib().casim_surrogate_rates(ctypes.byref(st), ncol, nlev, float(dt), _p(rates), _p(flags),
                                       _stream_handle(stream)), "casim_surrogate_rates")


class HostArray:
    """Page-locked host memory from casim_host_alloc, viewed as a float64 numpy
    array of the given shape; freed with ``free()`` (or when collected)."""

    def __init__(self, shape):
        import numpy as np
        self.shape = tuple(int(x) for x in shape)
        n = int(np.prod(self.shape))
        self._p = ctypes.c_void_p()
        _check(lib().casim_host_alloc(ctypes.byref(self._p), max(n, 1) * 8), "casim_host_alloc")
        buf = (ctypes.c_double * max(n, 1)).from_address(self._p.value)
        self.array = np.frombuffer(buf, dtype=np.float64, count=n).reshape(self.shape)

    def free(self):
        if self._p is not None and self._p.value:
            self.array = None
            _check(lib().casim_host_free(self._p), "casim_host_free")
        self._p = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def step_host(state, dz, dt: float, tend, sfc, ncol: int | None = None, nblocks: int = 0, stream=None):
    """Enqueue casim_step_host on host arrays: state (14, nlev, ld), tend
    (12, nlev, ld), sfc (8, >= ncol), float64 C-contiguous numpy arrays
    (page-locked, e.g. HostArray, for the copies to be asynchronous).  The
    outputs are valid after the stream is synchronised."""
    import numpy as np
    for name, a, lead in (("state", state, NIN), ("tend", tend, NTEND), ("sfc", sfc, NSFC)):
        if not (isinstance(a, np.ndarray) and a.dtype == np.float64 and a.flags.c_contiguous):
            raise ValueError("%s must be a C-contiguous float64 numpy array" % name)
        if a.shape[0] != lead:
            raise ValueError("%s must have %d fields" % (name, lead))
    nlev, ld = state.shape[1], state.shape[2]
    ncol = ld if ncol is None else int(ncol)
    if tend.shape[1:] != state.shape[1:] or sfc.shape[-1] < ncol:
        raise ValueError("tend must match state's (nlev, ld) and sfc hold ncol columns")
    hs = HostState()
    for f in range(NIN):
        hs.in_[f] = state[f].ctypes.data
    for f in range(NTEND):
        hs.tend[f] = tend[f].ctypes.data
    for f in range(NSFC):
        hs.sfc[f] = sfc[f].ctypes.data
    dzh = _dz_array(dz, nlev)
    hs.dz = dzh.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    hs.ld = ld
    _check(lib().casim_step_host(ctypes.byref(hs), ncol, nlev, float(dt), int(nblocks), _stream_handle(stream)),
           "casim_step_host")


def host_times():
    """(h2d_ms, step_ms, d2h_ms, nblocks) of the last casim_step_host."""
    h, k, d = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    nb = ctypes.c_int32()
    _check(lib().casim_host_times(ctypes.byref(h), ctypes.byref(k), ctypes.byref(d), ctypes.byref(nb)),
           "casim_host_times")
    return h.value, k.value, d.value, nb.value
