"""ctypes binding of libire (include/ire.h): argument marshalling only.

Every step of the tracing runs in the HIP kernels of libire.so; this module
raises ImportError when the library has not been built.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libire.so")

IRE_OK = 0
IRE_E_INVALID = -1
IRE_E_STATE = -2
IRE_E_NOMEM = -3
IRE_E_DEVICE = -4
IRE_E_LIMIT = -5
IRE_FP32 = 0
IRE_FP64 = 1

# every symbol include/ire.h declares
EXPORTS = ("ire_default_options", "ire_create", "ire_destroy", "ire_set_shells", "ire_set_dust",
           "ire_set_temperature_grid", "ire_set_external_field", "ire_set_point_source",
           "ire_set_options", "ire_run", "ire_begin", "ire_advance", "ire_reset", "ire_sync",
           "ire_get_results", "ire_get_stats", "ire_get_results_dev", "ire_last_error", "ire_planck")


class Options(ct.Structure):
    _fields_ = [("k_bg", ct.c_double), ("ffi", ct.c_int32), ("w_floor", ct.c_double),
                ("max_events", ct.c_uint64), ("stepping", ct.c_int32), ("max_lanes", ct.c_int32),
                ("reemit_uniform", ct.c_int32), ("aggregate", ct.c_int32), ("batch", ct.c_int32)]


class Stats(ct.Structure):
    _fields_ = [("L_ext", ct.c_double), ("L_ps", ct.c_double), ("escaped", ct.c_double * 2),
                ("ffi_escaped", ct.c_double), ("terminated", ct.c_double)] + [
        (f, ct.c_uint64) for f in ("n_launch", "n_cross", "n_scat", "n_abs", "n_escape", "n_direct",
                                   "n_limit", "n_floor", "n_below", "n_above", "n_reemit_above")] + [
        ("ms_tables", ct.c_float), ("ms_trace", ct.c_float), ("ms_finalize", ct.c_float)]


class IREError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libire error {code}: {msg}")
        self.code = code


if not os.path.exists(LIB_PATH):
    raise ImportError(f"libire.so is not built ({LIB_PATH}); run __graft_entry__.build()")

# PyTorch bundles its own HIP runtime under the same soname as the system one.
# Loading torch first makes libire bind to that same runtime, so device
# pointers and streams created by torch are valid in libire calls.
try:
    import torch  # noqa: F401
except ImportError:  # plain C-ABI use without torch
    torch = None

_lib = ct.CDLL(LIB_PATH)
_DP = ct.POINTER(ct.c_double)
_H = ct.c_void_p

_lib.ire_default_options.argtypes = [ct.POINTER(Options)]
_lib.ire_create.argtypes = [ct.c_int, ct.POINTER(_H)]
_lib.ire_destroy.argtypes = [_H]
_lib.ire_destroy.restype = None
_lib.ire_set_shells.argtypes = [_H, ct.c_int32, _DP, _DP]
_lib.ire_set_dust.argtypes = [_H, ct.c_int32, _DP, _DP, _DP, _DP]
_lib.ire_set_temperature_grid.argtypes = [_H, ct.c_double, ct.c_double, ct.c_int32]
_lib.ire_set_external_field.argtypes = [_H, _DP]
_lib.ire_set_point_source.argtypes = [_H, ct.c_double, _DP]
_lib.ire_set_options.argtypes = [_H, ct.POINTER(Options)]
_lib.ire_run.argtypes = [_H, ct.c_uint64, ct.c_uint64, ct.c_uint64, ct.c_void_p]
_lib.ire_begin.argtypes = [_H, ct.c_uint64, ct.c_uint64, ct.c_uint64]
_lib.ire_advance.argtypes = [_H, ct.c_uint64, ct.c_uint64, ct.c_void_p]
_lib.ire_reset.argtypes = [_H]
_lib.ire_sync.argtypes = [_H]
_lib.ire_get_results.argtypes = [_H, _DP, _DP, ct.POINTER(Stats)]
_lib.ire_get_stats.argtypes = [_H, ct.POINTER(Stats)]
_lib.ire_get_results_dev.argtypes = [_H, ct.c_void_p, ct.c_void_p, ct.c_void_p]
_lib.ire_last_error.argtypes = [_H]
_lib.ire_last_error.restype = ct.c_char_p
_lib.ire_planck.argtypes = [ct.c_int32, _DP, ct.c_double, _DP]


def library() -> ct.CDLL:
    return _lib


def _arr(a):
    if a is None:
        return None, None
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_DP)


def default_options(**kw) -> Options:
    o = Options()
    _lib.ire_default_options(ct.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def planck(nu, T: float) -> np.ndarray:
    nu, p = _arr(nu)
    out = np.zeros_like(nu)
    rc = _lib.ire_planck(len(nu), p, float(T), out.ctypes.data_as(_DP))
    if rc:
        raise IREError(rc, "ire_planck")
    return out


def _stream_ptr(stream) -> int | None:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


class IREModel:
    """One cloud model on one HIP device (a handle of include/ire.h)."""

    def __init__(self, device: int = 0):
        h = _H()
        rc = _lib.ire_create(int(device), ct.byref(h))
        if rc:
            raise IREError(rc, f"ire_create(device={device}) failed")
        self._h = h
        self.n = 0

    def close(self):
        if getattr(self, "_h", None):
            _lib.ire_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, rc: int):
        if rc not in (IRE_OK,):
            raise IREError(rc, _lib.ire_last_error(self._h).decode())

    def set_shells(self, r_edges, rho):
        r, pr = _arr(r_edges)
        d, pd = _arr(rho)
        self._check(_lib.ire_set_shells(self._h, len(d), pr, pd))
        self.n = len(d)

    def set_dust(self, nu, kabs, albedo, g):
        a = [_arr(x) for x in (nu, kabs, albedo, g)]
        self._check(_lib.ire_set_dust(self._h, len(a[0][0]), *[p for _, p in a]))

    def set_temperature_grid(self, t_min: float, t_max: float, n_t: int):
        self._check(_lib.ire_set_temperature_grid(self._h, float(t_min), float(t_max), int(n_t)))

    def set_external_field(self, J):
        a, p = _arr(J)
        self._check(_lib.ire_set_external_field(self._h, p))

    def set_point_source(self, L: float, spectrum):
        a, p = _arr(spectrum)
        self._check(_lib.ire_set_point_source(self._h, float(L), p))

    def set_options(self, **kw):
        self._check(_lib.ire_set_options(self._h, ct.byref(default_options(**kw))))

    def set_model(self, model: dict):
        """Set shells, dust, temperature grid and sources from a workload dict."""
        self.set_shells(model["r_edges"], model["rho"])
        self.set_dust(model["nu"], model["kabs"], model["albedo"], model["g"])
        self.set_temperature_grid(model["t_min"], model["t_max"], model["n_t"])
        self.set_external_field(model.get("J"))
        if model.get("S") is not None and (model.get("L_ps") or 0.0) > 0.0:
            self.set_point_source(model["L_ps"], model["S"])
        else:
            self.set_point_source(0.0, None)

    def run(self, n_ext: int = 0, n_ps: int = 0, seed: int = 1, stream=None):
        self._check(_lib.ire_run(self._h, int(n_ext), int(n_ps), int(seed), _stream_ptr(stream)))

    def begin(self, n_ext_total: int = 0, n_ps_total: int = 0, seed: int = 1):
        self._check(_lib.ire_begin(self._h, int(n_ext_total), int(n_ps_total), int(seed)))

    def advance(self, n_ext: int = 0, n_ps: int = 0, stream=None):
        self._check(_lib.ire_advance(self._h, int(n_ext), int(n_ps), _stream_ptr(stream)))

    def reset(self):
        self._check(_lib.ire_reset(self._h))

    def sync(self):
        self._check(_lib.ire_sync(self._h))

    def results(self, allow_limit: bool = False) -> dict:
        A = np.zeros(self.n)
        T = np.zeros(self.n)
        st = Stats()
        rc = _lib.ire_get_results(self._h, A.ctypes.data_as(_DP), T.ctypes.data_as(_DP), ct.byref(st))
        if not (rc == IRE_OK or (allow_limit and rc == IRE_E_LIMIT)):
            self._check(rc)
        stats = {f: getattr(st, f) for f, _ in Stats._fields_}
        stats["escaped"] = list(st.escaped)
        return dict(A=A, T=T, stats=stats, rc=rc)

    def stats(self) -> dict:
        st = Stats()
        self._check(_lib.ire_get_stats(self._h, ct.byref(st)))
        out = {f: getattr(st, f) for f, _ in Stats._fields_}
        out["escaped"] = list(st.escaped)
        return out

    def results_dev(self, absorbed_ptr: int | None, T_ptr: int | None, stream=None):
        self._check(_lib.ire_get_results_dev(self._h, absorbed_ptr, T_ptr, _stream_ptr(stream)))


def run_model(model: dict, n_ext: int = 0, n_ps: int = 0, seed: int = 1, device: int = 0,
              stream=None, allow_limit: bool = False, **opts) -> dict:
    """Convenience: one complete run of a workload dict."""
    with IREModel(device) as m:
        m.set_model(model)
        m.set_options(**opts)
        m.run(n_ext, n_ps, seed, stream)
        return m.results(allow_limit=allow_limit)
