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
           "ire_set_options", "ire_run", "ire_begin", "ire_advance", "ire_reset", "ire_tune_schedule", "ire_sync",
           "ire_get_results", "ire_get_stats", "ire_get_results_dev", "ire_get_sed", "ire_run_noalloc",
           "ire_last_error", "ire_planck",
           "ire_batch_default_options", "ire_batch_create", "ire_batch_destroy", "ire_batch_set_dust",
           "ire_batch_set_temperature_grid", "ire_batch_set_sources", "ire_batch_set_models",
           "ire_batch_set_options", "ire_batch_run", "ire_batch_get", "ire_batch_autotune",
           "ire_batch_last_error")
IRE_SRC_EXTERNAL = 0
IRE_SRC_POINT = 1


class Options(ct.Structure):
    _fields_ = [("k_bg", ct.c_double), ("ffi", ct.c_int32), ("w_floor", ct.c_double),
                ("max_events", ct.c_uint64), ("stepping", ct.c_int32), ("max_lanes", ct.c_int32),
                ("reemit_uniform", ct.c_int32), ("aggregate", ct.c_int32), ("batch", ct.c_int32),
                ("use_g_E", ct.c_int32), ("g_E", ct.c_double), ("use_g_S", ct.c_int32), ("g_S", ct.c_double),
                ("k_A", ct.c_double), ("k_S", ct.c_double), ("k_A_rho", ct.c_int32), ("k_A_lowest", ct.c_double),
                ("k_A_highest", ct.c_double), ("replicas", ct.c_int32), ("quorum", ct.c_int32)]


class Stats(ct.Structure):
    _fields_ = [("L_ext", ct.c_double), ("L_ps", ct.c_double), ("escaped", ct.c_double * 2),
                ("ffi_escaped", ct.c_double), ("terminated", ct.c_double)] + [
        (f, ct.c_uint64) for f in ("n_launch", "n_cross", "n_scat", "n_abs", "n_escape", "n_direct",
                                   "n_limit", "n_floor", "n_below", "n_above", "n_reemit_above", "n_pass", "n_step_slots")] + [
        ("ms_tables", ct.c_float), ("ms_trace", ct.c_float), ("ms_finalize", ct.c_float)]


class ModelDesc(ct.Structure):
    _fields_ = [("n_shells", ct.c_int32), ("source", ct.c_int32), ("scale", ct.c_double),
                ("n_packages", ct.c_uint64), ("seed", ct.c_uint64)]


_MODEL_DESC_DTYPE = np.dtype({"names": ["n_shells", "source", "scale", "n_packages", "seed"],
                              "formats": [np.int32, np.int32, np.float64, np.uint64, np.uint64],
                              "offsets": [getattr(ModelDesc, f).offset for f, _ in ModelDesc._fields_],
                              "itemsize": ct.sizeof(ModelDesc)})


class BatchOptions(ct.Structure):
    _fields_ = [("k_bg", ct.c_double), ("ffi", ct.c_int32), ("w_floor", ct.c_double),
                ("max_events", ct.c_uint64), ("reemit_uniform", ct.c_int32), ("aggregate", ct.c_int32),
                ("batch", ct.c_int32), ("item_packages", ct.c_uint64), ("use_graph", ct.c_int32),
                ("use_g_E", ct.c_int32), ("g_E", ct.c_double), ("use_g_S", ct.c_int32), ("g_S", ct.c_double),
                ("k_A", ct.c_double), ("k_S", ct.c_double), ("k_A_rho", ct.c_int32), ("k_A_lowest", ct.c_double),
                ("k_A_highest", ct.c_double)]


class BatchStats(ct.Structure):
    _fields_ = [("L_total", ct.c_double), ("escaped", ct.c_double), ("ffi_escaped", ct.c_double),
                ("terminated", ct.c_double)] + [
        (f, ct.c_uint64) for f in ("n_launch", "n_cross", "n_scat", "n_abs", "n_escape", "n_limit", "n_floor",
                                   "n_below", "n_above", "n_models", "n_items", "n_shells", "n_pass", "n_step_slots")] + [
        ("ms_run", ct.c_float)]


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
_lib.ire_tune_schedule.argtypes = [_H, ct.c_uint64, ct.c_uint64, ct.POINTER(ct.c_int32), ct.POINTER(ct.c_int32)]
_lib.ire_sync.argtypes = [_H]
_lib.ire_get_results.argtypes = [_H, _DP, _DP, ct.POINTER(Stats)]
_lib.ire_get_stats.argtypes = [_H, ct.POINTER(Stats)]
_lib.ire_get_results_dev.argtypes = [_H, ct.c_void_p, ct.c_void_p, ct.c_void_p]
_lib.ire_run_noalloc.argtypes = [_H, ct.c_uint64, ct.c_uint64, ct.c_uint64, ct.c_void_p, ct.c_void_p, ct.c_void_p]
_lib.ire_get_sed.argtypes = [_H, _DP, _DP]
_lib.ire_last_error.argtypes = [_H]
_lib.ire_last_error.restype = ct.c_char_p
_lib.ire_planck.argtypes = [ct.c_int32, _DP, ct.c_double, _DP]
_lib.ire_batch_default_options.argtypes = [ct.POINTER(BatchOptions)]
_lib.ire_batch_create.argtypes = [ct.c_int, ct.POINTER(_H)]
_lib.ire_batch_destroy.argtypes = [_H]
_lib.ire_batch_destroy.restype = None
_lib.ire_batch_set_dust.argtypes = [_H, ct.c_int32, _DP, _DP, _DP, _DP]
_lib.ire_batch_set_temperature_grid.argtypes = [_H, ct.c_double, ct.c_double, ct.c_int32]
_lib.ire_batch_set_sources.argtypes = [_H, _DP, _DP]
_lib.ire_batch_set_models.argtypes = [_H, ct.c_int32, ct.POINTER(ModelDesc), _DP, _DP]
_lib.ire_batch_set_options.argtypes = [_H, ct.POINTER(BatchOptions)]
_lib.ire_batch_run.argtypes = [_H, ct.c_void_p]
_lib.ire_batch_get.argtypes = [_H, _DP, _DP, ct.POINTER(BatchStats)]
_lib.ire_batch_autotune.argtypes = [_H, ct.c_double, ct.c_char_p, ct.POINTER(BatchOptions)]
_lib.ire_batch_last_error.argtypes = [_H]
_lib.ire_batch_last_error.restype = ct.c_char_p


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
        self.K = 0

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
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
        self.K = len(a[0][0])

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

    def tune_schedule(self, n_ext: int = 0, n_ps: int = 0) -> tuple[int, int]:
        """Time candidate event-pass schedules on this model and keep the fastest;
        returns (quorum, batch)."""
        q, b = ct.c_int32(), ct.c_int32()
        self._check(_lib.ire_tune_schedule(self._h, int(n_ext), int(n_ps), ct.byref(q), ct.byref(b)))
        return q.value, b.value

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

    def sed(self) -> dict:
        """Escaping spectrum per source and frequency: total and unscattered, [2, K] each."""
        K = self.K
        tot, direct = np.zeros(2 * K), np.zeros(2 * K)
        self._check(_lib.ire_get_sed(self._h, tot.ctypes.data_as(_DP), direct.ctypes.data_as(_DP)))
        return dict(sed=tot.reshape(2, K), sed_direct=direct.reshape(2, K))

    def results_dev(self, absorbed_ptr: int | None, T_ptr: int | None, stream=None):
        self._check(_lib.ire_get_results_dev(self._h, absorbed_ptr, T_ptr, _stream_ptr(stream)))

    def run_noalloc(self, n_ext: int, n_ps: int, seed: int, absorbed_ptr: int, T_ptr: int, stream=None):
        """ire_run_noalloc: a whole run into caller device memory, with no device allocation."""
        self._check(_lib.ire_run_noalloc(self._h, int(n_ext), int(n_ps), int(seed), absorbed_ptr, T_ptr,
                                         _stream_ptr(stream)))


def run_model(model: dict, n_ext: int = 0, n_ps: int = 0, seed: int = 1, device: int = 0,
              stream=None, allow_limit: bool = False, **opts) -> dict:
    """Convenience: one complete run of a workload dict."""
    with IREModel(device) as m:
        m.set_model(model)
        m.set_options(**opts)
        m.run(n_ext, n_ps, seed, stream)
        r = m.results(allow_limit=allow_limit)
        r.update(m.sed())
        return r


def default_batch_options(**kw) -> BatchOptions:
    o = BatchOptions()
    _lib.ire_batch_default_options(ct.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class IREBatch:
    """Many cloud models sharing dust, temperature grid and source shapes, run
    in one persistent launch (ire_batch_* of include/ire.h)."""

    def __init__(self, device: int = 0):
        h = _H()
        rc = _lib.ire_batch_create(int(device), ct.byref(h))
        if rc:
            raise IREError(rc, f"ire_batch_create(device={device}) failed")
        self._h = h
        self.n_shells = 0
        self.offsets = None

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.ire_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, rc: int, allow_limit: bool = False):
        if rc == IRE_OK or (allow_limit and rc == IRE_E_LIMIT):
            return rc
        raise IREError(rc, _lib.ire_batch_last_error(self._h).decode())

    def set_dust(self, nu, kabs, albedo, g):
        a = [_arr(x) for x in (nu, kabs, albedo, g)]
        self._check(_lib.ire_batch_set_dust(self._h, len(a[0][0]), *[p for _, p in a]))

    def set_temperature_grid(self, t_min: float, t_max: float, n_t: int):
        self._check(_lib.ire_batch_set_temperature_grid(self._h, float(t_min), float(t_max), int(n_t)))

    def set_sources(self, J_shape=None, S_shape=None):
        j, pj = _arr(J_shape)
        s, ps = _arr(S_shape)
        self._check(_lib.ire_batch_set_sources(self._h, pj, ps))

    def set_models(self, n_shells, source, scale, n_packages, seeds, r_edges_flat, rho_flat):
        M = len(n_shells)
        rec = np.zeros(M, dtype=_MODEL_DESC_DTYPE)
        rec["n_shells"] = n_shells
        rec["source"] = source
        rec["scale"] = scale
        rec["n_packages"] = n_packages
        rec["seed"] = seeds
        descs = rec.ctypes.data_as(ct.POINTER(ModelDesc))
        r, pr = _arr(r_edges_flat)
        d, pd = _arr(rho_flat)
        self._check(_lib.ire_batch_set_models(self._h, M, descs, pr, pd))
        self.n_shells = int(np.sum(n_shells))
        self.offsets = np.concatenate([[0], np.cumsum(n_shells)]).astype(np.int64)

    def set_options(self, **kw):
        self._check(_lib.ire_batch_set_options(self._h, ct.byref(default_batch_options(**kw))))

    def run(self, stream=None):
        self._check(_lib.ire_batch_run(self._h, _stream_ptr(stream)))

    def results(self, allow_limit: bool = False) -> dict:
        A = np.zeros(self.n_shells)
        T = np.zeros(self.n_shells)
        st = BatchStats()
        rc = self._check(_lib.ire_batch_get(self._h, A.ctypes.data_as(_DP), T.ctypes.data_as(_DP), ct.byref(st)),
                         allow_limit)
        return dict(A=A, T=T, stats={f: getattr(st, f) for f, _ in BatchStats._fields_}, rc=rc)

    def autotune(self, fraction: float = 0.02, cache_path: str | None = None) -> dict:
        o = BatchOptions()
        self._check(_lib.ire_batch_autotune(self._h, float(fraction),
                                            cache_path.encode() if cache_path else None, ct.byref(o)))
        return {f: getattr(o, f) for f, _ in BatchOptions._fields_}


def batch_from_workloads(params: dict, models: list[int] | None = None, device: int = 0,
                         package_scale: float = 1.0) -> IREBatch:
    """An IREBatch holding models of a batched parameter study (see workloads.batch_parameters)."""
    from paper_2408_13807_amd import workloads as wl
    idx = list(range(len(params["n"]))) if models is None else list(models)
    b = IREBatch(device)
    d = wl.synthetic_dust()
    b.set_dust(d["nu"], d["kabs"], d["albedo"], d["g"])
    b.set_temperature_grid(3.0, 1600.0, 512)
    b.set_sources(wl.isrf(d["nu"]), wl.blackbody(d["nu"], 5000.0))
    idx = np.asarray(idx, np.int64)
    r_flat, rho_flat = wl.study_shells(params, idx)
    central = params["central"][idx] == 1
    n_sh = params["n"][idx].astype(np.int64)
    src = np.where(central, IRE_SRC_POINT, IRE_SRC_EXTERNAL)
    scale = np.where(central, params["L"][idx], params["field_scale"][idx])
    npk = np.maximum(1, np.round(params["n_pkg"][idx] * package_scale)).astype(np.int64)
    seeds = params["seed"][idx]
    b.set_models(n_sh, src, scale, npk, seeds, r_flat, rho_flat)
    return b
