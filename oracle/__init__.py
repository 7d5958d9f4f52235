"""Python access to the serial FP64 IRE oracle (ire_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of bench.py.  The product library never imports it.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ire_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_ire_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with the host C compiler."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall",
                               "-Wno-unused-function", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Model(ct.Structure):
    _fields_ = [("n", ct.c_int32), ("r_edges", ct.POINTER(ct.c_double)),
                ("rho", ct.POINTER(ct.c_double)), ("K", ct.c_int32),
                ("nu", ct.POINTER(ct.c_double)), ("kabs", ct.POINTER(ct.c_double)),
                ("albedo", ct.POINTER(ct.c_double)), ("g", ct.POINTER(ct.c_double)),
                ("t_min", ct.c_double), ("t_max", ct.c_double), ("n_t", ct.c_int32),
                ("J", ct.POINTER(ct.c_double)), ("L_ps", ct.c_double),
                ("S", ct.POINTER(ct.c_double))]


class Options(ct.Structure):
    _fields_ = [("k_bg", ct.c_double), ("ffi", ct.c_int32), ("w_floor", ct.c_double),
                ("max_events", ct.c_uint64), ("table_mode", ct.c_int32),
                ("acc_bits", ct.c_int32), ("n_batches", ct.c_int32),
                ("reemit_uniform", ct.c_int32), ("use_g_E", ct.c_int32), ("g_E", ct.c_double),
                ("use_g_S", ct.c_int32), ("g_S", ct.c_double), ("k_A", ct.c_double), ("k_S", ct.c_double),
                ("k_A_rho", ct.c_int32), ("k_A_lowest", ct.c_double), ("k_A_highest", ct.c_double)]


class Stats(ct.Structure):
    _fields_ = [("L_ext", ct.c_double), ("L_ps", ct.c_double),
                ("escaped", ct.c_double * 2), ("ffi_escaped", ct.c_double),
                ("terminated", ct.c_double)] + [
        (f, ct.c_uint64) for f in ("n_launch", "n_cross", "n_scat", "n_abs", "n_escape",
                                   "n_direct", "n_limit", "n_floor", "n_below", "n_above",
                                   "n_reemit_above")] + [("terminated_floor", ct.c_double)]


_DP = ct.POINTER(ct.c_double)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ct.CDLL(_LIB_PATH)
        lib.or_run.argtypes = [ct.POINTER(Model), ct.POINTER(Options), ct.c_uint64, ct.c_uint64,
                               ct.c_uint64, _DP, _DP, ct.POINTER(Stats), _DP, _DP, _DP, _DP]
        lib.or_run.restype = ct.c_int
        lib.or_philox4x32_10.argtypes = [ct.POINTER(ct.c_uint32), ct.POINTER(ct.c_uint32),
                                         ct.POINTER(ct.c_uint32)]
        lib.or_planck.argtypes = [ct.c_double, ct.c_double]
        lib.or_planck.restype = ct.c_double
        lib.or_tables.argtypes = [ct.POINTER(Model)] + [_DP] * 7
        lib.or_tables.restype = ct.c_int
        lib.or_temperature.argtypes = [ct.POINTER(Model), ct.c_double, ct.c_int32]
        lib.or_temperature.restype = ct.c_double
        lib.or_eval_sampler.argtypes = [ct.c_int32, ct.c_double, ct.c_int64, _DP, _DP, _DP]
        lib.or_eval_sampler.restype = ct.c_int
        lib.or_default_options.argtypes = [ct.POINTER(Options)]
        lib.or_scatter_direction.argtypes = [_DP, _DP, ct.c_double, ct.c_double]
        lib.or_reemit_weighted.argtypes = [ct.c_double, ct.c_int32, ct.c_double, _DP]
        lib.or_reemit_weighted.restype = ct.c_double
        lib.or_scatter_weighted.argtypes = [_DP, _DP, ct.c_double, ct.c_double, ct.c_int32, ct.c_double,
                                            ct.c_double, _DP, _DP]
        lib.or_ffi_absorption.argtypes = [ct.c_double, ct.c_double, ct.c_double, _DP]
        lib.or_ffi_absorption.restype = ct.c_double
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(_DP) if a is not None else None


class _Pinned:
    """Keeps the numpy arrays behind a Model alive."""

    def __init__(self, model: dict):
        f = lambda k: None if model.get(k) is None else np.ascontiguousarray(model[k], np.float64)
        self.arrays = {k: f(k) for k in ("r_edges", "rho", "nu", "kabs", "albedo", "g", "J", "S")}
        a = self.arrays
        self.m = Model(n=len(a["rho"]), r_edges=_dp(a["r_edges"]), rho=_dp(a["rho"]),
                       K=len(a["nu"]), nu=_dp(a["nu"]), kabs=_dp(a["kabs"]),
                       albedo=_dp(a["albedo"]), g=_dp(a["g"]), t_min=float(model["t_min"]),
                       t_max=float(model["t_max"]), n_t=int(model["n_t"]), J=_dp(a["J"]),
                       L_ps=float(model.get("L_ps", 0.0) or 0.0), S=_dp(a["S"]))


def options(**kw) -> Options:
    o = Options()
    _load().or_default_options(ct.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def run(model: dict, n_ext: int = 0, n_ps: int = 0, seed: int = 1, reemit: bool = False,
        first_abs: bool = False, sed: bool = False, **opts) -> dict:
    """One oracle run; returns A, T, stats and the optional tallies."""
    lib = _load()
    pm = _Pinned(model)
    n, K = pm.m.n, pm.m.K
    A = np.zeros(n)
    T = np.zeros(n)
    R = np.zeros(n * K) if reemit else None
    F = np.zeros(n) if first_abs else None
    S = np.zeros(2 * K) if sed else None
    SD = np.zeros(2 * K) if sed else None
    st = Stats()
    o = options(**opts)
    rc = lib.or_run(ct.byref(pm.m), ct.byref(o), int(n_ext), int(n_ps), int(seed), _dp(A), _dp(T),
                    ct.byref(st), _dp(R), _dp(F), _dp(S), _dp(SD))
    if rc != 0:
        raise ValueError(f"oracle rejected the model (code {rc})")
    stats = {f: getattr(st, f) for f, _ in Stats._fields_}
    stats["escaped"] = list(st.escaped)
    out = dict(A=A, T=T, stats=stats)
    if reemit:
        out["reemit"] = R.reshape(n, K)
    if first_abs:
        out["first_abs"] = F
    if sed:
        out["sed"] = S.reshape(2, K)
        out["sed_direct"] = SD.reshape(2, K)
    return out


def ensemble(model: dict, n_ext: int = 0, n_ps: int = 0, seeds=range(1, 17), threads: int | None = None,
             **opts) -> dict:
    """Independent runs over seeds (threads release the GIL inside the C call)."""
    seeds = list(seeds)
    threads = threads or min(len(seeds), os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=threads) as ex:
        res = list(ex.map(lambda s: run(model, n_ext, n_ps, s, **opts), seeds))
    T = np.stack([r["T"] for r in res])
    A = np.stack([r["A"] for r in res])
    return dict(T=T, A=A, stats=[r["stats"] for r in res], seeds=seeds)


def philox4x32_10(ctr, key) -> np.ndarray:
    c = (ct.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (ct.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (ct.c_uint32 * 4)()
    _load().or_philox4x32_10(c, k, o)
    return np.array(list(o), dtype=np.uint32)


def planck(nu: float, T: float) -> float:
    return _load().or_planck(float(nu), float(T))


def tables(model: dict) -> dict:
    lib = _load()
    pm = _Pinned(model)
    n, K, nt = pm.m.n, pm.m.K, pm.m.n_t
    w, G, D = np.zeros(K), np.zeros(nt), np.zeros(nt * K)
    ce, cp, M, L = np.zeros(K), np.zeros(K), np.zeros(n), np.zeros(2)
    rc = lib.or_tables(ct.byref(pm.m), _dp(w), _dp(G), _dp(D), _dp(ce), _dp(cp), _dp(M), _dp(L))
    if rc != 0:
        raise ValueError(f"oracle rejected the model (code {rc})")
    return dict(w=w, G=G, D=D.reshape(nt, K), cdf_ext=ce, cdf_ps=cp, mass=M, L_ext=L[0], L_ps=L[1])


def temperature(model: dict, a: float, table_mode: int = 0) -> float:
    pm = _Pinned(model)
    return _load().or_temperature(ct.byref(pm.m), float(a), int(table_mode))


def eval_sampler(which: int, param: float, u: np.ndarray):
    u = np.ascontiguousarray(u, np.float64)
    out = np.zeros_like(u)
    w = np.zeros_like(u)
    rc = _load().or_eval_sampler(int(which), float(param), len(u), _dp(u), _dp(out), _dp(w))
    if rc != 0:
        raise ValueError("unknown sampler")
    return out, w


def scatter_direction(x, d, ct_: float, phi: float) -> np.ndarray:
    x = np.ascontiguousarray(x, np.float64)
    d = np.array(d, np.float64)
    _load().or_scatter_direction(_dp(x), _dp(d), float(ct_), float(phi))
    return d


def reemit_weighted(g_E: float, src: int, u: np.ndarray):
    """Radial direction cosines and weights of HG(g_E)-weighted re-emission."""
    lib = _load()
    out, w = np.zeros(len(u)), np.zeros(len(u))
    W = ct.c_double()
    for j, uj in enumerate(np.asarray(u, np.float64)):
        out[j] = lib.or_reemit_weighted(float(g_E), int(src), float(uj), ct.byref(W))
        w[j] = W.value
    return out, w


def scatter_weighted(x, d, g: float, g_S: float, src: int, u0: float, u1: float):
    """(new direction, cos of the scattering angle, weight) of HG(g_S)-weighted scattering."""
    x = np.ascontiguousarray(x, np.float64)
    d = np.array(d, np.float64)
    c, W = ct.c_double(), ct.c_double()
    _load().or_scatter_weighted(_dp(x), _dp(d), float(g), float(g_S), int(src), float(u0), float(u1),
                                ct.byref(c), ct.byref(W))
    return d, c.value, W.value


def ffi_absorption(tau0: float, albedo: float, u: np.ndarray):
    """Extinction depths and weights of the forced first interaction in absorption depth."""
    lib = _load()
    out, w = np.zeros(len(u)), np.zeros(len(u))
    W = ct.c_double()
    for j, uj in enumerate(np.asarray(u, np.float64)):
        out[j] = lib.or_ffi_absorption(float(tau0), float(albedo), float(uj), ct.byref(W))
        w[j] = W.value
    return out, w
