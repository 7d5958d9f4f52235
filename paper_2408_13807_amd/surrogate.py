"""Learned surrogate of the IRE temperature profile (sur_* of include/ire.h).

ctypes marshalling for the BF16-MFMA MLP ensemble, plus the parameter-study
pipeline around it: rows from batched IRE runs, ensemble prediction, and the
IRE fallback for every model whose ensemble spread exceeds a threshold.
"""
from __future__ import annotations

import ctypes as ct
import time

import numpy as np

from paper_2408_13807_amd import ire as _ire
from paper_2408_13807_amd import workloads as wl

_lib = _ire.library()
_FP = ct.POINTER(ct.c_float)
_H = ct.c_void_p


class TrainOpts(ct.Structure):
    _fields_ = [("batch", ct.c_int64), ("steps", ct.c_int64), ("lr", ct.c_double), ("lr_min", ct.c_double),
                ("beta1", ct.c_double), ("beta2", ct.c_double), ("eps", ct.c_double), ("seed", ct.c_uint64),
                ("use_graph", ct.c_int32)]


EXPORTS = ("sur_default_train_opts", "sur_create", "sur_destroy", "sur_set_normalization", "sur_param_count",
           "sur_get_params", "sur_set_params", "sur_train", "sur_gradients", "sur_predict", "sur_predict_dev",
           "sur_save", "sur_load", "sur_last_error")

_lib.sur_default_train_opts.argtypes = [ct.POINTER(TrainOpts)]
_lib.sur_create.argtypes = [ct.c_int, ct.c_int32, ct.c_int32, ct.c_int32, ct.c_uint64, ct.POINTER(_H)]
_lib.sur_destroy.argtypes = [_H]
_lib.sur_destroy.restype = None
_lib.sur_set_normalization.argtypes = [_H, _FP, _FP, ct.c_float, ct.c_float]
_lib.sur_param_count.argtypes = [_H]
_lib.sur_param_count.restype = ct.c_int64
_lib.sur_get_params.argtypes = [_H, _FP]
_lib.sur_set_params.argtypes = [_H, _FP]
_lib.sur_train.argtypes = [_H, _FP, _FP, ct.c_int64, ct.POINTER(TrainOpts), ct.c_void_p, _FP]
_lib.sur_gradients.argtypes = [_H, _FP, _FP, ct.c_int64, _FP, _FP]
_lib.sur_predict.argtypes = [_H, _FP, ct.c_int64, _FP, _FP]
_lib.sur_predict_dev.argtypes = [_H, ct.c_void_p, ct.c_int64, ct.c_void_p, ct.c_void_p, ct.c_void_p]
_lib.sur_save.argtypes = [_H, ct.c_char_p]
_lib.sur_load.argtypes = [_H, ct.c_char_p]
_lib.sur_last_error.argtypes = [_H]
_lib.sur_last_error.restype = ct.c_char_p


def _f32(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data_as(_FP)


def default_train_opts(**kw) -> TrainOpts:
    o = TrainOpts()
    _lib.sur_default_train_opts(ct.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class SurNet:
    """Ensemble of MLPs (6 inputs -> depth x 256 SiLU -> log10 T)."""

    def __init__(self, members: int = 5, depth: int = 4, seed: int = 1, device: int = 0):
        h = _H()
        rc = _lib.sur_create(int(device), int(members), 256, int(depth), int(seed), ct.byref(h))
        if rc:
            raise _ire.IREError(rc, "sur_create failed")
        self._h = h
        self.members, self.depth = members, depth
        self.n_params = int(_lib.sur_param_count(h))

    def close(self):
        if getattr(self, "_h", None):
            _lib.sur_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def _check(self, rc):
        if rc != _ire.IRE_OK:
            raise _ire.IREError(rc, _lib.sur_last_error(self._h).decode())

    def set_normalization(self, x_mean, x_std, y_mean: float, y_std: float):
        a, pa = _f32(x_mean)
        b, pb = _f32(x_std)
        self._check(_lib.sur_set_normalization(self._h, pa, pb, float(y_mean), float(y_std)))

    def get_params(self) -> np.ndarray:
        p = np.zeros(self.members * self.n_params, np.float32)
        self._check(_lib.sur_get_params(self._h, p.ctypes.data_as(_FP)))
        return p.reshape(self.members, self.n_params)

    def set_params(self, p):
        a, pa = _f32(np.asarray(p).reshape(-1))
        self._check(_lib.sur_set_params(self._h, pa))

    def train(self, X, y, stream=None, **opts) -> np.ndarray:
        x, px = _f32(X)
        t, pt = _f32(y)
        loss = np.zeros(self.members, np.float32)
        self._check(_lib.sur_train(self._h, px, pt, len(t), ct.byref(default_train_opts(**opts)),
                                   _ire._stream_ptr(stream), loss.ctypes.data_as(_FP)))
        return loss

    def gradients(self, X, y):
        x, px = _f32(X)
        t, pt = _f32(y)
        g = np.zeros(self.members * self.n_params, np.float32)
        loss = np.zeros(self.members, np.float32)
        self._check(_lib.sur_gradients(self._h, px, pt, len(t), g.ctypes.data_as(_FP), loss.ctypes.data_as(_FP)))
        return loss, g.reshape(self.members, self.n_params)

    def predict(self, X):
        x, px = _f32(X)
        n = len(x)
        mean = np.zeros(n, np.float32)
        spread = np.zeros(n, np.float32)
        self._check(_lib.sur_predict(self._h, px, n, mean.ctypes.data_as(_FP), spread.ctypes.data_as(_FP)))
        return mean, spread

    def predict_dev(self, X_ptr: int, n: int, mean_ptr: int, spread_ptr: int, stream=None):
        self._check(_lib.sur_predict_dev(self._h, X_ptr, int(n), mean_ptr, spread_ptr, _ire._stream_ptr(stream)))

    def save(self, path: str):
        self._check(_lib.sur_save(self._h, path.encode()))

    def load(self, path: str):
        self._check(_lib.sur_load(self._h, path.encode()))


# ---------------------------------------------------------------------------
# Parameter-study pipeline


def model_rows(params: dict, models) -> tuple[np.ndarray, np.ndarray]:
    """Surrogate inputs of every shell of the given models, and the row offsets per model."""
    feats, offs = [], [0]
    for m in models:
        mm = wl.batch_model(params, int(m))
        f = wl.surrogate_features(params, int(m), mm["r_edges"])
        feats.append(f)
        offs.append(offs[-1] + len(f))
    return np.concatenate(feats), np.asarray(offs, np.int64)


def ire_temperatures(params: dict, models, package_scale: float = 1.0, device: int = 0, autotune: bool = False):
    """Per-shell temperatures of the models from one batched IRE launch."""
    b = _ire.batch_from_workloads(params, models, device=device, package_scale=package_scale)
    if autotune:
        b.autotune(fraction=0.05)
    t0 = time.perf_counter()
    b.run()
    r = b.results(allow_limit=True)
    dt = time.perf_counter() - t0
    T = r["T"].copy()
    offs = b.offsets.copy()
    b.close()
    return T, offs, dt, r["stats"]


def predict_with_fallback(net: SurNet, params: dict, models, threshold: float = 0.02, package_scale: float = 1.0,
                          device: int = 0) -> dict:
    """Surrogate temperatures for every shell of the models; every model with a
    shell whose ensemble spread std(T)/mean(T) exceeds `threshold` is re-run with
    the batched IRE tracer and takes the tracer's temperatures."""
    t0 = time.perf_counter()
    X, offs = model_rows(params, models)
    t1 = time.perf_counter()
    mean_logT, spread = net.predict(X)
    t2 = time.perf_counter()
    T = 10.0 ** mean_logT.astype(np.float64)
    per_model = np.maximum.reduceat(spread, offs[:-1]) if len(models) else np.zeros(0)
    flagged = [m for m, s in zip(models, per_model) if s > threshold]
    ire_s = 0.0
    if flagged:
        Tf, offf, ire_s, _ = ire_temperatures(params, flagged, package_scale=package_scale, device=device)
        pos = {m: j for j, m in enumerate(models)}
        for j, m in enumerate(flagged):
            k = pos[m]
            T[offs[k]:offs[k + 1]] = Tf[offf[j]:offf[j + 1]]
    t3 = time.perf_counter()
    return dict(T=T, offsets=offs, spread=spread, flagged=flagged, seconds_features=t1 - t0,
                seconds_predict=t2 - t1, seconds_fallback=ire_s, seconds_total=t3 - t0)
