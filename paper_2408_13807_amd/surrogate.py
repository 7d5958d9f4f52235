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
           "sur_predict_models", "sur_predict_models_dev", "sur_save", "sur_load", "sur_last_error")

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
_I64P = ct.POINTER(ct.c_int64)
_lib.sur_predict_models.argtypes = [_H, ct.c_int64, _FP, _I64P, _I64P, _FP, ct.c_int64, _FP, _FP, _FP]
_lib.sur_predict_models_dev.argtypes = [_H, ct.c_int64, ct.c_int64, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                                        ct.c_void_p, ct.c_int64, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p]
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
        if getattr(self, "_h", None) and _lib is not None:
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

    def predict_models(self, model_x, row_off, radius_off, radius):
        """Whole-model prediction (sur_predict_models): per-row mean log10 T and
        spread, and the largest spread of every model."""
        x, px = _f32(model_x)
        ro = np.ascontiguousarray(row_off, dtype=np.int64)
        ra = np.ascontiguousarray(radius_off, dtype=np.int64)
        r, pr = _f32(radius)
        n_models, n_rows = len(ra), int(ro[-1])
        mean = np.zeros(n_rows, np.float32)
        spread = np.zeros(n_rows, np.float32)
        mspread = np.zeros(n_models, np.float32)
        self._check(_lib.sur_predict_models(self._h, n_models, px, ro.ctypes.data_as(_I64P), ra.ctypes.data_as(_I64P),
                                            pr, len(r), mean.ctypes.data_as(_FP), spread.ctypes.data_as(_FP),
                                            mspread.ctypes.data_as(_FP)))
        return mean, spread, mspread

    def predict_models_dev(self, n_models: int, n_rows: int, model_x_ptr: int, row_off_ptr: int, radius_off_ptr: int,
                           radius_ptr: int, n_radius: int, mean_ptr: int, spread_ptr: int, model_spread_ptr: int,
                           stream=None):
        self._check(_lib.sur_predict_models_dev(self._h, int(n_models), int(n_rows), model_x_ptr, row_off_ptr,
                                                radius_off_ptr, radius_ptr, int(n_radius), mean_ptr, spread_ptr,
                                                model_spread_ptr, _ire._stream_ptr(stream)))

    def save(self, path: str):
        self._check(_lib.sur_save(self._h, path.encode()))

    def load(self, path: str):
        self._check(_lib.sur_load(self._h, path.encode()))


# ---------------------------------------------------------------------------
# Parameter-study pipeline


def ire_profiles(params: dict, models, package_scale: float = 1.0, chunk: int = 16384, device: int = 0,
                 options: dict | None = None, progress=None) -> dict:
    """Per-shell temperatures of study models from batched IRE launches of at
    most `chunk` models each; T of all models end to end with row offsets.
    `progress(done, total, seconds)` is called after every launch; `seconds`
    is the wall time of all launches, host preparation included."""
    models = np.asarray(models, np.int64)
    T, A, pk = [], [], 0
    events = dict.fromkeys(("n_cross", "n_launch", "n_scat", "n_abs"), 0)
    device_ms = 0.0
    t_start = time.perf_counter()

    def make(c0):
        b = _ire.batch_from_workloads(params, models[c0:c0 + chunk], device=device, package_scale=package_scale)
        if options:
            b.set_options(**options)
        return b

    starts = list(range(0, len(models), chunk))
    cur = make(starts[0]) if starts else None
    if cur is not None:
        cur.run()
    for j, c0 in enumerate(starts):
        # the next launch's host-side inputs are built while this one runs on the device
        nxt = make(starts[j + 1]) if j + 1 < len(starts) else None
        r = cur.results(allow_limit=True)
        pk += int(r["stats"]["n_launch"])
        for k in events:
            events[k] += int(r["stats"][k])
        device_ms += float(r["stats"]["ms_run"])
        T.append(r["T"])
        A.append(r["A"])
        cur.close()
        if progress:
            progress(min(c0 + chunk, len(models)), len(models), time.perf_counter() - t_start)
        cur = nxt
        if cur is not None:
            cur.run()
    secs = time.perf_counter() - t_start
    n = params["n"][models].astype(np.int64)
    row_off = np.zeros(len(models) + 1, np.int64)
    np.cumsum(n, out=row_off[1:])
    return dict(T=np.concatenate(T) if T else np.zeros(0), A=np.concatenate(A) if A else np.zeros(0),
                row_off=row_off, seconds=secs, packages=pk, events=events, device_s=device_ms * 1e-3)


def training_set(params: dict, models, T: np.ndarray, t_floor: float = 3.0) -> tuple[np.ndarray, np.ndarray]:
    """Rows (features, log10 T) of the models for training; shells left at the
    temperature floor (no absorbed energy in the run) carry no information and
    are dropped."""
    X, _ = wl.study_features(params, models)
    keep = T > t_floor * (1 + 1e-6)
    return X[keep], np.log10(T[keep]).astype(np.float32)


def fit(X: np.ndarray, y: np.ndarray, members: int = 5, depth: int = 4, steps: int = 20000, batch: int = 4096,
        lr: float = 2e-3, lr_min: float = 2e-5, seed: int = 1, device: int = 0) -> SurNet:
    """Train an ensemble on (X, y) with inputs and target standardised."""
    net = SurNet(members=members, depth=depth, seed=seed, device=device)
    xs = X.std(axis=0)
    net.set_normalization(X.mean(axis=0), np.where(xs > 0, xs, 1.0), float(y.mean()), float(max(y.std(), 1e-6)))
    net.last_loss = net.train(X, y, steps=steps, batch=batch, lr=lr, lr_min=lr_min, seed=seed)
    return net


def predict_models(net: SurNet, params: dict, models) -> dict:
    """Surrogate temperatures of whole models (host arrays)."""
    q = wl.study_model_inputs(params, models)
    mean, spread, mspread = net.predict_models(q["model_x"], q["row_off"], q["radius_off"], q["radius"])
    return dict(logT=mean, spread=spread, model_spread=mspread, row_off=q["row_off"])


def predict_with_fallback(net: SurNet, params: dict, models, threshold: float = 0.02, package_scale: float = 1.0,
                          device: int = 0) -> dict:
    """Surrogate temperatures for every shell of the models; every model with a
    shell whose ensemble spread std(T)/mean(T) exceeds `threshold` is re-run with
    the batched IRE tracer and takes the tracer's temperatures."""
    models = np.asarray(models, np.int64)
    t0 = time.perf_counter()
    p = predict_models(net, params, models)
    t1 = time.perf_counter()
    T = 10.0 ** p["logT"].astype(np.float64)
    offs = p["row_off"]
    flagged = np.nonzero(p["model_spread"] > threshold)[0]
    ire_s = 0.0
    if len(flagged):
        r = ire_profiles(params, models[flagged], package_scale=package_scale, device=device)
        ire_s = r["seconds"]
        for j, k in enumerate(flagged):
            T[offs[k]:offs[k + 1]] = r["T"][r["row_off"][j]:r["row_off"][j + 1]]
    t2 = time.perf_counter()
    return dict(T=T, row_off=offs, spread=p["spread"], model_spread=p["model_spread"], flagged=flagged,
                seconds_predict=t1 - t0, seconds_fallback=ire_s, seconds_total=t2 - t0)


def model_errors(T: np.ndarray, T_ref: np.ndarray, row_off: np.ndarray, stat: str = "median") -> np.ndarray:
    """Per-model relative temperature error |T - T_ref| / T_ref over the shells
    of each model: "max" (the worst shell), "p95" (95th percentile over the
    shells), "median" or "mean".  The reference is itself a Monte Carlo run, so
    its own noise in rarely hit shells enters every statistic, most the max."""
    d = np.abs(T - T_ref) / T_ref
    n = np.diff(row_off)
    out = np.zeros(len(n))
    nz = n > 0
    if stat == "mean":
        out[nz] = np.add.reduceat(d, row_off[:-1][nz]) / n[nz]
        return out
    if stat == "max":
        out[nz] = np.maximum.reduceat(d, row_off[:-1][nz])
        return out
    q = {"median": 0.5, "p95": 0.95}[stat]
    for j in np.nonzero(nz)[0]:
        out[j] = np.quantile(d[row_off[j]:row_off[j + 1]], q)
    return out


def error_summary(T_sur: np.ndarray, T_ref: np.ndarray, row_off: np.ndarray, accepted: np.ndarray,
                  others: dict | None = None, limit: float = 0.02) -> dict:
    """Fractions of models within `limit` of the reference T_ref by each
    per-model statistic (worst shell, 95th percentile, median of the shells'
    relative errors): the surrogate on every model and on the models it
    accepts, and each tracer run in `others` (name -> T) on every model; with
    an "ire_1x" entry also every model after the fallback (accepted models from
    the surrogate, the others from that run)."""
    others = others or {}
    out = {}
    for stat in ("max", "p95", "median"):
        e_s = model_errors(T_sur, T_ref, row_off, stat)
        row = dict(surrogate_all=float(np.mean(e_s <= limit)),
                   surrogate_accepted=float(np.mean(e_s[accepted] <= limit)) if accepted.any() else None,
                   median_error_surrogate_accepted=float(np.median(e_s[accepted])) if accepted.any() else None)
        for name, T in others.items():
            e = model_errors(T, T_ref, row_off, stat)
            row[name] = float(np.mean(e <= limit))
            row[f"median_error_{name}"] = float(np.median(e))
            if name == "ire_1x":
                e_f = np.where(accepted, e_s, e)
                row["after_fallback"] = float(np.mean(e_f <= limit))
                row["median_error_after_fallback"] = float(np.median(e_f))
        out[stat] = row
    return out
