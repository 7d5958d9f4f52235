"""Seeded synthetic workloads (inputs only; none of the method's arithmetic).

The paper's test clouds are Bonnor-Ebert spheres with the Compiegne et al.
(2011) dust model, heated by the Black (1987) interstellar radiation field or
by a central 10 000 K star (Sect. 3).  Those tables are not available here, so
these analytic stand-ins keep the shapes the paper works with: ~100 shells,
central visual optical depths of order 1-100, 1e5-1e8 packages, and either an
external isotropic field or a central point source.

Every function returns plain numpy arrays in cgs units in a dict with keys
    r_edges (n+1), rho (n), nu, kabs, albedo, g (K), t_min, t_max, n_t,
    J (K or None), L_ps (float), S (K or None)
which both the library binding and the test oracle accept.
"""
from __future__ import annotations

import numpy as np

# physical constants (cgs) used to define the inputs
H = 6.62607015e-27
KB = 1.380649e-16
C = 2.99792458e10
PC = 3.0856775814913673e18
AU = 1.495978707e13
LSUN = 3.828e33
NU_V = C / 0.55e-4          # V band, 0.55 micron

R_OUT = 0.1 * PC
R0_CORE = 0.02 * PC


def blackbody(nu: np.ndarray, T: float) -> np.ndarray:
    """Planck intensity used to define source spectra (input definition only)."""
    x = H * nu / (KB * T)
    out = np.zeros_like(nu, dtype=np.float64)
    ok = x < 700.0
    out[ok] = 2.0 * H * nu[ok] ** 3 / C**2 / np.expm1(x[ok])
    return out


def frequency_grid(K: int = 64, lo: float = 3e11, hi: float = 3e15) -> np.ndarray:
    return lo * (hi / lo) ** (np.arange(K) / (K - 1))


def kappa_abs(nu: np.ndarray, kappa0: float = 1.0) -> np.ndarray:
    """kappa_abs proportional to nu^1.8 below 1e14 Hz and nu^1.0 above, continuous at 1e14 Hz."""
    nu = np.asarray(nu, dtype=np.float64)
    x = nu / 1e14
    return kappa0 * np.where(nu < 1e14, x**1.8, x**1.0)


def albedo(nu: np.ndarray) -> np.ndarray:
    nu = np.asarray(nu, dtype=np.float64)
    return np.where(nu > 3e14, 0.5, 0.0)


def synthetic_dust(K: int = 64, kappa0: float = 1.0, g: float = 0.5):
    nu = frequency_grid(K)
    return dict(nu=nu, kabs=kappa_abs(nu, kappa0), albedo=albedo(nu), g=np.full(K, g))


def kappa_ext_V(kappa0: float = 1.0) -> float:
    """Extinction opacity at the V band from the analytic dust law (not the grid)."""
    ka = float(kappa_abs(np.array([NU_V]), kappa0)[0])
    a = float(albedo(np.array([NU_V]))[0])
    return ka / (1.0 - a)


def isrf(nu: np.ndarray, scale: float = 1.0) -> np.ndarray:
    """Diluted blackbodies: W=1e-14 at 10^4 K plus W=1e-13 at 3500 K."""
    return scale * (1e-14 * blackbody(nu, 1e4) + 1e-13 * blackbody(nu, 3500.0))


def scale_to_tau_V(r_edges: np.ndarray, shape: np.ndarray, tau_V: float,
                   kappa0: float = 1.0) -> np.ndarray:
    """Scale a density shape so the radial V-band extinction depth equals tau_V."""
    dr = np.diff(r_edges)
    col = float(np.sum(shape * dr)) * kappa_ext_V(kappa0)
    return shape * (tau_V / col)


def external_sphere(n: int = 50, tau_V: float = 1.0, p: float = 2.0, field_scale: float = 1.0,
                    K: int = 64, kappa0: float = 1.0, g: float = 0.5, n_t: int = 512,
                    t_min: float = 3.0, t_max: float = 1600.0) -> dict:
    """Equal-width shells from r=0 to 0.1 pc, n(r) = (1+(r/0.02 pc)^2)^(-p/2) at mid-radii."""
    r = np.linspace(0.0, R_OUT, n + 1)
    rm = 0.5 * (r[1:] + r[:-1])
    shape = (1.0 + (rm / R0_CORE) ** 2) ** (-0.5 * p)
    rho = scale_to_tau_V(r, shape, tau_V, kappa0)
    d = synthetic_dust(K, kappa0, g)
    return dict(r_edges=r, rho=rho, **d, t_min=t_min, t_max=t_max, n_t=n_t,
                J=isrf(d["nu"], field_scale), L_ps=0.0, S=None)


def central_source(n: int = 200, tau_V: float = 100.0, p: float = 1.5, L: float = LSUN,
                   T_star: float = 5000.0, r_in: float = 10 * AU, K: int = 64,
                   kappa0: float = 1.0, g: float = 0.5, n_t: int = 512,
                   t_min: float = 3.0, t_max: float = 1600.0) -> dict:
    """Log-spaced shells from r_in (an empty cavity inside) to 0.1 pc, rho ~ r_mid^-p."""
    r = np.geomspace(r_in, R_OUT, n + 1)
    rm = 0.5 * (r[1:] + r[:-1])
    shape = rm ** (-p)
    rho = scale_to_tau_V(r, shape, tau_V, kappa0)
    d = synthetic_dust(K, kappa0, g)
    return dict(r_edges=r, rho=rho, **d, t_min=t_min, t_max=t_max, n_t=n_t,
                J=None, L_ps=L, S=blackbody(d["nu"], T_star))


def cfg_external_small() -> dict:
    """Plain IRE, externally heated sphere, 50 shells, central-ray tau_V = 1."""
    return external_sphere(n=50, tau_V=1.0)


def cfg_external_large() -> dict:
    """Externally heated sphere, 101 shells, central tau_V = 10."""
    return external_sphere(n=101, tau_V=10.0)


def cfg_central() -> dict:
    """Central 5000 K, 1 L_sun source, 200 log shells 10 AU - 0.1 pc, tau_V = 100."""
    return central_source()


def gray_model(n: int, tau: float, *, external: bool, kappa: float = 1.0, r_in: float = 0.0,
               K: int = 8, T_src: float = 6000.0) -> dict:
    """Uniform-density, pure-absorption, frequency-independent opacity model for
    closed-form checks; tau is the radial absorption depth."""
    r = np.linspace(r_in, R_OUT, n + 1)
    rho = np.full(n, tau / (kappa * (R_OUT - r_in)))
    nu = frequency_grid(K, 1e12, 1e15)
    d = dict(nu=nu, kabs=np.full(K, kappa), albedo=np.zeros(K), g=np.zeros(K))
    if external:
        return dict(r_edges=r, rho=rho, **d, t_min=3.0, t_max=1600.0, n_t=512,
                    J=1e-14 * blackbody(nu, T_src), L_ps=0.0, S=None)
    return dict(r_edges=r, rho=rho, **d, t_min=3.0, t_max=1600.0, n_t=512,
                J=None, L_ps=LSUN, S=blackbody(nu, T_src))


# ---------------------------------------------------------------------------
# Batched parameter study: 4096 models of uneven size and package budget.

def batch_parameters(n_models: int = 4096, seed: int = 3) -> dict:
    """Per-model parameters drawn with numpy's PCG64:
    shells ~ U{20..400}, tau_V ~ logU(0.1, 1000), density exponent ~ U(0, 2),
    source ~ Bernoulli(0.5) (1 = central), L ~ logU(0.1, 100) L_sun for central
    sources, external-field scale ~ logU(0.1, 100) for external ones,
    packages ~ logU(1e5, 1e7)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = rng.integers(20, 401, size=n_models)
    tau = 10.0 ** rng.uniform(-1.0, 3.0, size=n_models)
    p = rng.uniform(0.0, 2.0, size=n_models)
    central = rng.integers(0, 2, size=n_models)
    L = LSUN * 10.0 ** rng.uniform(-1.0, 2.0, size=n_models)
    s = 10.0 ** rng.uniform(-1.0, 2.0, size=n_models)
    npk = np.floor(10.0 ** rng.uniform(5.0, 7.0, size=n_models)).astype(np.int64)
    L = np.where(central == 1, L, 0.0)
    s = np.where(central == 1, 0.0, s)
    seeds = (np.uint64(seed) << np.uint64(32)) + np.arange(n_models, dtype=np.uint64)
    return dict(n=n.astype(np.int32), tau_V=tau, p=p, central=central.astype(np.int32), L=L,
                field_scale=s, n_pkg=npk, seed=seeds)


def batch_model(params: dict, m: int, K: int = 64) -> dict:
    """Model m of a batched study as a single-model dict."""
    n = int(params["n"][m])
    if params["central"][m]:
        return central_source(n=n, tau_V=float(params["tau_V"][m]), p=float(params["p"][m]),
                              L=float(params["L"][m]), K=K)
    return external_sphere(n=n, tau_V=float(params["tau_V"][m]), p=float(params["p"][m]),
                           field_scale=float(params["field_scale"][m]), K=K)


def surrogate_features(params: dict, m: int, r_edges: np.ndarray) -> np.ndarray:
    """[n, 6] inputs per shell: log10 tau_V, density exponent, log10 L/L_sun (0 for
    external), log10 field scale (0 for central), source type, r_mid / R_out."""
    n = len(r_edges) - 1
    rm = 0.5 * (r_edges[1:] + r_edges[:-1]) / r_edges[-1]
    central = int(params["central"][m])
    f = np.empty((n, 6), dtype=np.float32)
    f[:, 0] = np.log10(params["tau_V"][m])
    f[:, 1] = params["p"][m]
    f[:, 2] = np.log10(params["L"][m] / LSUN) if central else 0.0
    f[:, 3] = 0.0 if central else np.log10(params["field_scale"][m])
    f[:, 4] = central
    f[:, 5] = rm
    return f


def radius_table(n_max: int = 400) -> tuple[np.ndarray, np.ndarray]:
    """Relative shell mid-radii r_mid / R_out of every shell grid of the study:
    for k = 1..n_max shells, the equal-width grid from 0 (external_sphere) and
    the log-spaced grid from 10 AU (central_source), laid end to end.  Returns
    the table and start[2, n_max + 1] (start[g, k] = offset of grid g with k shells)."""
    base = np.zeros(n_max + 2, np.int64)
    np.cumsum(np.arange(n_max + 1), out=base[1:])
    tab = np.empty(2 * int(base[-1]), np.float64)
    for k in range(1, n_max + 1):
        e = np.linspace(0.0, R_OUT, k + 1)
        tab[base[k]:base[k + 1]] = 0.5 * (e[1:] + e[:-1]) / e[-1]
        e = np.geomspace(10 * AU, R_OUT, k + 1)
        tab[base[-1] + base[k]:base[-1] + base[k + 1]] = 0.5 * (e[1:] + e[:-1]) / e[-1]
    start = np.stack([base[:-1], base[:-1] + base[-1]])
    return tab, start


def study_model_inputs(params: dict, models=None) -> dict:
    """Per-model surrogate inputs of a study: model_x [m, 5] float32 (the first
    five columns of surrogate_features), row offsets [m + 1], and per-model
    offsets into the shared radius table (column 5)."""
    idx = np.arange(len(params["n"])) if models is None else np.asarray(models, np.int64)
    n = params["n"][idx].astype(np.int64)
    central = params["central"][idx].astype(np.int64)
    c = central == 1
    x = np.zeros((len(idx), 5), np.float64)
    x[:, 0] = np.log10(params["tau_V"][idx])
    x[:, 1] = params["p"][idx]
    x[c, 2] = np.log10(params["L"][idx][c] / LSUN)
    x[~c, 3] = np.log10(params["field_scale"][idx][~c])
    x[:, 4] = central
    row_off = np.zeros(len(idx) + 1, np.int64)
    np.cumsum(n, out=row_off[1:])
    tab, start = radius_table(int(n.max()) if len(n) else 1)
    return dict(model_x=x.astype(np.float32), row_off=row_off, radius_off=start[central, n],
                radius=tab.astype(np.float32))


def study_features(params: dict, models=None) -> tuple[np.ndarray, np.ndarray]:
    """surrogate_features of many models at once: [rows, 6] float32 and the row
    offsets per model ([len(models) + 1], int64)."""
    q = study_model_inputs(params, models)
    n = np.diff(q["row_off"])
    rows = int(q["row_off"][-1])
    f = np.empty((rows, 6), np.float32)
    f[:, :5] = np.repeat(q["model_x"], n, axis=0)
    local = np.arange(rows, dtype=np.int64) - np.repeat(q["row_off"][:-1], n)
    f[:, 5] = q["radius"][np.repeat(q["radius_off"], n) + local]
    return f, q["row_off"]


def study_shells(params: dict, models=None) -> tuple[np.ndarray, np.ndarray]:
    """Shell radii and densities of many study models at once, as batch_model
    builds them one by one: r_edges of every model end to end ([sum(n + 1)])
    and rho ([sum(n)])."""
    idx = np.arange(len(params["n"])) if models is None else np.asarray(models, np.int64)
    n = params["n"][idx].astype(np.int64)
    central = params["central"][idx].astype(np.int64)
    if len(idx) == 0:
        return np.zeros(0), np.zeros(0)
    # the distinct grids once (linear for external, logarithmic for central
    # sources), then every model's edges gathered from them
    uk, inv = np.unique(n, return_inverse=True)
    tables, g_off, o = [], np.zeros((2, len(uk)), np.int64), 0
    for c in (0, 1):
        for u, k in enumerate(uk):
            g = np.linspace(0.0, R_OUT, k + 1) if c == 0 else np.geomspace(10 * AU, R_OUT, k + 1)
            tables.append(g)
            g_off[c, u] = o
            o += k + 1
    table = np.concatenate(tables)
    cnt = n + 1
    e_off = np.zeros(len(idx), np.int64)
    np.cumsum(cnt[:-1], out=e_off[1:])
    src = np.repeat(g_off[central, inv] - e_off, cnt) + np.arange(int(cnt.sum()))
    r_flat = table[src]
    first = np.zeros(len(r_flat), bool)
    first[e_off] = True
    last = np.zeros(len(r_flat), bool)
    last[e_off + n] = True
    lo, hi = r_flat[~last], r_flat[~first]
    rm = 0.5 * (lo + hi)
    p = np.repeat(params["p"][idx], n)
    cen = np.repeat(central, n) == 1
    shape = np.where(cen, rm ** (-p), (1.0 + (rm / R0_CORE) ** 2) ** (-0.5 * p))
    off = np.zeros(len(idx), np.int64)
    np.cumsum(n[:-1], out=off[1:])
    col = np.add.reduceat(shape * (hi - lo), off) * kappa_ext_V()
    rho = shape * np.repeat(params["tau_V"][idx] / col, n)
    return r_flat, rho
