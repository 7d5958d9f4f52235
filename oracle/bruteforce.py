"""Deterministic solution of a small purely absorbing cloud (test infrastructure).

Used to pin the whole IRE oracle on clouds of a few shells.  With isotropic
re-emission spread uniformly over each shell's volume (the variant of Sect. 4
that randomises the re-emission position), the equilibrium of the immediate
re-emission method is the solution of

    A_i = S_i + sum_j sum_k E_jk P_{j->i,k},   E_jk = 4 pi M_j kappa_k B_k(T_j) w_k,
    A_j = M_j G(T_j),

where S_i is the first absorption of the source power in shell i and
P_{j->i,k} the probability that a package emitted at frequency k uniformly in
shell j, isotropically, is first absorbed in shell i.  The probabilities are
computed here by Gauss-Legendre quadrature over the emission radius (r^2
weighting) and direction cosine, tracing each ray through the spherical
boundaries; the equation is solved by fixed-point iteration on the shell
temperatures.  Everything is FP64 numpy, independent of the oracle's code.
"""
from __future__ import annotations

import numpy as np
from scipy import optimize

H, KB, C = 6.62607015e-27, 1.380649e-16, 2.99792458e10


def planck(nu, T):
    nu = np.asarray(nu, np.float64)
    if T <= 0:
        return np.zeros_like(nu)
    x = H * nu / (KB * T)
    out = np.zeros_like(nu)
    ok = x < 700
    out[ok] = 2 * H * nu[ok] ** 3 / C**2 / np.expm1(x[ok])
    return out


def trapezoid(nu):
    w = np.zeros_like(nu)
    w[1:] += 0.5 * np.diff(nu)
    w[:-1] += 0.5 * np.diff(nu)
    return w


def _ray_deposits(r_edges, chi_k, r0, mu):
    """First-absorption probabilities per shell (and escape) for rays starting at
    radii r0 with direction cosines mu, for every frequency (chi_k: [n, K]
    absorption coefficient per shell)."""
    n = len(r_edges) - 1
    R = np.asarray(r_edges, np.float64)
    b2 = r0**2 * (1 - mu**2)
    t0 = r0 * mu
    t_exit = np.sqrt(np.maximum(R[-1] ** 2 - b2, 0))
    # boundary crossings of the ray: t = +-sqrt(R_m^2 - b^2) for every sphere with R_m^2 > b^2
    cand = []
    for Rm in R:
        s = np.sqrt(np.maximum(Rm**2 - b2, 0.0))
        hit = Rm**2 > b2
        cand.append(np.where(hit, s, np.nan))
        cand.append(np.where(hit, -s, np.nan))
    T = np.stack(cand, axis=1)
    T = np.where((T > t0[:, None]) & (T <= t_exit[:, None]), T, np.nan)
    T = np.concatenate([t0[:, None], T], axis=1)
    T = np.sort(T, axis=1)                         # NaN last
    seg_len = np.diff(T, axis=1)
    tm = 0.5 * (T[:, 1:] + T[:, :-1])
    rm = np.sqrt(b2[:, None] + tm**2)
    shell = np.clip(np.searchsorted(R, rm) - 1, 0, n - 1)
    valid = np.isfinite(seg_len) & (seg_len > 0) & (rm >= R[0]) & (rm <= R[-1])
    seg_len = np.where(valid, seg_len, 0.0)
    K = chi_k.shape[1]
    dep = np.zeros((len(r0), n, K))
    tau = np.zeros((len(r0), K))
    for s in range(seg_len.shape[1]):
        dt = chi_k[shell[:, s]] * seg_len[:, s][:, None]   # [rays, K]
        p = np.exp(-tau) * -np.expm1(-dt)
        np.add.at(dep, (np.arange(len(r0)), shell[:, s]), p * valid[:, s][:, None])
        tau = tau + dt
    return dep, np.exp(-tau)


def transfer_matrix(r_edges, chi_k, n_r=48, n_mu=384):
    """P[j, i, k]: emitted uniformly in shell j, isotropically, first absorbed in shell i."""
    n = len(r_edges) - 1
    xr, wr = np.polynomial.legendre.leggauss(n_r)
    xm, wm = np.polynomial.legendre.leggauss(n_mu)
    P = np.zeros((n, n, chi_k.shape[1]))
    for j in range(n):
        a, b = r_edges[j], r_edges[j + 1]
        r = 0.5 * (b - a) * xr + 0.5 * (b + a)
        w_r = 0.5 * (b - a) * wr * r**2
        w_r = w_r / w_r.sum()
        rr, mm = np.meshgrid(r, xm, indexing="ij")
        ww = (w_r[:, None] * (0.5 * wm)[None, :]).ravel()
        dep, _ = _ray_deposits(r_edges, chi_k, rr.ravel(), mm.ravel())
        P[j] = np.einsum("r,rik->ik", ww, dep)
    return P


def central_first_deposits(r_edges, chi_k, L_k):
    """Source power first absorbed per shell for a point source at the centre (radial rays)."""
    dtau = chi_k * np.diff(r_edges)[:, None]
    cum = np.concatenate([np.zeros((1, chi_k.shape[1])), np.cumsum(dtau, axis=0)])
    return ((np.exp(-cum[:-1]) - np.exp(-cum[1:])) * L_k[None, :]).sum(axis=1)


def solve_central(model: dict, tol: float = 1e-12, max_iter: int = 500) -> dict:
    """Equilibrium temperatures of a purely absorbing cloud heated by its central source."""
    r = np.asarray(model["r_edges"], np.float64)
    rho = np.asarray(model["rho"], np.float64)
    nu = np.asarray(model["nu"], np.float64)
    kap = np.asarray(model["kabs"], np.float64)
    assert np.all(np.asarray(model["albedo"]) == 0), "pure absorption only"
    w = trapezoid(nu)
    chi = rho[:, None] * kap[None, :]
    M = rho * 4 / 3 * np.pi * (r[1:] ** 3 - r[:-1] ** 3)
    S = np.asarray(model["S"], np.float64) * w
    L_k = model["L_ps"] * S / S.sum()
    src = central_first_deposits(r, chi, L_k)
    P = transfer_matrix(r, chi)

    def G(T):
        return 4 * np.pi * np.sum(kap * planck(nu, T) * w)

    def T_of(a):
        return optimize.brentq(lambda T: G(T) - a, 1e-3, 1e5, xtol=1e-14, rtol=1e-14) if a > 0 else 0.0

    A = src.copy()
    for _ in range(max_iter):
        T = np.array([T_of(A[i] / M[i]) for i in range(len(M))])
        E = 4 * np.pi * M[:, None] * kap[None, :] * np.stack([planck(nu, t) for t in T]) * w[None, :]
        A_new = src + np.einsum("jk,jik->i", E, P)
        if np.max(np.abs(A_new / A - 1)) < tol:
            A = A_new
            break
        A = A_new
    T = np.array([T_of(A[i] / M[i]) for i in range(len(M))])
    return dict(A=A, T=T, source_deposit=src, P=P)
