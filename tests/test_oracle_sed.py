"""Pins of the oracle's escaping spectrum (per-source, per-frequency escape
tallies): the unscattered part against the e^-tau transmission of radial rays
computed here, bookkeeping identities, and the re-emitted part of an optically
thin cloud against the re-emission tally."""
import math

import numpy as np

from paper_2408_13807_amd import workloads as wl


def _binomial_ok(k, n, p, nsig=4.5):
    return abs(k - n * p) <= nsig * math.sqrt(n * p * (1 - p)) + 1


def _trapezoid(nu):
    w = np.zeros_like(nu)
    w[1:] += 0.5 * np.diff(nu)
    w[:-1] += 0.5 * np.diff(nu)
    return w


def test_central_direct_sed_is_transmitted_source_spectrum(orc):
    m = wl.central_source(n=30, tau_V=1.0, p=1.0)
    N = 400_000
    r = orc.run(m, n_ps=N, seed=21, sed=True)
    nu = m["nu"]
    q = m["S"] * _trapezoid(nu)
    q = q / q.sum()                                   # launch probability per frequency
    kext = m["kabs"] / (1 - m["albedo"])
    tau = kext * np.sum(m["rho"] * np.diff(m["r_edges"]))
    eps = m["L_ps"] / N
    counts = r["sed_direct"][1] / eps
    for k in range(len(nu)):
        assert _binomial_ok(counts[k], N, q[k] * math.exp(-tau[k])), (k, counts[k], N * q[k] * math.exp(-tau[k]))
    assert np.all(r["sed_direct"][0] == 0) and np.all(r["sed"][0] == 0)


def test_sed_sums_to_escaped_power(orc):
    m = dict(wl.cfg_external_small(), L_ps=wl.LSUN, S=wl.blackbody(wl.frequency_grid(), 5000.0))
    for opts in ({}, dict(ffi=1), dict(k_bg=0.3, k_A=1.5)):
        r = orc.run(m, n_ext=20_000, n_ps=20_000, seed=3, sed=True, **opts)
        s = r["stats"]
        ffi = s["ffi_escaped"]
        total = r["sed"].sum()
        assert abs(total - (sum(s["escaped"]) + ffi)) <= 1e-12 * total
        assert np.all(r["sed"] >= r["sed_direct"] - 1e-300)


def test_thin_cloud_reemission_escapes(orc):
    # optically thin and purely absorbing: re-emitted packages escape without
    # further events, so the escaping non-direct spectrum is the re-emission tally
    m = wl.central_source(n=10, tau_V=1e-3, p=1.0)
    m["albedo"] = np.zeros(64)
    r = orc.run(m, n_ps=200_000, seed=4, sed=True, reemit=True)
    dust = r["sed"][1] - r["sed_direct"][1]
    re = r["reemit"].sum(axis=0)
    assert abs(dust.sum() / re.sum() - 1) < 5e-3
    big = re > 1e-3 * re.max()
    assert np.allclose(dust[big], re[big], rtol=0.02)
