"""Pins of two rarely taken branches of the oracle: the weight floor
(Sect. 2.2.1: a package whose weight has fallen ten orders of magnitude, here
w_floor times its weight after launch, is stopped) and the re-emission of an
absorption whose slice point lies above the last point of the temperature
table (reading R7: the frequency is drawn from the last bin, and the draw is
counted).

The floor is pinned by a cloud where it decides at a known rate: a purely
absorbing gray sphere, one event per package (max_events = 1), and
re-emission cosines from HG(g_E) (Eq. 6), whose weight factor
0.5 / HG(mu') depends on the drawn cosine alone.  The package is stopped when
that factor is below w_floor, i.e. when HG(mu') > 0.5 / w_floor: a cosine
above a threshold mu_c that follows from the HG density in closed form.  The
stopped fraction, the power those packages carry, and the relation to the
launch weight (k_bg = 0.2 makes the launch weights differ widely) follow.

The clamp is pinned by a single shell heated by a central source: its running
total grows by the package energy eps at every absorption, so the absorptions
whose slices lie wholly below G(t_max) M are exactly the first
J = floor(G(t_max) M / eps); the next one straddles; every later one is above
the table.  The re-emitted spectrum is then the telescoped one up to t_max plus
the last bin's difference spectrum for the rest.
"""
import math

import numpy as np
import pytest
from scipy import integrate, stats

from paper_2408_13807_amd import workloads as wl


def hg_pdf(g, mu):
    return 0.5 * (1 - g * g) / (1 + g * g - 2 * g * mu) ** 1.5


def hg_cdf(g, mu):
    # cumulative law of the HG cosine (integral of hg_pdf from -1 to mu)
    return (1 - g * g) / (2 * g) * (1 / math.sqrt(1 + g * g - 2 * g * mu) - 1 / (1 + g))


def floor_threshold(g, w_floor):
    """mu_c with HG(mu_c) = 0.5 / w_floor: weight factors 0.5/HG(mu') below w_floor are cosines above mu_c."""
    c = 0.5 / w_floor
    return (1 + g * g - (0.5 * (1 - g * g) / c) ** (2.0 / 3.0)) / (2 * g)


G_E, W_FLOOR = 0.5, 0.5
FLOOR_OPTS = dict(use_g_E=1, g_E=G_E, w_floor=W_FLOOR, max_events=1)


def floor_model():
    return wl.gray_model(10, 2.0, external=True)


def test_threshold_closed_form():
    mu_c = floor_threshold(G_E, W_FLOOR)
    assert -1 < mu_c < 1
    assert abs(hg_pdf(G_E, mu_c) - 0.5 / W_FLOOR) < 1e-12
    # the cumulative law is the integral of the density
    assert abs(hg_cdf(G_E, mu_c) - integrate.quad(lambda x: hg_pdf(G_E, x), -1, mu_c)[0]) < 1e-10


@pytest.mark.parametrize("k_bg", [0.5, 0.2])
def test_weight_floor_stops_the_predicted_fraction(orc, k_bg):
    # one event per package: the first (absorption) event re-emits with weight
    # factor 0.5/HG(mu'); packages stopped there are the floor's, later events
    # would be the max_events limit's.  The fraction is relative to the launch
    # weight: with k_bg = 0.2 the launch weights range over (0.4, inf), and a
    # floor taken against weight 1 would stop a different share.
    N = 60_000
    r = orc.run(floor_model(), n_ext=N, seed=5, k_bg=k_bg, **FLOOR_OPTS)
    s = r["stats"]
    p = 1 - hg_cdf(G_E, floor_threshold(G_E, W_FLOOR))
    n = s["n_abs"]
    assert s["n_floor"] > 0
    assert abs(s["n_floor"] - n * p) <= 4.5 * math.sqrt(n * p * (1 - p)) + 1, (s["n_floor"], n * p)
    # every package ends in exactly one way
    assert s["n_escape"] + s["n_limit"] + s["n_floor"] == N
    assert s["terminated_floor"] > 0 and s["terminated"] >= s["terminated_floor"]


def test_weight_floor_tallies_the_stopped_power(orc):
    # unit launch weights: each absorbed package deposits eps, and a stopped one
    # carries eps * 0.5/HG(mu') into `terminated`; its expectation per absorbed
    # package is eps * int_{mu_c}^1 (0.5/HG) HG dmu = eps * 0.5 (1 - mu_c)
    N = 60_000
    m = floor_model()
    r = orc.run(m, n_ext=N, seed=6, **FLOOR_OPTS)
    s = r["stats"]
    eps = s["L_ext"] / N
    n = s["n_abs"]
    assert abs(r["A"].sum() / (n * eps) - 1) < 1e-12
    mu_c = floor_threshold(G_E, W_FLOOR)
    ey = 0.5 * (1 - mu_c)
    ey2 = integrate.quad(lambda x: 0.25 / hg_pdf(G_E, x), mu_c, 1)[0]
    sd = math.sqrt(n * (ey2 - ey * ey))
    assert abs(s["terminated_floor"] / eps - n * ey) <= 4.5 * sd, (s["terminated_floor"] / eps, n * ey, sd)


def test_weighted_energy_balance_with_floor(orc):
    # weighted runs conserve energy in expectation only: over 16 seeds the mean
    # of escaped + stopped power equals the source luminosity within 4 standard
    # errors.  Without an event limit every stopped package is the floor's.
    m = floor_model()
    out = []
    for seed in range(1, 17):
        s = orc.run(m, n_ext=5000, seed=seed, k_bg=0.2, use_g_E=1, g_E=G_E, w_floor=W_FLOOR)["stats"]
        assert s["n_floor"] > 0 and s["n_limit"] == 0
        assert s["terminated"] == s["terminated_floor"]
        assert s["n_escape"] + s["n_floor"] == 5000
        out.append((sum(s["escaped"]) + s["terminated"]) / s["L_ext"])
    out = np.array(out)
    assert abs(out.mean() - 1) <= 4 * out.std(ddof=1) / 4


# ---------------------------------------------------------------------------
# Re-emission above the temperature table

def trapezoid(nu):
    w = np.empty_like(nu)
    w[1:-1] = 0.5 * (nu[2:] - nu[:-2])
    w[0], w[-1] = 0.5 * (nu[1] - nu[0]), 0.5 * (nu[-1] - nu[-2])
    return w


def shell_mass_and_gmax(m):
    """Mass of the single shell and G(t_max) = 4 pi sum_k kappa_k B_k(t_max) w_k, from their definitions."""
    r0, r1 = m["r_edges"]
    M = m["rho"][0] * 4.0 / 3.0 * math.pi * (r1**3 - r0**3)
    G = 4 * math.pi * np.sum(m["kabs"] * wl.blackbody(m["nu"], m["t_max"]) * trapezoid(m["nu"]))
    return M, G


def clamp_model():
    m = wl.cfg_central()
    return dict(m, r_edges=m["r_edges"][[0, -1]], rho=np.array([m["rho"].mean()]), t_min=3.0, t_max=5.0, n_t=8)


def test_reemission_above_table_counts(orc):
    m = clamp_model()
    N = 5000
    r = orc.run(m, n_ps=N, seed=8, reemit=True)
    s = r["stats"]
    eps = m["L_ps"] / N
    M, Gmax = shell_mass_and_gmax(m)
    J = math.floor(Gmax * M / eps)
    assert 0 < J < s["n_abs"]
    # absorptions 1..J lie below G(t_max) M, absorption J+1 straddles it, all later ones are above
    assert s["n_abs"] - J - 1 <= s["n_reemit_above"] <= s["n_abs"] - J, (s["n_reemit_above"], s["n_abs"], J)
    # the final temperature is clamped to t_max and counted
    assert r["T"][0] == m["t_max"] and s["n_above"] == 1


def test_reemission_above_table_spectrum(orc):
    # Expected re-emitted spectrum of the shell: the slices below G(t_max) M tile
    # [0, G(t_max) M] and telescope to 4 pi M kappa B(t_max) w; the rest of the
    # absorbed power, A - G(t_max) M, is re-emitted from the last bin's
    # difference spectrum kappa [B(T_last) - B(T_prev)] w.
    m = clamp_model()
    N = 20000
    r = orc.run(m, n_ps=N, seed=9, reemit=True)
    eps = m["L_ps"] / N
    M, Gmax = shell_mass_and_gmax(m)
    nu, w, kap = m["nu"], trapezoid(m["nu"]), m["kabs"]
    T_prev = m["t_min"] * (m["t_max"] / m["t_min"]) ** ((m["n_t"] - 2) / (m["n_t"] - 1))
    last = kap * (wl.blackbody(nu, m["t_max"]) - wl.blackbody(nu, T_prev)) * w
    below = 4 * math.pi * M * kap * wl.blackbody(nu, m["t_max"]) * w
    expect = below + (r["A"][0] - Gmax * M) * last / last.sum()
    got = r["reemit"][0]
    assert abs(got.sum() / r["A"][0] - 1) < 1e-12
    # counts of re-emitted packages per frequency (each re-emission carries eps)
    obs, exp = got / eps, expect / eps
    keep = exp > 5
    chi2 = np.sum((obs[keep] - exp[keep]) ** 2 / exp[keep])
    assert stats.chi2.sf(chi2, keep.sum() - 1) > 1e-4, chi2
    # without the clamp the spectrum would be far hotter: the last bin is what the draw used
    assert abs(obs[keep].sum() - exp[keep].sum()) / exp[keep].sum() < 0.02
