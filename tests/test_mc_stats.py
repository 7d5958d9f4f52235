"""The ensemble criterion of mc_stats on synthetic compound-Poisson shells:
rare false alarms for runs from the same distribution, and certain detection
of a 3 % bias."""
import numpy as np

import mc_stats


def draw(rng, lam, runs):
    """Absorbed energy per shell: Poisson(lam) deposits of Exp(1) energy; T from
    A^(1/5.8) with a floor, as for dust with kappa ~ nu^1.8."""
    n = rng.poisson(lam, size=(runs, len(lam)))
    A = rng.gamma(np.maximum(n, 1), 1.0) * (n > 0)
    T = np.maximum(30.0 * (A / np.maximum(lam, 1e-9)) ** (1 / 5.8), 3.0)
    return T, A


def test_false_alarm_rate_is_small():
    rng = np.random.default_rng(5)
    lam = 10 ** rng.uniform(-0.3, 4, size=200)
    fails = 0
    for _ in range(400):
        T, A = draw(rng, lam, 17)
        ok, _ = mc_stats.compare_runs(T[0], T[1:], A[1:])
        fails += not ok
    assert fails <= 3, fails


def test_detects_three_percent_bias():
    rng = np.random.default_rng(6)
    lam = 10 ** rng.uniform(-0.3, 4, size=200)
    for _ in range(50):
        T, A = draw(rng, lam, 17)
        ok, _ = mc_stats.compare_runs(1.03 * T[0], T[1:], A[1:])
        assert not ok


def test_detects_one_wrong_well_sampled_shell():
    rng = np.random.default_rng(7)
    lam = np.full(100, 5000.0)
    T, A = draw(rng, lam, 17)
    t = T[0].copy()
    t[40] *= 1.05
    assert mc_stats.compare_runs(T[0], T[1:], A[1:])[0]
    assert not mc_stats.compare_runs(t, T[1:], A[1:])[0]


def test_pooled_sigma_uses_neighbours():
    mean = np.full(9, 10.0)
    std = np.array([1, 1, 1, 1, 0.01, 1, 1, 1, 1.0])
    s = mc_stats.pooled_sigma(mean, std)
    assert s[4] == 1.0 and np.all(s >= std)


def test_zero_deposit_check():
    rng = np.random.default_rng(3)
    eps = 2.5
    lam = np.array([0.5, 3.0, 8.0, 20.0, 200.0])
    # runs drawn from the reference distribution: misses only where exp(-lam) is not tiny
    for _ in range(200):
        A = rng.poisson(lam) * eps
        assert mc_stats.zero_deposit_failures(A, lam * eps, eps) == []
    # a well-hit shell left at zero fails
    A = rng.poisson(lam) * eps
    A[3] = 0.0
    assert mc_stats.zero_deposit_failures(A, lam * eps, eps) == [3]


def draw_correlated(rng, lam, runs, w=8):
    """As draw(), with every deposit shared by w neighbouring shells (packages
    that cross several shells), so neighbouring shells' values correlate."""
    lp = np.concatenate([lam, lam[:w]])
    n = rng.poisson(lp / w, size=(runs, len(lam) + w))
    n = np.stack([n[:, i:i + len(lam)] for i in range(w)]).sum(0)
    A = rng.gamma(np.maximum(n, 1), 1.0) * (n > 0)
    T = np.maximum(30.0 * (A / np.maximum(lam, 1e-9)) ** (1 / 5.8), 3.0)
    return T, A


def test_z_distribution_test_null_calibration():
    # runs from the reference distribution, independent or correlated shells:
    # the z-score test stays far from its 1e-6 level
    rng = np.random.default_rng(12)
    lam = 10 ** rng.uniform(-0.3, 4, size=200)
    for drawer in (draw, draw_correlated):
        p = [mc_stats.z_shift_pvalue(T[0], T[1:]) for T, _ in (drawer(rng, lam, 17) for _ in range(150))]
        assert min(p) > 1e-5, (drawer.__name__, min(p))
        assert 0.2 < np.median(p) < 0.9, (drawer.__name__, np.median(p))


def test_detects_a_shift_the_per_shell_rules_pass():
    # every shell moved by one sigma: within the 95 % / 6 sigma rules, caught
    # by the z-score distribution
    rng = np.random.default_rng(13)
    lam = 10 ** rng.uniform(1, 4, size=300)
    caught = 0
    for _ in range(20):
        T, A = draw(rng, lam, 17)
        t = T[0] + T[1:].std(0, ddof=1)
        assert mc_stats.compare_runs(t, T[1:], A[1:], ks_alpha=0)[0]
        caught += not mc_stats.compare_runs(t, T[1:], A[1:])[0]
    assert caught == 20
