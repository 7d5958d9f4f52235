"""Statistical comparison of one Monte Carlo run against an ensemble of runs.

A shell's absorbed energy is a sum of package deposits.  Where a shell takes
many deposits per run the sum is close to Gaussian, and a single run lies
within a few ensemble sigmas of the ensemble mean.  Where it takes only a few
(optically thin models, small package budgets) the distribution is discrete
and skewed, and a handful of reference runs neither measures its width
reliably nor bounds its tails.  The check therefore:

  * estimates each shell's sigma as the larger of its own ensemble scatter and
    the median relative scatter of its neighbours (a 16-run standard
    deviation is itself uncertain by ~18 %), widened by sqrt(1 + 1/R) for the
    uncertainty of the R-run mean;
  * asks for |T - <T>| <= max(1 %, 3 sigma) in at least `frac` of the shells;
  * asks for |T - <T>| <= max(1 %, 6 sigma) in every shell in the Gaussian
    regime, i.e. with an effective deposit count (<A> / sigma_A)^2 >= n_eff.

On synthetic compound-Poisson shells (tests/test_mc_stats.py) a run from the
same distribution fails this about once in 1500 comparisons, and a 5 % error
in a single well-sampled shell is always caught.
"""
from __future__ import annotations

import numpy as np


def pooled_sigma(mean, std, half_window: int = 3) -> np.ndarray:
    mean = np.asarray(mean, np.float64)
    std = np.asarray(std, np.float64)
    rel = np.where(mean > 0, std / np.where(mean > 0, mean, 1.0), 0.0)
    n = len(rel)
    med = np.array([np.median(rel[max(0, i - half_window):i + half_window + 1]) for i in range(n)])
    return np.maximum(std, med * mean)


def compare(T, T_mean, T_std, A_mean, A_std, R: int, frac: float = 0.95, rel: float = 0.01,
            n_eff: float = 50.0, k_hard: float = 6.0, name: str = "") -> tuple[bool, float]:
    """(passed, fraction of shells within max(rel, 3 sigma))."""
    T = np.asarray(T, np.float64)
    T_mean = np.asarray(T_mean, np.float64)
    A_mean = np.asarray(A_mean, np.float64)
    A_std = np.asarray(A_std, np.float64)
    sig = pooled_sigma(T_mean, T_std) * np.sqrt(1.0 + 1.0 / R)
    d = np.abs(T - T_mean)
    ok3 = d <= np.maximum(rel * T_mean, 3 * sig)
    gauss = (A_mean > 0) & (A_std > 0) & (A_mean**2 >= n_eff * A_std**2)
    ok5 = (d <= np.maximum(rel * T_mean, k_hard * sig)) | ~gauss
    passed = bool(ok3.mean() >= frac and ok5.all())
    if not passed:
        z = d / np.maximum(sig, 1e-300)
        worst = np.argsort(-z)[:5]
        print(f"{name}: worst shells (index, T, <T>, sigma, n_eff):",
              [(int(i), round(float(T[i]), 4), round(float(T_mean[i]), 4), round(float(sig[i]), 4),
                round(float(A_mean[i] ** 2 / max(A_std[i] ** 2, 1e-300)), 1)) for i in worst])
    return passed, float(ok3.mean())


def compare_runs(T, T_runs, A_runs, **kw) -> tuple[bool, float]:
    """compare() against an ensemble given as [R, n] arrays of T and A."""
    T_runs = np.asarray(T_runs, np.float64)
    A_runs = np.asarray(A_runs, np.float64)
    return compare(T, T_runs.mean(0), T_runs.std(0, ddof=1), A_runs.mean(0), A_runs.std(0, ddof=1),
                   len(T_runs), **kw)


def zero_deposit_failures(A, A_ref_mean, eps, p_max: float = 1e-6) -> list[int]:
    """Shells that took no deposit in the run (A = 0, so T sits at the table's
    floor) although the reference runs make that improbable.  In an unweighted
    run every deposit is one package energy eps, so a shell's deposit count is
    A / eps, close to Poisson with mean lam = <A_ref> / eps, and P(no deposit) =
    exp(-lam).  A shell fails when exp(-lam) < p_max.  (A check that every
    shell with all reference runs above the floor must be above it too would
    fail by chance where lam is a few deposits: with lam = 3 a run misses the
    shell 5 % of the time.)"""
    A = np.asarray(A, np.float64)
    lam = np.asarray(A_ref_mean, np.float64) / eps
    return [int(i) for i in np.nonzero((A == 0.0) & (np.exp(-lam) < p_max))[0]]
