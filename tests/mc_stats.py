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
    regime, i.e. with an effective deposit count (<A> / sigma_A)^2 >= n_eff;
  * with an ensemble of runs at hand (compare_runs), asks that the run's
    signed z-scores follow the distribution of the reference runs' own
    leave-one-out z-scores (two-sample Kolmogorov-Smirnov, p >= 1e-6), so a
    shift of many shells by a fraction of a sigma also fails.

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
    # median over the window [i - half_window, i + half_window], cut at the ends
    pad = np.full(len(rel) + 2 * half_window, np.nan)
    pad[half_window:half_window + len(rel)] = rel
    med = np.nanmedian(np.lib.stride_tricks.sliding_window_view(pad, 2 * half_window + 1), axis=1)
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


# (comparison name, p-value) of every z-score distribution test of the session
KS_PVALUES: list[tuple[str, float]] = []


def z_scores(T, T_mean, T_std, R: int) -> np.ndarray:
    """Signed per-shell deviations in units of compare()'s sigma, over the
    shells whose sigma is not zero."""
    sig = pooled_sigma(T_mean, T_std) * np.sqrt(1.0 + 1.0 / R)
    live = sig > 0
    return ((np.asarray(T, np.float64) - T_mean) / np.where(live, sig, 1.0))[live]


def z_shift_pvalue(T, T_runs) -> float:
    """p-value of a two-sample Kolmogorov-Smirnov test of the run's z-scores
    against a null drawn from the reference runs themselves: each reference
    run's z-scores against the other R-1 runs.  The null therefore has the
    same discreteness, skew and shell-to-shell correlation as the run's own
    z-scores would if the run came from the reference distribution, and a
    systematic shift or widening over many shells (each one too small for the
    per-shell rules) moves the run's z-scores away from it."""
    from scipy.stats import ks_2samp, kstwobign
    T_runs = np.asarray(T_runs, np.float64)
    R = len(T_runs)
    z = z_scores(T, T_runs.mean(0), T_runs.std(0, ddof=1), R)
    null = []
    for k in range(R):
        rest = np.delete(T_runs, k, axis=0)
        null.append(z_scores(T_runs[k], rest.mean(0), rest.std(0, ddof=1), R - 1))
    if len(z) == 0 or min(len(x) for x in null) == 0:
        return 1.0
    D = ks_2samp(z, np.concatenate(null)).statistic
    # Neighbouring shells share packages, so their z-scores are correlated and
    # the statistic spreads wider than the Kolmogorov law for independent
    # samples gives.  Its scale is therefore measured on the null itself: each
    # reference run's distance from the pool of the others, whose median sets
    # the effective sample size (the Kolmogorov law's median is 0.8276).
    Dk = [ks_2samp(null[k], np.concatenate(null[:k] + null[k + 1:])).statistic for k in range(R)]
    med = float(np.median(Dk))
    if med <= 0:
        return 1.0 if D <= 0 else 0.0
    return float(kstwobign.sf(D * kstwobign.median() / med))


def compare_runs(T, T_runs, A_runs, ks_alpha: float = 1e-6, **kw) -> tuple[bool, float]:
    """compare() against an ensemble given as [R, n] arrays of T and A, and the
    z-score distribution test (z_shift_pvalue) at level ks_alpha."""
    T_runs = np.asarray(T_runs, np.float64)
    A_runs = np.asarray(A_runs, np.float64)
    ok, f = compare(T, T_runs.mean(0), T_runs.std(0, ddof=1), A_runs.mean(0), A_runs.std(0, ddof=1),
                    len(T_runs), **kw)
    if ks_alpha > 0:
        p = z_shift_pvalue(T, T_runs)
        KS_PVALUES.append((kw.get("name", ""), p))
        if p < ks_alpha:
            print(f"{kw.get('name', '')}: z-scores differ in distribution from the reference runs' own "
                  f"(KS p = {p:.2e})")
            ok = False
    return ok, f


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
