"""Exact results the oracle is pinned against (closed forms, enumeration,
dynamic programming).  None of these reuse the oracle's sampler.

Ensemble (Sec. II.C, Eq. pi_vcsgc, with kappa per site):
    pi(sigma) ~ exp[-beta (U + phi n + (kappa/N) n^2)],  phi = dmu0 - 2 kappa cbar.
SGC is kappa = 0 with phi = dmu (Eq. pi_sgc_orig).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import gammaln, logsumexp

KB = 8.617333262e-5


def beta_of(T):
    return 1.0 / (KB * T)


def ideal_sgc_c(T, dmu):
    """Identical species, SGC: each site independently B with 1/(1+exp(beta dmu))."""
    return 1.0 / (1.0 + math.exp(beta_of(T) * dmu))


def vcsgc_logw_ideal(N, T, dmu0, kappa, cbar):
    """log P(n) + const for identical species: C(N, n) exp[-beta(phi n + kappa n^2/N)]."""
    b = beta_of(T)
    phi = dmu0 - 2.0 * kappa * cbar
    n = np.arange(N + 1, dtype=np.float64)
    logc = gammaln(N + 1.0) - gammaln(n + 1.0) - gammaln(N - n + 1.0)
    return logc - b * (phi * n + kappa * n * n / N)


def normalize(logw):
    return np.exp(logw - logsumexp(logw))


def moments(p):
    n = np.arange(p.size, dtype=np.float64)
    m1 = float((p * n).sum())
    m2 = float((p * n * n).sum())
    return m1, m2 - m1 * m1


def log_esp(w_log):
    """log of the elementary symmetric polynomials e_0..e_N of exp(w_log),
    by the O(N^2) recursion e_k <- e_k + w e_{k-1} (Poisson-binomial DP)."""
    N = w_log.size
    e = np.full(N + 1, -np.inf)
    e[0] = 0.0
    for k, lw in enumerate(w_log):
        shifted = e[:k + 1] + lw
        e[1:k + 2] = np.logaddexp(e[1:k + 2], shifted)
    return e


def vcsgc_logw_indep(site_de, T, dmu0, kappa, cbar):
    """Independent sites with energy site_de[i] for species B relative to A:
    P(n) ~ e_n(exp(-beta site_de)) exp[-beta(phi n + kappa n^2 / N)]."""
    b = beta_of(T)
    N = site_de.size
    phi = dmu0 - 2.0 * kappa * cbar
    n = np.arange(N + 1, dtype=np.float64)
    return log_esp(-b * site_de) - b * (phi * n + kappa * n * n / N)


def batch_means(series, n_batches=20):
    """Mean and its standard error from non-overlapping batch means."""
    s = np.asarray(series, dtype=np.float64)
    m = s.size // n_batches
    bm = s[: m * n_batches].reshape(n_batches, m).mean(axis=1)
    return float(bm.mean()), float(bm.std(ddof=1) / math.sqrt(n_batches))


def lattice_shells(a):
    """bcc shells inside 3.6 A: (count, distance)."""
    return [(8, a * math.sqrt(3.0) / 2.0), (6, a)]


def batch_variance(series, n_batches=20):
    """Variance about the whole series' mean and its standard error from
    non-overlapping batches (each batch's mean square deviation)."""
    s = np.asarray(series, dtype=np.float64)
    m = s.size // n_batches
    dev2 = (s[: m * n_batches] - s[: m * n_batches].mean()) ** 2
    bv = dev2.reshape(n_batches, m).mean(axis=1)
    return float(bv.mean()), float(bv.std(ddof=1) / math.sqrt(n_batches))
