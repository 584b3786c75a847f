"""Host-side analysis of Monte Carlo time series (chains' per-sweep observables).

* Autocorrelation A_O(t) of the supplement's section I.3 (eq. (5)): the covariance of O at sweeps
  i and i + t over the variance of O, averages over the reference time i.  For many independent
  chains the numerator and denominator are averaged over chains too, with one common mean.
* Integrated autocorrelation time tau = 1/2 + sum_{t >= 1} A(t), summed up to the first t where A
  drops below zero (a self-consistent window would do as well at these lengths).
* Convergence curve: the chain average of O after each sweep (the paper's Fig. 3 form).
* Percentage overlap of two histograms over a common range in a fixed number of bins
  (%OL = sum_i min(P_r(i), P_theta(i)), main text, with 20 bins).
* Standard error of the mean over independent chains, and over bins of one long chain.
"""
from __future__ import annotations

from typing import Tuple

import numpy as np


def autocorrelation(series: np.ndarray, t_max: int) -> np.ndarray:
    """A(t) for t = 0 .. t_max of series [chains][time] (or [time])."""
    x = np.asarray(series, dtype=np.float64)
    if x.ndim == 1:
        x = x[None]
    n = x.shape[1]
    t_max = min(int(t_max), n - 1)
    mean = x.mean()
    var = (x * x).mean() - mean * mean
    out = np.empty(t_max + 1)
    for t in range(t_max + 1):
        out[t] = ((x[:, : n - t] * x[:, t:]).mean() - mean * mean) / var
    return out


def integrated_time(a: np.ndarray) -> float:
    """1/2 + sum of A(t) for t >= 1 up to the first negative value."""
    tau = 0.5
    for v in a[1:]:
        if v < 0:
            break
        tau += float(v)
    return tau


def convergence_curve(series: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Mean over chains after each sweep and its standard error, series [chains][time]."""
    x = np.asarray(series, dtype=np.float64)
    return x.mean(0), x.std(0, ddof=1) / np.sqrt(x.shape[0])


def percent_overlap(a: np.ndarray, b: np.ndarray, bins: int = 20, value_range=None) -> float:
    """sum_i min(P_a(i), P_b(i)) of the two normalised histograms on a common binning."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    if value_range is None:
        value_range = (min(a.min(), b.min()), max(a.max(), b.max()))
    pa, _ = np.histogram(a, bins=bins, range=value_range)
    pb, _ = np.histogram(b, bins=bins, range=value_range)
    return float(np.minimum(pa / pa.sum(), pb / pb.sum()).sum())


def mean_and_error(per_chain: np.ndarray) -> Tuple[float, float]:
    """Mean over independent chains and its standard error."""
    v = np.asarray(per_chain, dtype=np.float64)
    return float(v.mean()), float(v.std(ddof=1) / np.sqrt(len(v)))


def binned_error(series: np.ndarray, n_bins: int) -> Tuple[float, float]:
    """Mean of one long series and the standard error from n_bins consecutive bin means."""
    x = np.asarray(series, dtype=np.float64).ravel()
    m = len(x) // n_bins
    bm = x[: m * n_bins].reshape(n_bins, m).mean(1)
    return float(x.mean()), float(bm.std(ddof=1) / np.sqrt(n_bins))
