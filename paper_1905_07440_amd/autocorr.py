"""Autocorrelation of a Monte Carlo time series by binning (host-side
analysis of observables read through the C ABI).

The paper compares samplers by the autocorrelation time tau_L of the CDW
structure factor S_CDW(pi, pi) (Benchmarks; the autocorrelation figure and
its n_u inset) without fixing an estimator.  Here: the integrated
autocorrelation time tau_int = 1/2 + sum_{t >= 1} rho(t), so that the variance
of the mean of n correlated samples is var(x) 2 tau_int / n, estimated by
binning: the means of bins of B consecutive samples have variance
var(x) 2 tau_int / B once B >> tau_int, so

    tau_B = (B var(bin means) / var(x) - 1) / 2 + 1/2 = B var(bin means) / (2 var(x))

rises with B to a plateau at tau_int.  The estimate is tau_B at the largest B
that still leaves `min_bins` bins.  Uncorrelated samples give 1/2.
"""
import numpy as np


def binning_curve(x, min_bins=64):
    """(B, tau_B) for B = 1, 2, 4, ... while at least min_bins bins remain."""
    x = np.asarray(x, dtype=np.float64)
    if x.ndim != 1 or x.size < 2 * min_bins:
        raise ValueError("need a 1-D series of at least %d samples" % (2 * min_bins))
    var = x.var()
    if not var > 0.0:
        raise ValueError("the series is constant")
    out = []
    B = 1
    while x.size // B >= min_bins:
        nb = x.size // B
        means = x[:nb * B].reshape(nb, B).mean(axis=1)
        out.append((B, B * means.var() / (2.0 * var)))
        B *= 2
    return out


def tau_int(x, min_bins=64):
    """Integrated autocorrelation time of one series (in samples)."""
    return binning_curve(x, min_bins)[-1][1]


def tau_int_chains(series, min_bins=64):
    """tau_int of several independent chains' series ([chains][samples]):
    the binned variances are averaged over chains before the ratio."""
    s = np.asarray(series, dtype=np.float64)
    if s.ndim != 2:
        raise ValueError("need [chains][samples]")
    n = s.shape[1]
    if n < 2 * min_bins:
        raise ValueError("need at least %d samples per chain" % (2 * min_bins))
    var = s.var(axis=1).mean()
    if not var > 0.0:
        raise ValueError("the series are constant")
    B = 1
    tau = 0.5
    while n // B >= min_bins:
        nb = n // B
        means = s[:, :nb * B].reshape(s.shape[0], nb, B).mean(axis=2)
        tau = B * means.var(axis=1).mean() / (2.0 * var)
        B *= 2
    return tau
