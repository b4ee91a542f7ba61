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
that still leaves `min_bins` bins; it is reported as converged only when
tau_B has stopped rising (tau_B / tau_{B/2} - 1 below `plateau_tol`), and
otherwise as a lower bound.  Uncorrelated samples give 1/2.

A series whose spread is at the rounding level of its values is constant
(a chain that never moves): numpy's variance of identical doubles need not
be exactly zero, so the test is against (64 eps |mean|)^2.
"""
import numpy as np

EPS = np.finfo(np.float64).eps


def _constant(x, axis=None):
    """Whether the values (of each chain) are equal up to rounding."""
    x = np.asarray(x, dtype=np.float64)
    ptp = np.ptp(x, axis=axis)
    var = x.var(axis=axis)
    scale = 64.0 * EPS * np.abs(x.mean(axis=axis))
    return (ptp == 0.0) | (var <= scale * scale)


def binning_curve(x, min_bins=64):
    """(B, tau_B) for B = 1, 2, 4, ... while at least min_bins bins remain."""
    x = np.asarray(x, dtype=np.float64)
    if x.ndim != 1 or x.size < 2 * min_bins:
        raise ValueError("need a 1-D series of at least %d samples" % (2 * min_bins))
    if _constant(x):
        raise ValueError("the series is constant")
    var = x.var()
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


def binning_curve_chains(series, min_bins=64):
    """(B, tau_B) of several independent chains' series ([chains][samples]):
    the binned variances are averaged over chains before the ratio.  Chains
    whose series is constant are refused."""
    s = np.asarray(series, dtype=np.float64)
    if s.ndim != 2:
        raise ValueError("need [chains][samples]")
    n = s.shape[1]
    if n < 2 * min_bins:
        raise ValueError("need at least %d samples per chain" % (2 * min_bins))
    frozen = _constant(s, axis=1)
    if np.any(frozen):
        raise ValueError("%d of %d chains have a constant series" % (int(frozen.sum()), s.shape[0]))
    var = s.var(axis=1).mean()
    out = []
    B = 1
    while n // B >= min_bins:
        nb = n // B
        means = s[:, :nb * B].reshape(s.shape[0], nb, B).mean(axis=2)
        out.append((B, B * means.var(axis=1).mean() / (2.0 * var)))
        B *= 2
    return out


def tau_int_chains(series, min_bins=64):
    """tau_int of several independent chains' series ([chains][samples])."""
    return binning_curve_chains(series, min_bins)[-1][1]


def estimate_chains(series, min_bins=64, plateau_tol=0.05):
    """tau_int with its convergence: {"tau": tau_B at the largest B, "B": B,
    "converged": whether tau_B / tau_{B/2} - 1 < plateau_tol, "curve": ...}.
    An estimate that has not converged is a lower bound of tau_int."""
    curve = binning_curve_chains(series, min_bins)
    B, tau = curve[-1]
    converged = len(curve) >= 2 and tau / curve[-2][1] - 1.0 < plateau_tol
    return {"tau": tau, "B": B, "converged": bool(converged), "curve": curve}
