"""The binning estimate of the integrated autocorrelation time against closed
forms: white noise (tau = 1/2) and the AR(1) process x_t = rho x_{t-1} + e_t,
whose autocorrelation is rho^t, so tau_int = 1/2 + rho / (1 - rho) =
(1 + rho) / (2 (1 - rho))."""
import numpy as np
import pytest

from paper_1905_07440_amd import autocorr


def ar1(rho, n, chains, seed):
    rng = np.random.default_rng(seed)
    e = rng.standard_normal((chains, n))
    x = np.empty((chains, n))
    x[:, 0] = e[:, 0] / np.sqrt(1.0 - rho * rho)          # stationary start
    for t in range(1, n):
        x[:, t] = rho * x[:, t - 1] + e[:, t]
    return x


def test_white_noise_gives_one_half():
    x = np.random.default_rng(1).standard_normal((16, 8192))
    assert abs(autocorr.tau_int_chains(x) - 0.5) < 0.05
    assert abs(autocorr.tau_int(x[0]) - 0.5) < 0.15


@pytest.mark.parametrize("rho", [0.5, 0.8, 0.9])
def test_ar1_closed_form(rho):
    exact = (1.0 + rho) / (2.0 * (1.0 - rho))
    x = ar1(rho, 16384, 16, seed=int(100 * rho))
    est = autocorr.tau_int_chains(x)
    assert abs(est - exact) < 0.08 * exact, (est, exact)


def test_binning_curve_starts_at_one_half_and_rises():
    x = ar1(0.8, 4096, 1, seed=3)[0]
    curve = autocorr.binning_curve(x)
    assert curve[0][0] == 1 and abs(curve[0][1] - 0.5) < 1e-12   # B = 1: var(x) / (2 var(x))
    assert curve[-1][1] > 3.0                                     # exact 4.5


def test_rejects_short_or_constant_series():
    with pytest.raises(ValueError):
        autocorr.tau_int(np.arange(10.0))
    with pytest.raises(ValueError):
        autocorr.tau_int(np.ones(1000))


def test_frozen_chains_are_refused():
    """Copies of one value: numpy's variance is ~1e-31, not 0; still constant."""
    x = np.full((64, 1024), 0.9660547121099028)
    assert x.var(axis=1).max() >= 0.0
    with pytest.raises(ValueError):
        autocorr.tau_int_chains(x)
    y = np.random.default_rng(2).standard_normal((4, 1024))
    y[1] = 0.25                                     # one frozen chain among moving ones
    with pytest.raises(ValueError):
        autocorr.tau_int_chains(y)


def test_short_runs_are_flagged_as_lower_bounds():
    """AR(1) with tau = 9.5 over 1024 samples: the largest bin (16) is below
    the plateau, so the estimate is not converged; over 65536 samples it is."""
    rho = 0.9
    exact = (1.0 + rho) / (2.0 * (1.0 - rho))
    short = autocorr.estimate_chains(ar1(rho, 1024, 64, seed=5))
    assert not short["converged"] and short["tau"] < exact
    long = autocorr.estimate_chains(ar1(rho, 65536, 4, seed=6))
    assert long["converged"] and abs(long["tau"] - exact) < 0.1 * exact
