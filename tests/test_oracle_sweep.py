"""Pins of the oracle's sweep: the local and block-move Metropolis ratios
against weights computed from scratch, the rank-1 update and the wrap against
the from-scratch G, and the sampled distribution against exact results (the
two-slice atomic limit by quadrature; the g = 0 oscillator by its closed form)."""
import math
from dataclasses import replace

import numpy as np
import pytest

from oracle import dqmc, model, philox, udt
from oracle.model import Params


def small_params(**kw):
    base = dict(nx=4, beta=2.0, g=1.2, n_stab=5, local_width=0.5)
    base.update(kw)
    return Params(**base)


def test_local_ratio_equals_weight_ratio():
    """r^2 exp(-dS_b) = W(x')/W(x) with both weights from scratch."""
    p = small_params()
    ch = dqmc.Chain(p, seed=21, chain=0)
    base = ch.log_weight()
    rs = np.random.default_rng(1)
    for l in (0, 3, 9):
        # bring G to slice l: G_l = (I + B_l ... B_0 B_{L-1} ... B_{l+1})^-1
        G_l, _ = udt.green_and_logdet(p, ch.expk, ch.x, (l + 1) % p.L)
        for _ in range(4):
            i, d = int(rs.integers(p.n)), float(rs.uniform(-0.5, 0.5))
            delta = math.expm1(-p.dtau * p.g * d)
            r = 1.0 + delta * (1.0 - G_l[i, i])
            L = p.L
            ds = model.local_action_change(p, ch.x[l, i], ch.x[(l - 1) % L, i], ch.x[(l + 1) % L, i], d)
            xp = ch.x.copy()
            xp[l, i] += d
            assert abs((2 * math.log(abs(r)) - ds) - (ch.log_weight(xp) - base)) < 1e-10


def test_rank1_updates_match_recompute_and_logdet_tracks():
    p = small_params(g=1.5, local_width=1.0)
    ch = dqmc.Chain(p, seed=3, chain=1)
    for l in range(7):
        ch.wrap(l)
        for i in range(p.n):
            ch.local_move(l, i)
        G_ref, ld_ref = udt.green_and_logdet(p, ch.expk, ch.x, (l + 1) % p.L)
        assert np.max(np.abs(ch.G - G_ref)) < 1e-11
        assert abs(ch.logdet - ld_ref) < 1e-10
    assert ch.local_accepts > 10


def test_wrap_matches_recompute():
    p = small_params()
    ch = dqmc.Chain(p, seed=8, chain=0)
    for l in range(p.L):
        ch.G, _ = udt.green_and_logdet(p, ch.expk, ch.x, l)      # G_{l-1}, fresh
        ch.wrap(l)
        G_ref, _ = udt.green_and_logdet(p, ch.expk, ch.x, (l + 1) % p.L)
        assert np.max(np.abs(ch.G - G_ref)) < 1e-12


def test_unwrap_matches_recompute():
    """B_l^-1 G_l B_l = G_{l-1}, both from scratch."""
    p = small_params()
    ch = dqmc.Chain(p, seed=8, chain=0)
    for l in range(p.L):
        ch.G, _ = udt.green_and_logdet(p, ch.expk, ch.x, (l + 1) % p.L)   # G_l, fresh
        ch.unwrap(l)
        G_ref, _ = udt.green_and_logdet(p, ch.expk, ch.x, l)             # G_{l-1}
        assert np.max(np.abs(ch.G - G_ref)) < 1e-12


def test_downward_sweep_tracks_recompute():
    """A downward sweep: after the moves of slice l the tracked G equals G_l from
    scratch; its slice order and recompute points are as documented."""
    p = small_params(g=1.5, local_width=1.0)
    ch = dqmc.Chain(p, seed=3, chain=1)
    ch.sweep()
    assert ch.downward()
    seen = []
    orig = ch.local_move

    def spy(l, i):
        if i == 0:
            G_ref, _ = udt.green_and_logdet(p, ch.expk, ch.x, (l + 1) % p.L)
            assert np.max(np.abs(ch.G - G_ref)) < 1e-10
            seen.append(l)
        return orig(l, i)

    ch.local_move = spy
    ch.sweep()
    assert seen == list(range(p.L - 1, -1, -1))
    G_ref, ld_ref = udt.green_and_logdet(p, ch.expk, ch.x, 0)
    assert np.max(np.abs(ch.G - G_ref)) < 1e-13 and abs(ch.logdet - ld_ref) < 1e-12
    assert ch.max_drift_g < 1e-10
    # block moves keep every sweep upward
    q = dqmc.Chain(small_params(global_width=1.0), seed=3, chain=1)
    q.sweep()
    assert not q.downward()


def test_sweep_invariants_and_decision_log():
    p = small_params(beta=4.0, n_stab=10)
    ch = dqmc.Chain(p, seed=1, chain=0)
    ch.sweep()
    ch.sweep()
    assert ch.sweep_index == 2
    assert ch.local_proposals == 2 * p.L * p.n
    assert len(ch.decisions) == ch.local_proposals
    assert ch.max_drift_g < 1e-10 and ch.max_drift_logdet < 1e-9
    G_ref, ld_ref = udt.green_and_logdet(p, ch.expk, ch.x, 0)
    assert np.max(np.abs(ch.G - G_ref)) < 1e-13
    for dec in ch.decisions:
        assert dec.accept == (dec.margin < 0)


def test_global_ratio_equals_weight_ratio():
    p = small_params(global_width=1.0)
    ch = dqmc.Chain(p, seed=2, chain=0)
    base = ch.log_weight()
    for i in range(p.n):
        d = 0.37 * (i - 7)
        xp = ch.x.copy()
        xp[:, i] += d
        _, ld_new = udt.green_and_logdet(p, ch.expk, xp, 0)
        ds = model.global_action_change(p, float(np.sum(ch.x[:, i])), d, p.L)
        assert abs((2 * (ld_new - ch.logdet) - ds) - (ch.log_weight(xp) - base)) < 1e-10


def test_global_sweep_keeps_state_consistent():
    p = small_params(global_width=1.0, beta=2.0)
    ch = dqmc.Chain(p, seed=6, chain=0)
    ch.sweep()
    assert ch.global_proposals == p.n
    G_ref, ld_ref = udt.green_and_logdet(p, ch.expk, ch.x, 0)
    assert np.max(np.abs(ch.G - G_ref)) < 1e-13 and abs(ch.logdet - ld_ref) < 1e-12


def test_deterministic_given_seed():
    p = small_params()
    a = dqmc.Chain(p, seed=5, chain=2)
    b = dqmc.Chain(p, seed=5, chain=2)
    a.sweep()
    b.sweep()
    assert np.array_equal(a.x, b.x)
    c = dqmc.Chain(p, seed=5, chain=3)
    c.sweep()
    assert not np.array_equal(a.x, c.x)


def test_observables_free_half_filling():
    """g = 0, mu = 0: <n> = 1 exactly for every field (particle-hole symmetric spectrum)."""
    p = Params(nx=4, beta=4.0, g=0.0)
    ch = dqmc.Chain(p, seed=1, chain=0)
    obs = ch.observables()
    assert abs(obs["density"] - 1.0) < 1e-12
    # S_CDW against a direct double sum written with numpy
    G = ch.G
    n = p.n
    eps = np.array([(-1) ** (i % 4 + i // 4) for i in range(n)], dtype=float)
    occ = 1 - np.diag(G)
    nn = 4 * np.outer(occ, occ) + 2 * (np.eye(n) - G.T) * G
    assert abs(obs["s_cdw"] - eps @ nn @ eps / n) < 1e-12


def _binned_mean(samples, nbins=20):
    s = np.asarray(samples)
    b = s[: len(s) // nbins * nbins].reshape(nbins, -1).mean(axis=1)
    return b.mean(), b.std(ddof=1) / math.sqrt(nbins)


@pytest.mark.slow
def test_sampling_two_slice_atomic_limit():
    """t = 0, N = 1, L = 2: the chain samples W(x0, x1) = exp(-S_b) (1 + e^{-dtau g (x0+x1)})^2.

    Moments of x0 + x1 from the Markov chain against 2-D quadrature of the explicit weight."""
    # a stiff oscillator (Omega = 5) keeps the autocorrelation far below the bin length; with
    # Omega = 1 the sum x0 + x1 random-walks for hundreds of sweeps and binned errors undercount
    p = Params(nx=1, t=0.0, mu=0.0, beta=0.2, dtau=0.1, g=1.5, omega=5.0, n_stab=2, local_width=1.0)
    ch = dqmc.Chain(p, seed=17, chain=0, x=np.zeros((2, 1)))
    samples = []
    for _ in range(12000):
        ch.sweep()
        samples.append(float(ch.x[0, 0] + ch.x[1, 0]))
    samples = samples[200:]
    grid = np.linspace(-6, 6, 801)
    x0, x1 = np.meshgrid(grid, grid, indexing="ij")
    sb = (p.mass / p.dtau) * (x1 - x0) ** 2 + p.dtau * 0.5 * p.omega ** 2 * (x0 ** 2 + x1 ** 2) \
        - p.dtau * p.g * (x0 + x1)
    w = np.exp(-sb) * (1 + np.exp(-p.dtau * p.g * (x0 + x1))) ** 2
    w /= w.sum()
    exact_mean = float(np.sum(w * (x0 + x1)))
    exact_sq = float(np.sum(w * (x0 + x1) ** 2))
    m, e = _binned_mean(samples)
    m2, e2 = _binned_mean(np.square(samples))
    assert abs(m - exact_mean) < 4.5 * e + 1e-3
    assert abs(m2 - exact_sq) < 4.5 * e2 + 1e-3


@pytest.mark.slow
def test_sampling_free_oscillator_link_variance():
    """g = 0 decouples the fermions; the field is a discretised harmonic oscillator with
    <x_l x_{l+d}> = (dtau/M) cosh((L/2 - d) a) / (2 sinh a sinh(L a / 2)), cosh a = 1 + dtau^2 Omega^2/2.
    Check <(x_{l+1} - x_l)^2> = 2 (C(0) - C(1)), a short-correlated observable."""
    p = Params(nx=1, t=1.0, beta=2.0, dtau=0.1, g=0.0, omega=1.0, n_stab=10, local_width=0.5)
    L = p.L
    a = math.acosh(1 + 0.5 * (p.dtau * p.omega) ** 2)

    def C(d):
        return (p.dtau / p.mass) * math.cosh((L / 2 - d) * a) / (2 * math.sinh(a) * math.sinh(L * a / 2))

    ch = dqmc.Chain(p, seed=4, chain=0, x=np.zeros((L, 1)))
    vals = []
    for k in range(2500):
        ch.sweep()
        if k >= 100:
            vals.append(float(np.mean((np.roll(ch.x[:, 0], -1) - ch.x[:, 0]) ** 2)))
    m, e = _binned_mean(vals)
    assert abs(m - 2 * (C(0) - C(1))) < 4.5 * e
    # the closed form itself against the inverse of the circulant action matrix
    A = np.zeros((L, L))
    for l in range(L):
        A[l, l] = (p.mass / p.dtau) * (2 + (p.dtau * p.omega) ** 2)
        A[l, (l + 1) % L] -= p.mass / p.dtau
        A[l, (l - 1) % L] -= p.mass / p.dtau
    cov = np.linalg.inv(A)
    assert abs(cov[0, 0] - C(0)) < 1e-12 and abs(cov[0, 1] - C(1)) < 1e-12


def test_make_chains_draws_couplings():
    p = Params(nx=2, beta=1.0)
    chains = dqmc.make_chains(p, seed=4, n_chains=3, g_range=(0.8, 1.6))
    assert [c.p.g for c in chains] == [model.chain_coupling(4, c, 0.8, 1.6) for c in range(3)]
    assert replace(p).g == 1.0
    assert philox.KIND_COUPLING == 5
