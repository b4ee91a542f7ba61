"""Pins of the oracle's model matrices and of its stabilised G / log|det M|
against things the oracle does not compute itself: plane-wave closed forms,
the atomic limit, brute-force dense determinants (numpy at small beta, mpmath
at 50 digits at large beta) and the particle-hole symmetry of the half-filled
bipartite lattice."""
import math
from dataclasses import replace

import mpmath
import numpy as np
import pytest

from oracle import model, udt
from oracle.model import Params


def plane_wave_green(p, shift=0.0):
    """(I + exp(-beta (K + shift)))^-1 and its log|det| for the periodic square lattice.

    K is diagonal in plane waves k = 2 pi (mx, my)/Nx with eps_k = -2t(cos kx + cos ky) - mu.
    """
    nx, n = p.nx, p.n
    ks = [(2 * math.pi * mx / nx, 2 * math.pi * my / nx) for my in range(nx) for mx in range(nx)]
    eps = np.array([-2 * p.t * (math.cos(kx) + math.cos(ky)) - p.mu + shift for kx, ky in ks])
    occ = 1.0 / (1.0 + np.exp(-p.beta * eps))
    G = np.zeros((n, n))
    for i in range(n):
        xi, yi = i % nx, i // nx
        for j in range(n):
            dx, dy = xi - j % nx, yi - j // nx
            G[i, j] = sum(o * math.cos(kx * dx + ky * dy) for o, (kx, ky) in zip(occ, ks)) / n
    logdet = float(np.sum(np.log1p(np.exp(-p.beta * eps))))
    return G, logdet


def random_fields(p, seed, scale=1.0):
    return scale * np.random.default_rng(seed).standard_normal((p.L, p.n))


@pytest.mark.parametrize("nx,mu,sign", [(1, 0.2, -1.0), (2, 0.0, -1.0), (3, 0.4, 1.0), (6, -0.3, -1.0), (12, 0.0, 1.0)])
def test_exp_hopping_is_a_kronecker_square(nx, mu, sign):
    """The wraps and block products use exp(s dtau K) = E1 (x) E1 with E1 the
    exponential of the nx-site ring carrying half the chemical potential
    (site i = ix + nx iy); checked against the oracle's eigen-decomposition of
    the full K, with E1 from scipy's expm of the ring."""
    import scipy.linalg
    p = Params(nx=nx, beta=1.0, mu=mu)
    ring = np.zeros((nx, nx))
    for a in range(nx):
        ring[a, a] -= 0.5 * mu
        for d in (1, -1):
            ring[a, (a + d) % nx] -= p.t
    e1 = scipy.linalg.expm(sign * p.dtau * ring)
    assert np.allclose(np.kron(e1, e1), model.exp_hopping(p, sign), rtol=0, atol=1e-14)


@pytest.mark.parametrize("nx,beta,mu", [(2, 2.0, 0.0), (4, 4.0, 0.0), (4, 8.0, 0.3), (6, 10.0, -0.5)])
def test_hopping_spectrum_matches_plane_waves(nx, beta, mu):
    p = Params(nx=nx, beta=beta, mu=mu)
    w = np.sort(np.linalg.eigvalsh(model.hopping_matrix(p)))
    ks = [2 * math.pi * m / nx for m in range(nx)]
    eps = np.sort([-2 * (math.cos(a) + math.cos(b)) - mu for a in ks for b in ks])
    assert np.allclose(w, eps, atol=1e-12)


@pytest.mark.parametrize("nx,beta,ns", [(2, 4.0, 10), (4, 4.0, 10), (4, 12.0, 8), (6, 10.0, 10)])
def test_free_fermions_g0(nx, beta, ns):
    """g = 0: every B_l = exp(-dtau K) and G = (I + exp(-beta K))^-1 exactly."""
    p = Params(nx=nx, beta=beta, g=0.0, n_stab=ns)
    x = random_fields(p, 1)
    expk = model.exp_hopping(p, -1.0)
    G, ld = udt.green_and_logdet(p, expk, x, 0)
    Gc, ldc = plane_wave_green(p)
    assert np.max(np.abs(G - Gc)) < 1e-12
    assert abs(ld - ldc) < 1e-10 * max(1.0, abs(ldc))


@pytest.mark.parametrize("c", [-0.7, 0.4])
def test_uniform_field(c):
    """x = c everywhere: prod B = exp(-beta g c) exp(-beta K)."""
    p = Params(nx=4, beta=8.0, g=1.3, n_stab=10)
    x = np.full((p.L, p.n), c)
    expk = model.exp_hopping(p, -1.0)
    for start in (0, 10, 40):
        G, ld = udt.green_and_logdet(p, expk, x, start)
        Gc, ldc = plane_wave_green(p, shift=p.g * c)
        assert np.max(np.abs(G - Gc)) < 1e-12
        assert abs(ld - ldc) < 1e-10 * max(1.0, abs(ldc))


def test_atomic_limit():
    """t = 0: B_l is diagonal and G_ii = 1/(1 + exp(dtau sum_l (mu - g x_li)))."""
    p = Params(nx=3, t=0.0, mu=0.2, beta=6.0, g=1.1, n_stab=6)
    x = random_fields(p, 7)
    expk = model.exp_hopping(p, -1.0)
    G, ld = udt.green_and_logdet(p, expk, x, 0)
    a = p.dtau * np.sum(p.mu - p.g * x, axis=0)
    assert np.max(np.abs(G - np.diag(1.0 / (1.0 + np.exp(a))))) < 1e-13
    assert abs(ld - float(np.sum(np.log1p(np.exp(a))))) < 1e-11


@pytest.mark.parametrize("nx,beta,ns,start", [(2, 1.0, 5, 0), (4, 2.0, 4, 8), (4, 2.0, 5, 15), (3, 1.0, 2, 4)])
def test_brute_force_small_beta(nx, beta, ns, start):
    """Dense product, determinant and inverse in plain float64 (well conditioned at small beta)."""
    p = Params(nx=nx, beta=beta, g=1.2, mu=0.1, n_stab=ns)
    x = random_fields(p, 3)
    expk = model.exp_hopping(p, -1.0)
    prod = np.eye(p.n)
    for l in udt.product_order(p.L, start):
        prod = model.b_matrix(p, expk, x[l]) @ prod
    m = np.eye(p.n) + prod
    G, ld = udt.green_and_logdet(p, expk, x, start)
    assert np.max(np.abs(G - np.linalg.inv(m))) < 1e-12
    assert abs(ld - np.linalg.slogdet(m)[1]) < 1e-12 * max(1.0, abs(ld))


def test_brute_force_mpmath_large_beta():
    """beta = 16 on 2x2: the product spans ~e^{+-70}; 50-digit arithmetic needs no stabilisation."""
    mpmath.mp.dps = 50
    p = Params(nx=2, beta=16.0, g=1.2, n_stab=10)
    x = random_fields(p, 11)
    n = p.n
    K = mpmath.matrix(model.hopping_matrix(p).tolist())
    expk = mpmath.expm(-p.dtau * K)
    prod = mpmath.eye(n)
    for l in range(p.L):
        d = mpmath.diag([mpmath.exp(-p.dtau * p.g * x[l, i]) for i in range(n)])
        prod = d * expk * prod
    m = mpmath.eye(n) + prod
    ginv = m ** -1
    ld_ref = float(mpmath.log(abs(mpmath.det(m))))
    G, ld = udt.green_and_logdet(p, model.exp_hopping(p, -1.0), x, 0)
    g_ref = np.array(ginv.tolist(), dtype=float)
    assert np.max(np.abs(G - g_ref)) < 1e-11
    assert abs(ld - ld_ref) < 1e-11 * abs(ld_ref)


def test_particle_hole_symmetry():
    """mu = 0, even Nx: G(-x) = P (I - G(x)^T) P with P = diag((-1)^(ix+iy)), log W(-x) = log W(x).

    This fixes the sign of the bosonic linear term that the g x (n - 1) coupling brings in."""
    p = Params(nx=4, beta=4.0, g=1.0, mu=0.0, n_stab=10)
    x = random_fields(p, 5)
    expk = model.exp_hopping(p, -1.0)
    G1, ld1 = udt.green_and_logdet(p, expk, x, 0)
    G2, ld2 = udt.green_and_logdet(p, expk, -x, 0)
    P = np.diag([(-1.0) ** (i % 4 + i // 4) for i in range(p.n)])
    assert np.max(np.abs(G2 - P @ (np.eye(p.n) - G1.T) @ P)) < 1e-12
    lw1 = 2 * ld1 - model.bosonic_action(p, x)
    lw2 = 2 * ld2 - model.bosonic_action(p, -x)
    assert abs(lw1 - lw2) < 1e-10 * abs(lw1)


def test_bosonic_action_local_and_global_changes():
    p = Params(nx=3, beta=2.0, g=0.9, omega=1.3, mass=1.7, n_stab=5)
    x = random_fields(p, 9)
    L = p.L
    rs = np.random.default_rng(4)
    for _ in range(20):
        l, i, d = int(rs.integers(L)), int(rs.integers(p.n)), float(rs.uniform(-1, 1))
        xp = x.copy()
        xp[l, i] += d
        ref = model.bosonic_action(p, xp) - model.bosonic_action(p, x)
        got = model.local_action_change(p, x[l, i], x[(l - 1) % L, i], x[(l + 1) % L, i], d)
        assert abs(got - ref) < 1e-11
        xp = x.copy()
        xp[:, i] += d
        ref = model.bosonic_action(p, xp) - model.bosonic_action(p, x)
        got = model.global_action_change(p, float(np.sum(x[:, i])), d, L)
        assert abs(got - ref) < 1e-11


def test_bosonic_action_l2_kinetic_counts_both_links():
    p = Params(nx=1, beta=0.2, dtau=0.1, g=0.0, omega=0.0)
    x = np.array([[0.3], [1.0]])
    # two links (1 -> 0 and 0 -> 1), each (M / 2 dtau)(0.7)^2
    assert abs(model.bosonic_action(p, x) - 2 * 0.49 / 0.2) < 1e-14


def test_initial_fields_are_standard_normal():
    p = Params(nx=8, beta=8.0)
    x = model.initial_fields(p, seed=2, chain=0)
    assert abs(np.mean(x)) < 4 / math.sqrt(x.size)
    assert abs(np.var(x) - 1.0) < 4 * math.sqrt(2.0 / x.size)


def test_chain_coupling_range():
    gs = [model.chain_coupling(4, c, 0.8, 1.6) for c in range(128)]
    assert min(gs) >= 0.8 and max(gs) < 1.6
    assert abs(np.mean(gs) - 1.2) < 4 * 0.8 / math.sqrt(12 * 128)


def test_stack_order_is_cyclic_invariant_for_logdet():
    p = Params(nx=4, beta=4.0, g=1.0, n_stab=10)
    x = random_fields(p, 13)
    expk = model.exp_hopping(p, -1.0)
    lds = [udt.green_and_logdet(p, expk, x, s)[1] for s in (0, 10, 20, 30)]
    assert max(lds) - min(lds) < 1e-11 * abs(lds[0])


def test_replace_params_keeps_L():
    p = replace(Params(nx=4), beta=12.0)
    assert p.L == 120
