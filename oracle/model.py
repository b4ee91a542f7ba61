"""The Holstein model on an Nx x Nx periodic square lattice, discretised in
imaginary time (paper: Model; Determinant quantum Monte Carlo).

Conventions (the paper leaves these open; the readings are listed in the
design notes):
  * site i = ix + Nx*iy; hopping -t to the four periodic neighbours, counted
    with multiplicity (Nx = 2 gives -2t), chemical potential -mu on the diagonal.
  * slices l = 0..L-1 with L = beta/dtau, periodic in imaginary time
    (x[L] == x[0], as the trace in Z requires).
  * coupling g*x_i*(n_i - 1): the fermion matrix of slice l is
    B_l = diag(exp(-dtau*g*x[l,:])) @ exp(-dtau*K), interaction on the left as
    in the paper's B_l = exp(-dtau H_eph) exp(-dtau H_0), and the constant
    part exp(+dtau*g*x) of each slice goes into the bosonic action.
  * weight W(x) = exp(-S_b(x)) * det(I + B_{L-1}...B_0)^2 (two equal spins),
    with S_b = dtau * S_ph - dtau*g*sum(x), S_ph as printed in the paper.

Parity: the matrices here are pinned by closed forms (g = 0 free fermions,
uniform field, t = 0 atomic limit) and by brute-force determinants in
tests/test_oracle_model.py.
"""
import math
from dataclasses import dataclass

import numpy as np

from . import philox


@dataclass
class Params:
    nx: int
    t: float = 1.0
    mu: float = 0.0
    mass: float = 1.0
    omega: float = 1.0
    g: float = 1.0
    beta: float = 4.0
    dtau: float = 0.1
    n_stab: int = 10
    local_width: float = 0.5
    global_width: float = 0.0

    @property
    def n(self):
        return self.nx * self.nx

    @property
    def L(self):
        L = int(round(self.beta / self.dtau))
        if abs(L * self.dtau - self.beta) > 1e-9 or L < 2:
            raise ValueError("beta/dtau must be an integer >= 2")
        return L


def hopping_matrix(p):
    """K with K_ij = -t for each periodic nearest-neighbour offset, K_ii = -mu."""
    nx, n = p.nx, p.n
    K = np.zeros((n, n))
    for iy in range(nx):
        for ix in range(nx):
            i = ix + nx * iy
            K[i, i] -= p.mu
            for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                j = (ix + dx) % nx + nx * ((iy + dy) % nx)
                K[i, j] -= p.t
    return K


def exp_hopping(p, sign):
    """exp(sign * dtau * K) through the eigen-decomposition of the symmetric K."""
    w, v = np.linalg.eigh(hopping_matrix(p))
    return (v * np.exp(sign * p.dtau * w)) @ v.T


def b_matrix(p, expk, x_slice):
    """B_l = diag(exp(-dtau*g*x[l,:])) @ exp(-dtau*K)."""
    return np.exp(-p.dtau * p.g * x_slice)[:, None] * expk


def bosonic_action(p, x):
    """S_b(x) = sum_{l,i} [ M/(2 dtau) (x[l+1,i]-x[l,i])^2 + dtau*M*Omega^2/2 x^2 - dtau*g*x ]."""
    kin = np.sum((np.roll(x, -1, axis=0) - x) ** 2) * p.mass / (2.0 * p.dtau)
    pot = p.dtau * 0.5 * p.mass * p.omega ** 2 * np.sum(x * x)
    lin = -p.dtau * p.g * np.sum(x)
    return kin + pot + lin


def local_action_change(p, a, prev, nxt, d):
    """S_b(x') - S_b(x) for x[l,i]: a -> a + d, with neighbours prev = x[l-1,i], nxt = x[l+1,i].

    The two kinetic links touching (i, l) change by (M/dtau)(d(2a - prev - nxt) + d^2);
    the on-site terms by dtau*M*Omega^2/2 (2 a d + d^2) - dtau*g*d.
    """
    kin = (p.mass / p.dtau) * (d * (2.0 * a - prev - nxt) + d * d)
    pot = p.dtau * 0.5 * p.mass * p.omega ** 2 * (2.0 * a * d + d * d)
    return kin + pot - p.dtau * p.g * d


def global_action_change(p, column_sum, d, L):
    """S_b change when every slice of one site moves by d (the kinetic links are unchanged)."""
    m_om2 = p.mass * p.omega ** 2
    return p.dtau * (m_om2 * d * column_sum + 0.5 * m_om2 * L * d * d - p.g * L * d)


def initial_fields(p, seed, chain):
    """x[l, i] ~ N(0, 1) by Box-Muller on two uniforms of the KIND_INIT block at slot l*N + i."""
    L, n = p.L, p.n
    x = np.empty((L, n))
    for l in range(L):
        for i in range(n):
            u0, u1 = philox.uniforms(seed, chain, 0, l * n + i, philox.KIND_INIT)
            x[l, i] = math.sqrt(-2.0 * math.log(1.0 - u0)) * math.cos(2.0 * math.pi * u1)
    return x


def chain_coupling(seed, chain, g_lo, g_hi):
    """Per-chain coupling g ~ U(g_lo, g_hi) from word 0 of the KIND_COUPLING block."""
    u0, _ = philox.uniforms(seed, chain, 0, 0, philox.KIND_COUPLING)
    return g_lo + (g_hi - g_lo) * u0
