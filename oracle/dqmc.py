"""The conventional DQMC sweep of the Holstein model (paper: Determinant quantum
Monte Carlo, Local Updates intro, Benchmarks protocol), plain and serial in FP64.

One sweep visits every slice once.  G_l = (I + B_l...B_0 B_{L-1}...B_{l+1})^-1
is the Green's function "at slice l", the one whose local moves at slice l
are rank-1 updates.  Upward (even sweeps, and every sweep of a chain with
block moves):
  for l = 0..L-1:
      wrap      G <- B_l G B_l^-1              (G_{l-1} -> G_l)
      for i = 0..N-1: local move x[l,i] += d, d ~ U(-w, w)
          det ratio of one spin  r = 1 + delta (1 - G_ii), delta = exp(-dtau g d) - 1
          Metropolis ratio       R = r^2 exp(-(S_b(x') - S_b(x)))      (W'/W)
          accept iff u < R; then G <- G - (delta/r) G[:,i] (e_i - G[i,:])   (rank 1)
      if (l+1) % n_stab == 0: recompute G_l and log|det M| from scratch (UDT chain)
Downward (odd sweeps of a chain without block moves):
  for l = L-1..0:
      the same N local moves at slice l
      unwrap    G <- B_l^-1 G B_l             (G_l -> G_{l-1})
      if l % n_stab == 0: recompute G_{l-1} and log|det M| from scratch
Both end at G_{L-1}, the state every sweep starts from.  The paper fixes no
order; alternating lets an implementation reuse the products of the previous
sweep (the blocks above slice l in an upward sweep are exactly those the
downward sweep has just updated).  Then, if block moves are enabled, for
i = 0..N-1: shift x[:,i] by d ~ U(-w_g, w_g) and accept with
exp(2 (log|det M'| - log|det M|) - dS_b), the determinant evaluated from
scratch (no fast update exists for block moves).

The rank-1 form follows from det(I + (I+Delta) A) = det(I + A) det(I + Delta(I - G))
with Delta = delta e_i e_i^T and A the cyclic product that starts at B_l.

Parity: the ratio is pinned against exp(log W(x') - log W(x)) with both
weights from scratch, the rank-1 update against the recomputed G, and the
sampling against the g = 0 oscillator closed form and <n> = 1
(tests/test_oracle_sweep.py).
"""
import math

import numpy as np

from . import philox
from .model import (bosonic_action, chain_coupling, exp_hopping, global_action_change,
                    initial_fields, local_action_change)
from .udt import green_and_logdet


class Decision:
    __slots__ = ("kind", "sweep", "slot", "accept", "margin")

    def __init__(self, kind, sweep, slot, accept, margin):
        self.kind, self.sweep, self.slot = kind, sweep, slot
        self.accept, self.margin = accept, margin


def log_margin(u, R):
    """ln u - ln R (negative means accept); used to locate near-ties."""
    if R <= 0.0:
        return math.inf
    if u <= 0.0:
        return -math.inf
    return math.log(u) - math.log(R)


class Chain:
    """One Markov chain of the conventional DQMC (FP64, rank-1 updates)."""

    def __init__(self, p, seed, chain, x=None):
        self.p = p
        self.seed = seed
        self.chain = chain
        self.expk = exp_hopping(p, -1.0)
        self.expkinv = exp_hopping(p, +1.0)
        self.x = initial_fields(p, seed, chain) if x is None else np.array(x, dtype=float)
        self.sweep_index = 0
        self.G, self.logdet = green_and_logdet(p, self.expk, self.x, 0)
        self.decisions = []
        self.local_accepts = 0
        self.local_proposals = 0
        self.global_accepts = 0
        self.global_proposals = 0
        self.max_drift_g = 0.0
        self.max_drift_logdet = 0.0

    # -- one slice -------------------------------------------------------
    def wrap(self, l):
        dvec = np.exp(-self.p.dtau * self.p.g * self.x[l])
        self.G = (dvec[:, None] * (self.expk @ self.G @ self.expkinv)) / dvec[None, :]

    def unwrap(self, l):
        """G <- B_l^-1 G B_l, from the slice-l Green's function to slice l-1's."""
        dvec = np.exp(-self.p.dtau * self.p.g * self.x[l])
        self.G = self.expkinv @ ((self.G / dvec[:, None]) * dvec[None, :]) @ self.expk

    def local_move(self, l, i):
        p, x, G = self.p, self.x, self.G
        L = x.shape[0]
        u0, u1 = philox.uniforms(self.seed, self.chain, self.sweep_index, l * p.n + i,
                                 philox.KIND_LOCAL)
        d = p.local_width * (2.0 * u0 - 1.0)
        delta = math.expm1(-p.dtau * p.g * d)
        r = 1.0 + delta * (1.0 - G[i, i])
        ds = local_action_change(p, x[l, i], x[(l - 1) % L, i], x[(l + 1) % L, i], d)
        R = r * r * math.exp(-ds)
        accept = u1 < R
        self.decisions.append(Decision(philox.KIND_LOCAL, self.sweep_index, l * p.n + i,
                                       accept, log_margin(u1, R)))
        self.local_proposals += 1
        if accept:
            col = G[:, i].copy()
            row = -G[i, :].copy()
            row[i] += 1.0
            self.G = G - (delta / r) * np.outer(col, row)
            x[l, i] += d
            self.logdet += math.log(abs(r))
            self.local_accepts += 1
        return accept

    def recompute(self, l):
        """Replace G (after slice l) and log|det M| by the from-scratch values.
        The tracked pair is kept as G_tracked, logdet_tracked (for comparisons
        of the state a sweep carries before it is replaced)."""
        g_rec, ld_rec = green_and_logdet(self.p, self.expk, self.x, (l + 1) % self.p.L)
        self.G_tracked, self.logdet_tracked = self.G.copy(), self.logdet
        self.max_drift_g = max(self.max_drift_g, float(np.max(np.abs(self.G - g_rec))))
        self.max_drift_logdet = max(self.max_drift_logdet, abs(self.logdet - ld_rec))
        self.G, self.logdet = g_rec, ld_rec

    def downward(self):
        """Whether this sweep runs downward: odd sweeps, when there are no block moves."""
        return self.p.global_width == 0.0 and self.sweep_index % 2 == 1

    def local_sweep(self):
        p = self.p
        if not self.downward():
            for l in range(p.L):
                self.wrap(l)
                for i in range(p.n):
                    self.local_move(l, i)
                if (l + 1) % p.n_stab == 0:
                    self.recompute(l)
            return
        for l in range(p.L - 1, -1, -1):
            for i in range(p.n):
                self.local_move(l, i)
            self.unwrap(l)
            if l % p.n_stab == 0:
                self.recompute(l - 1)

    def global_sweep(self):
        p, L = self.p, self.p.L
        for i in range(p.n):
            u0, u1 = philox.uniforms(self.seed, self.chain, self.sweep_index, i,
                                     philox.KIND_GLOBAL)
            d = p.global_width * (2.0 * u0 - 1.0)
            xp = self.x.copy()
            xp[:, i] += d
            g_new, ld_new = green_and_logdet(p, self.expk, xp, 0)
            ds = global_action_change(p, float(np.sum(self.x[:, i])), d, L)
            R = math.exp(min(2.0 * (ld_new - self.logdet) - ds, 700.0))
            accept = u1 < R
            self.decisions.append(Decision(philox.KIND_GLOBAL, self.sweep_index, i, accept,
                                           log_margin(u1, R)))
            self.global_proposals += 1
            if accept:
                self.x, self.G, self.logdet = xp, g_new, ld_new
                self.global_accepts += 1

    def sweep(self):
        self.local_sweep()
        if self.p.global_width > 0.0:
            self.global_sweep()
        self.sweep_index += 1

    # -- weights and observables -----------------------------------------
    def log_weight(self, x=None):
        """log W(x) = 2 log|det M(x)| - S_b(x), from scratch."""
        x = self.x if x is None else x
        _, ld = green_and_logdet(self.p, self.expk, x, 0)
        return 2.0 * ld - bosonic_action(self.p, x)

    def observables(self):
        return equal_time_observables(self.p, self.G, self.x)


def density_correlations(G):
    """<n_i n_j> for one field configuration, n_i = n_i,up + n_i,dn, two equal spins.

    Wick's theorem with G_ij = <c_i c_j^dagger> (the same for both spins):
      <n_is n_js'> = (1 - G_ii)(1 - G_jj)                      for s != s'
      <n_is n_js>  = (1 - G_ii)(1 - G_jj) + (delta_ij - G_ji) G_ij
    and summing the four spin pairs,
      <n_i n_j> = 4 (1 - G_ii)(1 - G_jj) + 2 (delta_ij - G_ji) G_ij.
    """
    n = G.shape[0]
    occ = 1.0 - np.diag(G)
    nn = np.empty((n, n))
    for i in range(n):
        for j in range(n):
            nn[i, j] = 4.0 * occ[i] * occ[j] + 2.0 * ((1.0 if i == j else 0.0) - G[j, i]) * G[i, j]
    return nn


def equal_time_observables(p, G, x):
    """Equal-time estimators for one field configuration (two equal spins).

    density     <n>        = (2/N) sum_i (1 - G_ii)
    double occ. <n_u n_d>  = (1/N) sum_i (1 - G_ii)^2     (the spins are independent
                                                           for a fixed field)
    S_CDW(pi,pi)           = (1/N) sum_ij (-1)^(i+j) <n_i n_j>, <n_i n_j> from
                             density_correlations
    <x>, <x^2>             field moments over all (l, i)

    Parity: pinned against traces over the full 2N-mode Fock space of a 2x2
    lattice (tests/test_oracle_observables.py).
    """
    n = p.n
    nx = p.nx
    eps = np.array([(-1.0) ** ((i % nx) + (i // nx)) for i in range(n)])
    occ = 1.0 - np.diag(G)
    nn = density_correlations(G)
    s_cdw = 0.0
    for i in range(n):
        for j in range(n):
            s_cdw += eps[i] * eps[j] * nn[i, j]
    return {
        "density": 2.0 * float(np.sum(occ)) / n,
        "double_occupancy": float(np.sum(occ * occ)) / n,
        "s_cdw": s_cdw / n,
        "x_mean": float(np.mean(x)),
        "x2_mean": float(np.mean(x * x)),
    }


def make_chains(p, seed, n_chains, g_range=None):
    """Chains 0..n_chains-1 of one lattice; g per chain from U(g_range) when given."""
    chains = []
    for c in range(n_chains):
        pc = p
        if g_range is not None:
            from dataclasses import replace
            pc = replace(p, g=chain_coupling(seed, c, *g_range))
        chains.append(Chain(pc, seed, c))
    return chains
