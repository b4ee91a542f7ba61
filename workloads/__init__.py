"""Seeded synthetic workloads shared by the tests, the benchmark and the smoke
check.  This module holds parameter sets and seeded random inputs only; none of
the method's arithmetic lives here, so both the oracle and the GPU library can
be driven from it without sharing code.

Each workload stands in for the paper's DQMC runs of the 2D Holstein model at
half filling (paper: Model; Benchmarks).  The paper uses no dataset: its inputs
are the model parameters, a seed and Gaussian initial fields.
"""
from dataclasses import dataclass, field, asdict
from typing import List, Optional, Tuple

import numpy as np


@dataclass
class Lattice:
    """One group of chains that share a lattice size and model parameters."""
    nx: int
    n_chains: int
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
    g_range: Optional[Tuple[float, float]] = None   # per-chain g ~ U(lo, hi)
    proposal: int = 0                              # 0 exact DQMC, 1 network + cumulative
    nn_sweeps: int = 1                             # network: inner sweeps of each kind per cumulative accept


@dataclass
class Workload:
    name: str
    seed: int
    groups: List[Lattice]
    precision: int = 0          # 0 FP64, 1 mixed (FP32 wraps/updates, FP64 stabilisation)
    delay: int = 0              # delayed-update depth (0: library default)
    sweeps: int = 0             # sweeps the workload description asks for (0: unspecified)
    note: str = ""

    @property
    def n_chains(self):
        return sum(g.n_chains for g in self.groups)

    def as_dict(self):
        return asdict(self)


def holstein_4x4_single():
    return Workload("holstein-4x4-L40-fp64-1chain", 1,
                    [Lattice(nx=4, n_chains=1, g=1.0, beta=4.0, n_stab=10)], sweeps=20)


def holstein_8x8_batched_global():
    return Workload("holstein-8x8-L80-fp64-64chains-global", 2,
                    [Lattice(nx=8, n_chains=64, g=1.2, beta=8.0, n_stab=8, global_width=1.0)])


def holstein_12x12_mixed(precision=1, n_stab=10):
    return Workload("holstein-12x12-L120-%s-nstab%d-128chains" % ("mixed" if precision else "fp64", n_stab), 3,
                    [Lattice(nx=12, n_chains=128, g=1.5, beta=12.0, n_stab=n_stab)],
                    precision=precision)


def holstein_uneven_batch(n_stab=5):
    # FP32 wraps drift past 1e-5 within 10 slices on every lattice of this
    # batch (3e-5 .. 7e-5), so the recompute interval is 5, a divisor of L = 100
    return Workload("holstein-uneven-6/8/10/16-L100-mixed-nstab%d-4x32chains" % n_stab, 4,
                    [Lattice(nx=n, n_chains=32, beta=10.0, n_stab=n_stab, g_range=(0.8, 1.6))
                     for n in (6, 8, 10, 16)], precision=1)


def holstein_16x16_network():
    return Workload("holstein-16x16-L160-network-64chains", 5,
                    [Lattice(nx=16, n_chains=64, g=1.2, beta=16.0, n_stab=10, proposal=1)])


def holstein_16x16_network_block():
    # the paper's full network sweep: network local moves at every (i, l),
    # then a network block move at every site, then one cumulative accept
    return Workload("holstein-16x16-L160-network-blockmoves-64chains", 5,
                    [Lattice(nx=16, n_chains=64, g=1.2, beta=16.0, n_stab=10, proposal=1,
                             global_width=1.0)])


def holstein_16x16_dqmc():
    # the network workload's lattice and chains under the conventional sweep
    # (mixed precision, recompute every 5 slices): the reference the paper
    # compares the network sampler with
    return Workload("holstein-16x16-L160-dqmc-mixed-nstab5-64chains", 5,
                    [Lattice(nx=16, n_chains=64, g=1.2, beta=16.0, n_stab=5)], precision=1)


ALL = {
    "c1": holstein_4x4_single,
    "c2": holstein_8x8_batched_global,
    "c3": holstein_12x12_mixed,
    "c3-fp64": lambda: holstein_12x12_mixed(0),
    # mixed precision with the FP64 recompute every 6 slices: the largest
    # interval (a divisor of L = 120) whose drift stays within 1e-5
    "c3-gate": lambda: holstein_12x12_mixed(1, n_stab=6),
    "c4": holstein_uneven_batch,
    "c5": holstein_16x16_network,
    "c5-block": holstein_16x16_network_block,
    "c5-dqmc": holstein_16x16_dqmc,
}


def shrink(w, n_chains=None, beta=None, nx=None):
    """A smaller copy of a workload (fewer chains / slices / sites) for parity tests."""
    import copy
    w = copy.deepcopy(w)
    for g in w.groups:
        if n_chains is not None:
            g.n_chains = min(g.n_chains, n_chains)
        if beta is not None:
            g.beta = beta
        if nx is not None:
            g.nx = nx
    return w


def random_fields(seed, L, n, scale=1.0):
    """Gaussian fields x[l, i] from numpy's generator (for tests that set fields directly)."""
    return scale * np.random.default_rng(seed).standard_normal((L, n))


def random_network(seed, scale=0.2):
    """A random flat FP32 weight vector of the 45-64-64-1 network (7169 values)."""
    return (scale * np.random.default_rng(seed).standard_normal(7169)).astype(np.float32)


def random_block_network(seed, L, scale=0.05):
    """A random flat FP32 weight vector of the block-move network for L slices (64 L + 117 values)."""
    return (scale * np.random.default_rng(seed).standard_normal(64 * L + 117)).astype(np.float32)
