"""Write the oracle's results for the large parity cases into tests/golden/.

    python tests/golden/make_golden.py [case ...]

Only oracle/ and the seeded inputs of workloads/ are used: every stored value
comes from the plain FP64 CPU implementation, never from the GPU library.  The
GPU tests replay the stored decisions inside the tie band and compare fields,
G and log|det M| with the stored values.  G is stored in FP32: the mixed
precision bar is 1e-5 relative, 150 times the FP32 rounding of the stored
copy.

Cases
  c3gate  128 chains of 12x12, L = 120, n_stab = 6 (the mixed workload at the
          stated accuracy): chains 0 and 127, one upward and one downward
          sweep; the tracked G and log det before the last recompute of each
          sweep are kept too
  c4n16   the uneven batch (6x6 ... 16x16, L = 100, n_stab = 5, g per chain):
          chain 96, the first 16x16 chain, one upward sweep
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import dqmc, philox  # noqa: E402
from oracle.model import Params, chain_coupling  # noqa: E402
import workloads  # noqa: E402


def params_of(g, gval=None):
    return Params(nx=g.nx, t=g.t, mu=g.mu, mass=g.mass, omega=g.omega, g=g.g if gval is None else gval,
                  beta=g.beta, dtau=g.dtau, n_stab=g.n_stab, local_width=g.local_width,
                  global_width=g.global_width)


def local_bits(ch, sweep):
    bits = np.zeros(ch.p.L * ch.p.n, dtype=np.uint8)
    for d in ch.decisions:
        if d.kind == philox.KIND_LOCAL and d.sweep == sweep:
            bits[d.slot] = 1 if d.accept else 0
    return bits


def run_chain(p, seed, chain, sweeps):
    ch = dqmc.Chain(p, seed, chain)
    out = {}
    for s in range(sweeps):
        ch.sweep()
        out["bits%d" % s] = np.packbits(local_bits(ch, s))
        out["G%d" % s] = ch.G.astype(np.float32)
        out["Gtr%d" % s] = ch.G_tracked.astype(np.float32)
        out["logdet%d" % s] = np.array(ch.logdet)
        out["logdet_tr%d" % s] = np.array(ch.logdet_tracked)
        out["accepts%d" % s] = np.array(ch.local_accepts)
        out["x%d" % s] = ch.x.copy()
    out["g"] = np.array(p.g)
    return out


def case_c3gate():
    w = workloads.ALL["c3-gate"]()
    g = w.groups[0]
    for c in (0, 127):
        t0 = time.time()
        out = run_chain(params_of(g), w.seed, c, 2)
        np.savez_compressed(os.path.join(HERE, "c3gate_chain%d.npz" % c), **out)
        print("c3gate chain %d: %.0f s" % (c, time.time() - t0), flush=True)


def case_c4n16():
    w = workloads.ALL["c4"]()
    g = w.groups[3]
    c = 96
    gval = chain_coupling(w.seed, c, *g.g_range)
    t0 = time.time()
    out = run_chain(params_of(g, gval), w.seed, c, 1)
    np.savez_compressed(os.path.join(HERE, "c4n16_chain%d.npz" % c), **out)
    print("c4n16 chain %d: %.0f s" % (c, time.time() - t0), flush=True)


CASES = {"c3gate": case_c3gate, "c4n16": case_c4n16}

if __name__ == "__main__":
    for name in (sys.argv[1:] or list(CASES)):
        CASES[name]()
