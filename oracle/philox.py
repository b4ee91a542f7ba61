"""Philox4x64-10 counter-based random numbers, written from its published
definition (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as
1, 2, 3", SC'11).  Pure Python integers, so it is exact.

The paper does not say how its random numbers are drawn.  Both the oracle and
the GPU library draw every random number of the method from this generator at a
counter that is a pure function of (chain, sweep, slot, kind), so the draws do
not depend on execution order.

Parity: pinned against numpy.random.Philox (an independent implementation of
the same generator) in tests/test_oracle_rng.py.
"""

MASK64 = (1 << 64) - 1

# Round multipliers and Weyl key increments of Philox4x64.
PHILOX_M0 = 0xD2E7470EE14C6C93
PHILOX_M1 = 0xCA5A826395121157
PHILOX_W0 = 0x9E3779B97F4A7C15
PHILOX_W1 = 0xBB67AE8584CAA73B

# Counter word 3: which random decision of the method a block feeds.
KIND_LOCAL = 0      # local move (i, l): word 0 -> displacement, word 1 -> accept
KIND_GLOBAL = 1     # block move of site i: word 0 -> shift, word 1 -> accept
KIND_INIT = 2       # initial field x[l, i]: words 0, 1 -> Box-Muller
KIND_NN = 3         # network-proposed local move: word 0 -> displacement, 1 -> accept
KIND_CUMULATIVE = 4  # cumulative update of one sweep: word 0 -> accept
KIND_COUPLING = 5   # per-chain coupling g: word 0
KIND_NN_GLOBAL = 6  # network-proposed block move of site i: word 0 -> shift, word 1 -> accept
KIND_SCAN = 7       # visiting direction of a network sweep (chain 0, slot 0): word 0 < 1/2 -> forward


def philox4x64_10(ctr, key):
    """One Philox4x64 block of 10 rounds: 4 counter words, 2 key words -> 4 words."""
    x0, x1, x2, x3 = (int(c) & MASK64 for c in ctr)
    k0, k1 = (int(k) & MASK64 for k in key)
    for rnd in range(10):
        p0 = PHILOX_M0 * x0
        p1 = PHILOX_M1 * x2
        hi0, lo0 = p0 >> 64, p0 & MASK64
        hi1, lo1 = p1 >> 64, p1 & MASK64
        x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
        if rnd < 9:
            k0 = (k0 + PHILOX_W0) & MASK64
            k1 = (k1 + PHILOX_W1) & MASK64
    return x0, x1, x2, x3


def uniform53(word):
    """Top 53 bits of a 64-bit word as a double in [0, 1); exact."""
    return (int(word) >> 11) * (1.0 / 9007199254740992.0)


def draw(seed, chain, sweep, slot, kind):
    """The four words of the block at counter (chain, sweep, slot, kind), key (seed, 0)."""
    return philox4x64_10((chain, sweep, slot, kind), (seed, 0))


def uniforms(seed, chain, sweep, slot, kind):
    """Two uniforms in [0, 1) from words 0 and 1 of the block."""
    w = draw(seed, chain, sweep, slot, kind)
    return uniform53(w[0]), uniform53(w[1])
