"""The library's random draws, recomputed on the host (vectorised numpy).

Every random number of the sweep comes from Philox4x64-10 (Salmon, Moraes,
Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11) at counter
(chain, sweep, slot, kind) with key (seed, 0); a uniform is the top 53 bits
of a word.  The training tool uses this to recover the displacement and the
uniform of each logged decision.  Written from the published definition,
like the library's device copy; pinned against numpy.random.Philox.
"""
import numpy as np

M0 = np.uint64(0xD2E7470EE14C6C93)
M1 = np.uint64(0xCA5A826395121157)
W0 = np.uint64(0x9E3779B97F4A7C15)
W1 = np.uint64(0xBB67AE8584CAA73B)
_M32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)

KIND_LOCAL, KIND_GLOBAL, KIND_INIT, KIND_NN, KIND_CUMULATIVE, KIND_COUPLING, KIND_NN_GLOBAL, KIND_SCAN = range(8)


def _mulhilo(a, b):
    """High and low 64-bit words of a * b for a uint64 constant a and uint64 array b."""
    al, ah = a & _M32, a >> _S32
    bl, bh = b & _M32, b >> _S32
    ll, lh, hl, hh = al * bl, al * bh, ah * bl, ah * bh
    mid = (ll >> _S32) + (lh & _M32) + (hl & _M32)
    hi = hh + (lh >> _S32) + (hl >> _S32) + (mid >> _S32)
    return hi, a * b


def philox4x64_10(c0, c1, c2, c3, k0, k1):
    """The four output words of one block for broadcastable counter words."""
    with np.errstate(over="ignore"):
        c0, c1, c2, c3, k0, k1 = np.broadcast_arrays(*(np.asarray(v, dtype=np.uint64) for v in
                                                       (c0, c1, c2, c3, k0, k1)))
        c0, c1, c2, c3, k0, k1 = (v.copy() for v in (c0, c1, c2, c3, k0, k1))
        for rnd in range(10):
            hi0, lo0 = _mulhilo(M0, c0)
            hi1, lo1 = _mulhilo(M1, c2)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
            if rnd < 9:
                k0 = k0 + W0
                k1 = k1 + W1
    return c0, c1, c2, c3


def uniform53(w):
    return (np.asarray(w, dtype=np.uint64) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def uniforms(seed, chain, sweep, slot, kind):
    """Words 0 and 1 of the block at (chain, sweep, slot, kind) as uniforms in [0, 1)."""
    w = philox4x64_10(chain, sweep, slot, kind, seed, 0)
    return uniform53(w[0]), uniform53(w[1])
