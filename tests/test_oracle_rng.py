"""Pin the oracle's Philox4x64-10 against numpy.random.Philox, an independent
implementation of the same published generator.  numpy advances its counter
by one before it produces each block, so block(ctr) equals numpy's first block
when it is seeded with ctr - 1."""
import numpy as np
import pytest

from oracle import philox


def numpy_block(ctr, key):
    c = list(ctr)
    # ctr - 1 as a 256-bit little-endian integer
    v = sum(int(w) << (64 * k) for k, w in enumerate(c)) - 1
    v %= 1 << 256
    c = [(v >> (64 * k)) & philox.MASK64 for k in range(4)]
    bg = np.random.Philox(counter=np.array(c, dtype=np.uint64),
                          key=np.array([int(k) for k in key], dtype=np.uint64))
    return tuple(int(w) for w in bg.random_raw(4))


@pytest.mark.parametrize("ctr,key", [
    ((0, 0, 0, 0), (0, 0)),
    ((1, 0, 0, 0), (0, 0)),
    ((5, 6, 7, 8), (11, 12)),
    ((127, 3, 144 * 120 - 1, philox.KIND_LOCAL), (3, 0)),
    ((2**64 - 1, 2**64 - 1, 2**64 - 1, 2**64 - 1), (2**64 - 1, 2**64 - 1)),
    ((0x243F6A8885A308D3, 0x13198A2E03707344, 0xA4093822299F31D0, 0x082EFA98EC4E6C89),
     (0x452821E638D01377, 0xBE5466CF34E90C6C)),
])
def test_philox_matches_numpy(ctr, key):
    assert philox.philox4x64_10(ctr, key) == numpy_block(ctr, key)


def test_philox_random_counters_match_numpy():
    rs = np.random.default_rng(20190517)
    for _ in range(50):
        ctr = tuple(int(v) for v in rs.integers(0, 2**63, size=4))
        key = tuple(int(v) for v in rs.integers(0, 2**63, size=2))
        assert philox.philox4x64_10(ctr, key) == numpy_block(ctr, key)


def test_uniform53_range_and_exactness():
    assert philox.uniform53(0) == 0.0
    top = philox.uniform53(2**64 - 1)
    assert top < 1.0 and top == 1.0 - 2.0**-53
    # the displacement w(2u - 1) is exact in binary64 for w = 0.5
    u = philox.uniform53(0x9E3779B97F4A7C15)
    d = 0.5 * (2.0 * u - 1.0)
    k = 0x9E3779B97F4A7C15 >> 11
    assert d == (2 * k - 2**53) * 2.0**-54
