"""The host copy of the library's draws (paper_1905_07440_amd/draws.py, used
by the training tool) against numpy.random.Philox, an independent
implementation of the same generator (numpy advances its counter before each
block, so block(ctr) is numpy's first block seeded with ctr - 1)."""
import numpy as np

from paper_1905_07440_amd import draws


def numpy_block(ctr, key):
    v = (sum(int(w) << (64 * k) for k, w in enumerate(ctr)) - 1) % (1 << 256)
    c = [(v >> (64 * k)) & ((1 << 64) - 1) for k in range(4)]
    bg = np.random.Philox(counter=np.array(c, dtype=np.uint64), key=np.array(key, dtype=np.uint64))
    return [int(w) for w in bg.random_raw(4)]


def test_vectorised_blocks_match_numpy():
    rs = np.random.default_rng(5)
    ctr = rs.integers(0, 2**63, size=(4, 40), dtype=np.uint64)
    ctr[:, 0] = 0
    ctr[:, 1] = np.iinfo(np.uint64).max
    key = rs.integers(0, 2**63, size=(2, 40), dtype=np.uint64)
    out = draws.philox4x64_10(ctr[0], ctr[1], ctr[2], ctr[3], key[0], key[1])
    for j in range(40):
        ref = numpy_block([int(ctr[k, j]) for k in range(4)], [int(key[0, j]), int(key[1, j])])
        assert [int(out[k][j]) for k in range(4)] == ref


def test_uniforms_are_top_53_bits():
    u0, u1 = draws.uniforms(3, np.arange(5), 7, 11, draws.KIND_LOCAL)
    w = draws.philox4x64_10(np.arange(5), 7, 11, 0, 3, 0)
    assert np.array_equal(u0, (w[0] >> np.uint64(11)).astype(np.float64) / 2.0**53)
    assert np.all((u1 >= 0) & (u1 < 1))
