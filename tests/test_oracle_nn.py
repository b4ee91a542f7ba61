"""Pins of the oracle's network path: the forward pass against torch's own
layers on the same FP32 weights, the patch layout against a direct index
formula, the colour classes against the patch geometry, and the cumulative
ratio against log W from scratch."""
import math

import numpy as np
import pytest
import torch

from oracle import dqmc, model, nnmc
from oracle.model import Params


def random_weights(seed):
    return (0.2 * np.random.default_rng(seed).standard_normal(nnmc.N_WEIGHTS)).astype(np.float32)


@pytest.mark.parametrize("kind", [0, 1])
def test_forward_matches_torch(kind):
    w = random_weights(1)
    W1, b1, W2, b2, W3, b3 = nnmc.unpack(w)
    net = torch.nn.Sequential(
        torch.nn.Linear(45, 64), torch.nn.ReLU() if kind == 0 else torch.nn.Softplus(),
        torch.nn.Linear(64, 64), torch.nn.ReLU() if kind == 0 else torch.nn.Softplus(),
        torch.nn.Linear(64, 1)).double()
    with torch.no_grad():
        net[0].weight.copy_(torch.from_numpy(W1)); net[0].bias.copy_(torch.from_numpy(b1))
        net[2].weight.copy_(torch.from_numpy(W2)); net[2].bias.copy_(torch.from_numpy(b2))
        net[4].weight.copy_(torch.from_numpy(W3[None, :])); net[4].bias.fill_(float(b3))
    rs = np.random.default_rng(2)
    for _ in range(10):
        inp = rs.standard_normal(45)
        ref = float(net(torch.from_numpy(inp)[None, :])[0, 0])
        assert abs(nnmc.forward(nnmc.unpack(w), inp, kind) - ref) < 1e-12


def test_weight_count():
    assert nnmc.N_WEIGHTS == 7169


def test_patch_layout():
    nx, L = 4, 8
    x = np.arange(L * nx * nx, dtype=float).reshape(L, nx * nx)
    l, i, d = 1, 3, 0.25            # site (3, 0): x-neighbours wrap to ix = 0 and 2
    pt = nnmc.patch(nx, x, l, i, d)
    assert pt[22] == d
    assert pt[9 * 0 + 3 * 1 + 1] == x[(l - 2) % L, i]           # dl=-2, same site
    assert pt[9 * 2 + 3 * 1 + 2] == x[l, 0]                     # dx=+1 wraps
    assert pt[9 * 2 + 3 * 0 + 0] == x[l, 2 + nx * 3]            # dx=-1, dy=-1 wraps in y
    assert pt[9 * 4 + 3 * 2 + 1] == x[(l + 2) % L, 3 + nx * 1]  # dl=+2, dy=+1


def test_colour_classes_do_not_interact():
    nx, L = 4, 8
    order = nnmc.colour_order(nx, L)
    assert sorted(order) == sorted((l, i) for l in range(L) for i in range(nx * nx))
    size = len(order) // 16
    for k in range(16):
        cls = order[k * size:(k + 1) * size]
        for (l1, i1) in cls:
            for (l2, i2) in cls:
                if (l1, i1) == (l2, i2):
                    continue
                dl = min((l1 - l2) % L, (l2 - l1) % L)
                dx = min((i1 % nx - i2 % nx) % nx, (i2 % nx - i1 % nx) % nx)
                dy = min((i1 // nx - i2 // nx) % nx, (i2 // nx - i1 // nx) % nx)
                assert not (dl <= 2 and dx <= 1 and dy <= 1)


def test_colour_order_rejects_odd_lattice():
    with pytest.raises(ValueError):
        nnmc.colour_order(3, 8)


def test_cumulative_ratio_is_exact_weight_ratio_minus_network_path():
    """log p_c + sum y = 2 dlogdet = (log W(X') - log W(X)) + dS_b."""
    p = Params(nx=4, beta=0.8, g=1.2, n_stab=4, local_width=0.5)
    ch = dqmc.Chain(p, seed=5, chain=0)
    nn = nnmc.NNChain(ch, random_weights(3))
    x0 = ch.x.copy()
    lw0 = ch.log_weight()
    nn.sweep()
    assert nn.inner_proposals == p.L * p.n
    # reconstruct X' from the inner decisions
    xp = x0.copy()
    from oracle import philox
    for kind, sw, slot, acc, _ in nn.decisions:
        if kind == philox.KIND_NN and acc:
            u0, _ = philox.uniforms(5, 0, 0, slot, philox.KIND_NN)
            xp[slot // p.n, slot % p.n] += p.local_width * (2 * u0 - 1)
    lw1 = ch.log_weight(xp)
    dsb = model.bosonic_action(p, xp) - model.bosonic_action(p, x0)
    assert abs((nn.last_log_pc + nn.last_sum_y) - (lw1 - lw0 + dsb)) < 1e-9
    if nn.cumulative_accepts:
        assert np.array_equal(ch.x, xp)
    else:
        assert np.array_equal(ch.x, x0)
    assert math.isfinite(nn.last_log_pc)
