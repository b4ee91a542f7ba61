"""Pins of the oracle's network path: the forward pass against torch's own
layers on the same FP32 weights, the patch layout against a direct index
formula, the colour classes against the patch geometry, and the cumulative
ratio against log W from scratch."""
import math

import numpy as np
import pytest
import torch
import torch.nn.functional as F

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


def random_cnn(seed, L, scale=0.2):
    return (scale * np.random.default_rng(seed).standard_normal(nnmc.cnn_count(L))).astype(np.float32)


@pytest.mark.parametrize("L", [8, 20])
def test_cnn_forward_matches_torch(L):
    """The block-move network against torch.nn.functional: circular padding
    on the right by K - 1, conv1d with stride S, sigmoid, channel-major
    flatten, linear + sigmoid, linear."""
    w = random_cnn(11, L)
    Wc, bc, Wd, bd, Wo, bo = nnmc.unpack_cnn(w, L)
    rng = np.random.default_rng(3)
    for _ in range(4):
        inp = rng.standard_normal((3, L))
        t = torch.tensor(inp, dtype=torch.float64)[None]
        t = torch.cat([t, t[:, :, :nnmc.CNN_K - 1]], dim=2)
        h = torch.sigmoid(F.conv1d(t, torch.tensor(Wc), torch.tensor(bc), stride=nnmc.CNN_S))
        h = torch.sigmoid(F.linear(h.reshape(-1), torch.tensor(Wd), torch.tensor(bd)))
        ref = float(F.linear(h, torch.tensor(Wo)[None], torch.tensor([bo]))[0])
        assert abs(nnmc.cnn_forward((Wc, bc, Wd, bd, Wo, bo), inp) - ref) < 1e-12


def test_cnn_weight_count():
    assert nnmc.cnn_count(80) == 64 * 80 + 117
    with pytest.raises(ValueError):
        nnmc.cnn_count(9)


def test_cnn_inputs_are_c4_symmetric():
    """Rotating the lattice by 90 degrees about site i leaves its three input
    channels unchanged (the neighbour means are what gives the network C4
    symmetry); the channels are the column and the hand-summed means."""
    nx, L = 6, 4
    x = np.random.default_rng(9).standard_normal((L, nx * nx))
    i = 2 + nx * 3
    ix, iy = i % nx, i // nx
    rot = np.empty_like(x)
    for jy in range(nx):
        for jx in range(nx):
            dx, dy = jx - ix, jy - iy
            kx, ky = (ix - dy) % nx, (iy + dx) % nx       # (dx, dy) -> (-dy, dx)
            rot[:, kx + nx * ky] = x[:, jx + nx * jy]
    assert np.allclose(nnmc.cnn_inputs(nx, x, i), nnmc.cnn_inputs(nx, rot, i), atol=1e-14)
    inp = nnmc.cnn_inputs(nx, x, i)
    s = lambda dx, dy: x[:, (ix + dx) % nx + nx * ((iy + dy) % nx)]
    assert np.allclose(inp[0], x[:, i])
    assert np.allclose(inp[1], (s(1, 0) + s(-1, 0) + s(0, 1) + s(0, -1)) / 4)
    assert np.allclose(inp[2], (s(1, 1) + s(1, -1) + s(-1, 1) + s(-1, -1)) / 4)


def test_cnn_colour_classes_do_not_interact():
    nx = 6
    order = nnmc.cnn_colour_order(nx)
    assert sorted(order) == list(range(nx * nx))
    per = nx * nx // 4
    for k in range(4):
        cls = order[k * per:(k + 1) * per]
        for a in cls:
            for b in cls:
                if a == b:
                    continue
                dx = min((a % nx - b % nx) % nx, (b % nx - a % nx) % nx)
                dy = min((a // nx - b // nx) % nx, (b // nx - a // nx) % nx)
                assert max(dx, dy) >= 2, (a, b)
    with pytest.raises(ValueError):
        nnmc.cnn_colour_order(5)


def test_cumulative_ratio_with_block_moves_and_two_inner_sweeps():
    """With network block moves and n_u = 2 the sweep's proposal X' follows
    from the recorded decisions, and log p_c + sum y = 2 dlogdet =
    (log W(X') - log W(X)) + dS_b."""
    from oracle import philox
    p = Params(nx=4, beta=0.8, g=1.2, n_stab=4, local_width=0.5, global_width=0.4)
    ch = dqmc.Chain(p, seed=7, chain=1)
    nn = nnmc.NNChain(ch, random_weights(3), cnn=random_cnn(5, p.L), nu=2)
    x0 = ch.x.copy()
    lw0 = ch.log_weight()
    nn.sweep()
    assert nn.inner_proposals == 2 * p.L * p.n and nn.block_proposals == 2 * p.n
    xp = x0.copy()
    for kind, sw, slot, acc, _ in nn.decisions:
        if kind == philox.KIND_NN and acc:
            u0, _ = philox.uniforms(7, 1, 0, slot, philox.KIND_NN)
            r = slot % (p.L * p.n)
            xp[r // p.n, r % p.n] += p.local_width * (2 * u0 - 1)
        if kind == philox.KIND_NN_GLOBAL and acc:
            u0, _ = philox.uniforms(7, 1, 0, slot, philox.KIND_NN_GLOBAL)
            xp[:, slot % p.n] += p.global_width * (2 * u0 - 1)
    lw1 = ch.log_weight(xp)
    dsb = model.bosonic_action(p, xp) - model.bosonic_action(p, x0)
    assert abs((nn.last_log_pc + nn.last_sum_y) - (lw1 - lw0 + dsb)) < 1e-9
    assert np.array_equal(ch.x, xp if nn.cumulative_accepts else x0)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_local_and_block_estimates_are_odd_under_the_reverse_move(seed):
    """The estimate of a move and of the move that undoes it cancel: for a
    local move y(x -> x + d e_li) = -y(x + d e_li -> x), and for a block
    move f(x_i + D) - f(x_i) = -(f((x_i + D) - D) - f(x_i + D))."""
    rng = np.random.default_rng(seed)
    nx, L = 4, 8
    x = rng.standard_normal((L, nx * nx))
    w = nnmc.unpack(random_weights(seed))
    cnn = nnmc.unpack_cnn(random_cnn(seed, L), L)
    for _ in range(5):
        l, i, d = int(rng.integers(L)), int(rng.integers(nx * nx)), float(rng.uniform(-0.5, 0.5))
        xm = x.copy()
        xm[l, i] += d
        y = nnmc.local_estimate(w, nx, x, l, i, d)
        assert abs(y + nnmc.local_estimate(w, nx, xm, l, i, -d)) < 1e-12 * max(1.0, abs(y))
        # the raw output is not odd: the reverse move of f(d) alone would not cancel
        f_fwd = nnmc.forward(w, nnmc.patch(nx, x, l, i, d))
        f_rev = nnmc.forward(w, nnmc.patch(nx, xm, l, i, -d))
        assert abs(f_fwd + f_rev) > 1e-6
        xb = x.copy()
        xb[:, i] += d
        yb = nnmc.block_estimate(cnn, nx, x, i, d)
        assert abs(yb + nnmc.block_estimate(cnn, nx, xb, i, -d)) < 1e-12 * max(1.0, abs(yb))


def _path_log_prob(nn, p, steps, x_start):
    """log of the probability (proposal densities left out: uniform and
    symmetric) that the network sweep takes the given steps from x_start,
    each step's points with their displacement and decision; every estimate
    evaluated afresh with the network on the state the step starts from."""
    w, cnn = nn.weights, nn.cnn
    x = x_start.copy()
    L = p.L
    lp = 0.0
    for kind, pts in steps:
        for l, i, d, accepted in pts:
            if kind == "local":
                y = nnmc.local_estimate(w, p.nx, x, l, i, d)
                ds = model.local_action_change(p, x[l, i], x[(l - 1) % L, i], x[(l + 1) % L, i], d)
            else:
                y = nnmc.block_estimate(cnn, p.nx, x, i, d)
                ds = model.global_action_change(p, float(np.sum(x[:, i])), d, L)
            a = y - ds
            lp += min(0.0, a) if accepted else math.log1p(-math.exp(min(0.0, a)))
        for l, i, d, accepted in pts:
            if accepted:
                if kind == "local":
                    x[l, i] += d
                else:
                    x[:, i] += d
    return lp, x


@pytest.mark.parametrize("seed,nu,block", [(5, 1, False), (6, 2, False), (7, 1, True), (8, 2, True)])
def test_cumulative_ratio_is_the_metropolis_hastings_ratio_of_the_composite_move(seed, nu, block):
    """The cumulative accept is exact: with P(path) the probability of the
    inner sweep's steps from X to X' and P(reverse) that of the same steps
    in reverse order, each accepted move undone by its opposite displacement
    and each rejected one rejected again, taken from X' by the opposite scan
    direction,
        log p_c = [log W(X') + log P(reverse)] - [log W(X) + log P(path)].
    Both path probabilities are evaluated step by step with fresh network
    evaluations, so an estimate that is not odd under the reverse move fails."""
    p = Params(nx=4, beta=0.8, g=1.2, n_stab=4, local_width=0.5, global_width=0.4 if block else 0.0)
    ch = dqmc.Chain(p, seed=seed, chain=0)
    nn = nnmc.NNChain(ch, random_weights(seed), cnn=random_cnn(seed + 1, p.L) if block else None, nu=nu)
    reversed_seen = set()
    for _ in range(4):
        x0 = ch.x.copy()
        lw0 = ch.log_weight()
        nn.sweep()
        reversed_seen.add(nn.last_reversed)
        fwd = [(kind, [(l, i, d, acc) for l, i, d, acc, _, _ in pts]) for kind, _, pts, _ in nn.path]
        lp_f, xp = _path_log_prob(nn, p, fwd, x0)
        assert np.array_equal(xp, nn.proposal)
        back = [(kind, [(l, i, -d if acc else d, acc) for l, i, d, acc in pts]) for kind, pts in fwd[::-1]]
        lp_r, xb = _path_log_prob(nn, p, back, xp)
        assert np.allclose(xb, x0, rtol=0, atol=1e-12)
        lw1 = ch.log_weight(xp)
        assert abs((lw1 + lp_r) - (lw0 + lp_f) - nn.last_log_pc) < 1e-9
    assert reversed_seen == {False, True}, "both scan directions occur"


def test_reversed_sweep_visits_the_schedule_backwards():
    p = Params(nx=4, beta=0.8, g=1.2, n_stab=4, global_width=0.4)
    for s in range(8):
        ch = dqmc.Chain(p, seed=9, chain=0)
        ch.sweep_index = s
        nn = nnmc.NNChain(ch, random_weights(9), cnn=random_cnn(10, p.L), nu=2)
        nn.sweep()
        kinds = [k for k, _, _, _ in nn.path]
        us = [u for _, u, _, _ in nn.path]
        fwd_kinds = ["local"] * 32 + ["block"] * 8
        fwd_us = [0] * 16 + [1] * 16 + [0] * 4 + [1] * 4
        if nnmc.scan_reversed(9, s):
            assert kinds == fwd_kinds[::-1] and us == fwd_us[::-1]
        else:
            assert kinds == fwd_kinds and us == fwd_us
