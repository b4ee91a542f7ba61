"""The training tool writes weights in the layouts the library reads: the
flat vectors of its torch models, read back by the oracle's own network
forwards (written from the layer definitions), give the same outputs; and the
replay of a sweep from logged decisions reproduces the fields."""
import numpy as np
import torch

from oracle import nnmc
from paper_1905_07440_amd import train


def test_local_weights_layout_matches_the_oracle_forward():
    torch.manual_seed(3)
    net = train._local_model(torch).double()
    flat = train.local_flat(net)
    w = nnmc.unpack(flat)
    # compare on the FP32-rounded weights
    with torch.no_grad():
        for p in net.parameters():
            p.copy_(p.float().double())
    X = torch.tensor(np.random.default_rng(1).standard_normal((8, 45)))
    ref = net(X)[:, 0].detach().numpy()
    got = np.array([nnmc.forward(w, X[k].numpy()) for k in range(8)])
    assert np.allclose(got, ref, rtol=0, atol=1e-10)
    est = train.local_estimate(net, X).detach().numpy()
    for k in range(8):
        inp = X[k].numpy()
        m = inp.copy()
        m[22] = -m[22]
        assert abs(est[k] - 0.5 * (nnmc.forward(w, inp) - nnmc.forward(w, m))) < 1e-10


def test_block_weights_layout_matches_the_oracle_forward():
    torch.manual_seed(4)
    L = 12
    bn = train.BlockNet(torch, L)
    for m in (bn.conv, bn.dense, bn.out):
        m.double()
    flat = bn.flat()
    with torch.no_grad():
        for p in bn.parameters():
            p.copy_(p.float().double())
    w = nnmc.unpack_cnn(flat, L)
    inp = torch.tensor(np.random.default_rng(2).standard_normal((5, 3, L)))
    D = torch.tensor([0.3, -0.7, 0.1, 0.9, -0.2], dtype=torch.float64)
    got = bn.estimate(inp, D).detach().numpy()
    for k in range(5):
        x = inp[k].numpy()
        moved = x.copy()
        moved[0] += float(D[k])
        assert abs(got[k] - (nnmc.cnn_forward(w, moved) - nnmc.cnn_forward(w, x))) < 1e-10


def test_replay_reproduces_a_logged_oracle_sweep():
    """A sweep of the oracle with block moves, replayed by the training tool from
    the fields before it and its logged decisions, ends at the oracle's fields,
    and the labels it recovers are the oracle's 2 ln|r| and 2 dln|det M|."""
    from oracle import dqmc, philox
    from oracle.model import Params
    p = Params(nx=4, g=1.2, beta=0.8, n_stab=4, local_width=0.5, global_width=1.0)
    ch = dqmc.Chain(p, seed=13, chain=2)
    x0 = ch.x.copy()
    ch.sweep()
    L, n = p.L, p.n
    acc = np.zeros(L * n, dtype=np.uint8)
    margin = np.zeros(L * n, dtype=np.float32)
    gacc = np.zeros(n, dtype=np.uint8)
    gmargin = np.zeros(n, dtype=np.float32)
    for d in ch.decisions:
        if d.kind == philox.KIND_LOCAL:
            acc[d.slot], margin[d.slot] = d.accept, d.margin
        if d.kind == philox.KIND_GLOBAL:
            gacc[d.slot], gmargin[d.slot] = d.accept, d.margin
    pd = dict(nx=p.nx, L=L, mass=p.mass, omega=p.omega, dtau=p.dtau, g=p.g, local_width=p.local_width,
              global_width=p.global_width)
    Xl, yl, Xb, Db, yb, x_end = train.replay_sweep(pd, x0, acc, margin, gacc, gmargin, 13, 2, 0,
                                                   np.arange(L * n), np.arange(n))
    assert np.allclose(x_end, ch.x, rtol=0, atol=1e-12)
    assert Xl.shape == (L * n, 45) and Xb.shape == (n, 3, L)
    # the labels against the oracle's own ratios (margins are stored in FP32)
    assert np.all(np.isfinite(yl)) and np.all(np.isfinite(yb))
    ch2 = dqmc.Chain(p, seed=13, chain=2)
    import math
    l, i = 0, 5
    ch2.wrap(0)
    for j in range(i):
        ch2.local_move(0, j)
    u0, _ = philox.uniforms(13, 2, 0, l * n + i, philox.KIND_LOCAL)
    d = p.local_width * (2 * u0 - 1)
    r = 1.0 + math.expm1(-p.dtau * p.g * d) * (1.0 - ch2.G[i, i])
    assert abs(yl[l * n + i] - 2 * math.log(abs(r))) < 1e-5
