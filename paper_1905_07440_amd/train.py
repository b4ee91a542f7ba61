"""Training of the two proposal networks from DQMC runs of this library.

Paper, Local Updates and Global Updates: the networks are fitted to the
weight ratios that conventional DQMC gives on configurations it samples,
8 x 10^4 samples, 6 x 10^4 to train on and 2 x 10^4 to validate.  Here the
conventional sweep is the library's own (FP64), and the ratio of every
proposal is read back from its decision log.  The log holds ln u - ln R, the
draws u and d are recomputed on the host (draws.py), so
    local move   2 ln|r|          = ln u - margin + dS_b(d)
    block move   2 dln|det M|     = ln u - margin + dS_b(column shift d)
the fermionic parts the networks estimate (the sampler adds the bosonic
change exactly).  The field configuration at each proposal is replayed from
the fields before the sweep and the logged decisions; the replay must end at
the fields the library holds after the sweep.

The workloads (t = 1, mu = 0, Omega = 1, g = 1.2, dtau = 0.1, local moves
U(-0.5, 0.5), one block move U(-1, 1) per site and sweep): for the local-move
network, which sees five slices and three sites in each direction, the
batched 8x8 lattice at beta = 8 (L = 80), 64 chains; for the block-move
network, whose dense layer is sized by L and whose estimate of a column
shift depends on the lattice it was fitted on, the lattice it runs on,
16x16 at beta = 16 (L = 160), 32 chains.  Samples are drawn uniformly at
random from the proposals of many chains and sweeps after a warm-up.

    python -m paper_1905_07440_amd.train data [--kind local|block] [--out F]   (GPU)
    python -m paper_1905_07440_amd.train fit  [--kind local|block] [--data F]  (torch)

`fit` writes the flat FP32 weights that hq_set_network / hq_set_block_network
take into paper_1905_07440_amd/weights/, with a JSON report beside them.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "weights")

LATTICE = dict(t=1.0, mu=0.0, mass=1.0, omega=1.0, g=1.2, dtau=0.1, local_width=0.5, global_width=1.0)
KINDS = {"local": dict(nx=8, beta=8.0, n_stab=8, chains=64),
         "block": dict(nx=16, beta=16.0, n_stab=10, chains=32)}
SEED = 1001
N_TRAIN, N_VAL = 60000, 20000


def weight_file(kind, L=None, folder=WEIGHTS):
    return os.path.join(folder, "local_45_64_64_1.npy" if kind == "local" else "block_L%d.npy" % L)


def load_weights(kind, L=None):
    """The trained flat FP32 weights (None if they have not been trained)."""
    f = weight_file(kind, L)
    return np.load(f).astype(np.float32) if os.path.exists(f) else None


# ---------------------------------------------------------------------------
# data
# ---------------------------------------------------------------------------
def _neighbours(nx):
    idx = np.arange(nx * nx)
    ix, iy = idx % nx, idx // nx
    site = lambda dx, dy: (ix + dx) % nx + nx * ((iy + dy) % nx)
    patch = np.stack([site(dx, dy) for dy in (-1, 0, 1) for dx in (-1, 0, 1)], axis=1)   # [N][9], 3(dy+1)+(dx+1)
    nn = np.stack([site(1, 0), site(-1, 0), site(0, 1), site(0, -1)], axis=1)
    nnn = np.stack([site(1, 1), site(1, -1), site(-1, 1), site(-1, -1)], axis=1)
    return patch, nn, nnn


def replay_sweep(p, x_before, acc, margin, gacc, gmargin, seed, chain, sweep, want_local, want_block):
    """Replay one sweep (slices ascending, sites ascending, then one block move
    per site) of one chain.  want_local: slots whose (patch, label) to return;
    want_block: sites whose (channels, shift, label) to return.  Returns
    (local inputs [k][45], local labels, block channels [k][3][L], shifts,
    block labels, fields after the sweep)."""
    from . import draws
    nx, L = p["nx"], p["L"]
    n = nx * nx
    patch_sites, nn, nnn = _neighbours(nx)
    slots = np.arange(L * n)
    u0, u1 = draws.uniforms(seed, chain, sweep, slots, draws.KIND_LOCAL)
    d = p["local_width"] * (2.0 * u0 - 1.0)
    x = x_before.copy()
    kin_c = p["mass"] / p["dtau"]
    pot_c = p["dtau"] * 0.5 * p["mass"] * p["omega"] ** 2
    Xl, yl = [], []
    want = np.zeros(L * n, dtype=bool)
    want[want_local] = True
    for l in range(L):
        dl = d[l * n:(l + 1) * n]
        al = acc[l * n:(l + 1) * n].astype(bool)
        row0 = x[l].copy()
        for i in np.nonzero(want[l * n:(l + 1) * n])[0]:
            row = row0 + np.where(al & (np.arange(n) < i), dl, 0.0)   # moves of this slice before site i
            inp = np.empty(45)
            for k, dlk in enumerate(range(-2, 3)):
                src = row if dlk == 0 else x[(l + dlk) % L]
                inp[9 * k:9 * k + 9] = src[patch_sites[i]]
            inp[22] = dl[i]
            a, prev, nxt = row[i], x[(l - 1) % L, i], x[(l + 1) % L, i]
            ds = kin_c * (dl[i] * (2 * a - prev - nxt) + dl[i] ** 2) + pot_c * (2 * a * dl[i] + dl[i] ** 2) \
                - p["dtau"] * p["g"] * dl[i]
            Xl.append(inp)
            yl.append(np.log(u1[l * n + i]) - float(margin[l * n + i]) + ds)
        x[l] = row0 + np.where(al, dl, 0.0)
    # block moves, sites ascending
    sites = np.arange(n)
    g0, g1 = draws.uniforms(seed, chain, sweep, sites, draws.KIND_GLOBAL)
    D = p["global_width"] * (2.0 * g0 - 1.0)
    mo2 = p["mass"] * p["omega"] ** 2
    Xb, Db, yb = [], [], []
    wantb = set(int(v) for v in want_block)
    for i in range(n):
        if i in wantb:
            ch = np.stack([x[:, i], x[:, nn[i]].mean(axis=1), x[:, nnn[i]].mean(axis=1)])
            ds = p["dtau"] * (mo2 * D[i] * x[:, i].sum() + 0.5 * mo2 * L * D[i] ** 2 - p["g"] * L * D[i])
            Xb.append(ch)
            Db.append(D[i])
            yb.append(np.log(g1[i]) - float(gmargin[i]) + ds)
        if gacc[i]:
            x[:, i] += D[i]
    return (np.array(Xl).reshape(-1, 45), np.array(yl), np.array(Xb).reshape(-1, 3, L), np.array(Db),
            np.array(yb), x)


def generate(kind, out, warmup=20, samples=N_TRAIN + N_VAL, seed=SEED, log=print):
    """Run the library's FP64 sweep and collect `samples` proposals of one kind."""
    import torch   # noqa: F401  (initialises the device before the library loads)
    from . import hq
    cfg = dict(LATTICE, **KINDS[kind])
    chains = cfg.pop("chains")
    L = int(round(cfg["beta"] / cfg["dtau"]))
    n = cfg["nx"] ** 2
    p = dict(cfg, L=L)
    grp = hq.make_group(cfg["nx"], chains, t=cfg["t"], mu=cfg["mu"], mass=cfg["mass"], omega=cfg["omega"],
                        g=cfg["g"], beta=cfg["beta"], dtau=cfg["dtau"], n_stab=cfg["n_stab"],
                        local_width=cfg["local_width"], global_width=cfg["global_width"])
    ctx = hq.Context([grp], precision=hq.PREC_FP64, seed=seed, record=True)
    t0 = time.time()
    ctx.sweep(warmup)
    rng = np.random.default_rng(seed)
    # local moves: 10 sweeps of every chain, a random subset of each sweep's
    # L N proposals; block moves: every site of enough sweeps
    sweeps = 10 if kind == "local" else int(np.ceil(samples / (chains * n)))
    quota = int(np.ceil(samples / (sweeps * chains)))
    if kind == "block":
        quota = min(quota, n)
    X, Y, D = [], [], []
    sweep = warmup
    for s in range(sweeps):
        before = [ctx.fields(c) for c in range(chains)]
        ctx.sweep(1)
        for c in range(chains):
            acc, margin = ctx.decisions(c, hq.KIND_LOCAL)
            gacc, gmargin = ctx.decisions(c, hq.KIND_GLOBAL)
            if kind == "local":
                wl, wb = rng.choice(L * n, size=quota, replace=False), []
            else:
                wl, wb = [], rng.choice(n, size=quota, replace=False)
            Xl, yl, Xb, Db, yb, x_end = replay_sweep(p, before[c], acc, margin, gacc, gmargin, seed, c, sweep,
                                                     wl, wb)
            after = ctx.fields(c)
            err = float(np.max(np.abs(x_end - after)))
            if err > 1e-9:
                raise RuntimeError("replay of chain %d sweep %d ends %g away from the library's fields"
                                   % (c, sweep, err))
            if kind == "local":
                X.append(Xl); Y.append(yl)
            else:
                X.append(Xb); Y.append(yb); D.append(Db)
        sweep += 1
        log("sweep %d/%d: %d samples, %.0f s" % (s + 1, sweeps, sum(len(v) for v in Y), time.time() - t0))
    st = [ctx.stats(c) for c in range(chains)]
    ctx.close()
    X = np.concatenate(X)[:samples]
    Y = np.concatenate(Y)[:samples]
    extra = {"D": np.concatenate(D)[:samples]} if kind == "block" else {}
    meta = dict(kind=kind, chains=chains, warmup=warmup, sweeps=sweeps, seed=seed, L=L, **cfg,
                local_acceptance=sum(v["local_accepts"] for v in st) / sum(v["local_proposals"] for v in st),
                block_acceptance=sum(v["global_accepts"] for v in st) / max(1, sum(v["global_proposals"] for v in st)))
    np.savez_compressed(out, X=X.astype(np.float32), Y=Y, meta=json.dumps(meta), **extra)
    log("wrote %s: %d samples" % (out, len(Y)))
    return out


# ---------------------------------------------------------------------------
# fitting (torch)
# ---------------------------------------------------------------------------
def _local_model(torch):
    return torch.nn.Sequential(torch.nn.Linear(45, 64), torch.nn.ReLU(), torch.nn.Linear(64, 64), torch.nn.ReLU(),
                               torch.nn.Linear(64, 1))


def local_flat(net):
    """The 7169 FP32 values of hq_set_network: W1[64][45], b1, W2[64][64], b2, W3[64], b3."""
    W1, b1, W2, b2, W3, b3 = (v.detach().cpu().numpy() for v in net.parameters())
    flat = np.concatenate([W1.reshape(-1), b1, W2.reshape(-1), b2, W3.reshape(-1), b3]).astype(np.float32)
    assert flat.size == 7169
    return flat


def local_estimate(net, X):
    """The sampler's estimate: the odd part (f(d) - f(-d)) / 2, d at input 22."""
    Xm = X.clone()
    Xm[:, 22] = -Xm[:, 22]
    return 0.5 * (net(X) - net(Xm))[:, 0]


class BlockNet:
    """The block-move network of hq_set_block_network: circular conv along l
    (4 channels, kernel 4, stride 2), sigmoid, 32 sigmoid units, linear."""

    def __init__(self, torch, L):
        self.t = torch
        self.L = L
        self.conv = torch.nn.Conv1d(3, 4, 4, stride=2)
        self.dense = torch.nn.Linear(4 * (L // 2), 32)
        self.out = torch.nn.Linear(32, 1)

    def parameters(self):
        return list(self.conv.parameters()) + list(self.dense.parameters()) + list(self.out.parameters())

    def f(self, inp):
        t = self.t
        h = t.cat([inp, inp[:, :, :3]], dim=2)                        # periodic in l: slices 2p .. 2p+3 mod L
        h = t.sigmoid(self.conv(h)).reshape(inp.shape[0], -1)         # channel-major c * (L/2) + p
        return self.out(t.sigmoid(self.dense(h)))[:, 0]

    def estimate(self, inp, D):
        moved = inp.clone()
        moved[:, 0, :] += D[:, None]
        return self.f(moved) - self.f(inp)

    def flat(self):
        parts = [self.conv.weight, self.conv.bias, self.dense.weight, self.dense.bias, self.out.weight[0],
                 self.out.bias]
        return np.concatenate([v.detach().cpu().numpy().reshape(-1) for v in parts]).astype(np.float32)


def fit(kind, data, epochs=None, seed=SEED, log=print, device="cpu", folder=WEIGHTS):
    import torch
    torch.manual_seed(seed)
    z = np.load(data)
    meta = json.loads(str(z["meta"]))
    X = torch.tensor(z["X"], dtype=torch.float32, device=device)
    Y = torch.tensor(z["Y"], dtype=torch.float32, device=device)
    n = min(len(Y), N_TRAIN + N_VAL)
    ntr = n * N_TRAIN // (N_TRAIN + N_VAL)
    perm = torch.randperm(n, generator=torch.Generator().manual_seed(seed)).to(device)
    tr, va = perm[:ntr], perm[ntr:n]
    if kind == "local":
        net = _local_model(torch).to(device)
        params = list(net.parameters())
        est = lambda idx: local_estimate(net, X[idx])
        epochs = epochs or 150
    else:
        D = torch.tensor(z["D"], dtype=torch.float32, device=device)
        bn = BlockNet(torch, meta["L"])
        for m in (bn.conv, bn.dense, bn.out):
            m.to(device)
        params = bn.parameters()
        est = lambda idx: bn.estimate(X[idx], D[idx])
        epochs = epochs or 300
    # the labels are fitted in units of their spread; the output layer takes
    # the factor back before the weights are written
    scale = float(torch.sqrt(torch.mean(Y[tr] ** 2)))
    Yn = Y / scale
    opt = torch.optim.Adam(params, lr=2e-3)
    sched = torch.optim.lr_scheduler.CosineAnnealingLR(opt, T_max=epochs)
    bs = 512
    t0 = time.time()
    for ep in range(epochs):
        order = tr[torch.randperm(ntr, device=device)]
        for k in range(0, ntr, bs):
            idx = order[k:k + bs]
            loss = torch.mean((est(idx) - Yn[idx]) ** 2)
            opt.zero_grad()
            loss.backward()
            opt.step()
        sched.step()
        if ep % 25 == 0 or ep == epochs - 1:
            with torch.no_grad():
                r_tr = scale * float(torch.sqrt(torch.mean((est(tr) - Yn[tr]) ** 2)))
                r_va = scale * float(torch.sqrt(torch.mean((est(va) - Yn[va]) ** 2)))
            log("epoch %d: rms error train %.4g, validation %.4g (%.0f s)" % (ep, r_tr, r_va, time.time() - t0))
    with torch.no_grad():
        last = net[4] if kind == "local" else bn.out
        last.weight.mul_(scale)
        last.bias.mul_(scale)
        res = est(va) - Y[va]
        yv = Y[va]
        report = {"kind": kind, "samples": {"train": int(ntr), "validation": int(n - ntr)}, "epochs": epochs,
                  "seed": seed, "data": meta,
                  "validation": {"rms_error": float(torch.sqrt(torch.mean(res ** 2))),
                                 "rms_label": float(torch.sqrt(torch.mean(yv ** 2))),
                                 "r2": float(1.0 - torch.mean(res ** 2) / torch.var(yv)),
                                 "max_abs_error": float(torch.max(torch.abs(res)))}}
    if kind == "local":
        flat = local_flat(net)
        out = weight_file("local", folder=folder)
    else:
        flat = bn.flat()
        assert flat.size == 64 * meta["L"] + 117
        out = weight_file("block", meta["L"], folder=folder)
    os.makedirs(folder, exist_ok=True)
    np.save(out, flat)
    with open(out.replace(".npy", ".json"), "w") as f:
        json.dump(report, f, indent=1)
    log("wrote %s: validation rms error %.4g against rms label %.4g (R^2 %.4f)"
        % (out, report["validation"]["rms_error"], report["validation"]["rms_label"], report["validation"]["r2"]))
    return report


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("step", choices=["data", "fit"])
    ap.add_argument("--kind", choices=["local", "block"], default="local")
    ap.add_argument("--out", default=None)
    ap.add_argument("--data", default=None)
    ap.add_argument("--epochs", type=int, default=None)
    ap.add_argument("--device", default="cpu")
    ap.add_argument("--weights-dir", default=WEIGHTS)
    a = ap.parse_args(argv)
    log = lambda m: print(m, flush=True)
    if a.step == "data":
        generate(a.kind, a.out or "train_%s.npz" % a.kind, log=log)
    else:
        fit(a.kind, a.data or "train_%s.npz" % a.kind, epochs=a.epochs, log=log, device=a.device,
            folder=a.weights_dir)


if __name__ == "__main__":
    sys.exit(main())
