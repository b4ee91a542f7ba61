"""Network-proposed local and block moves and the cumulative update (paper:
Local Updates; Global Updates and the p_c equation after it).

The fully connected network sees the proposed displacement and the fields
around the spacetime point (i, l): nearest and next-nearest neighbours in
space (a 3 x 3 patch) and in imaginary time (slices l-2 .. l+2), 45 inputs
in all.  Input p = 9 (dl + 2) + 3 (dy + 1) + (dx + 1) holds x at slice l+dl,
site (ix+dx, iy+dy), periodic in both, except the centre p = 22, which holds
the displacement d.  Two hidden layers of 64 units (ReLU, or the paper's
softplus), one linear output f.  The estimate of the move's fermionic change
of log W (2 log|r|) is the odd part in d,
    y = (f(patch, d) - f(patch, -d)) / 2,
so that the move back from x + d by -d (the same patch: only the centre
changed) has estimate -y.  The bosonic change is exact, so a proposal is
accepted inside the sweep iff u < exp(y - dS_b).

After the inner sweeps the whole proposal X' is accepted with
    log p_c = 2 (log|det M(X')| - log|det M(X)|) - sum of accepted y,
the determinant from scratch in FP64.  Why this is exact: the inner sweeps
are a path of Metropolis steps X = X_0 -> ... -> X_T = X'.  The same steps in
reverse order, each move undone by its opposite displacement, are a path of
the reversed schedule from X' back to X; a rejected step has the same
probability on both paths, and an accepted one contributes
min(1, e^a) / min(1, e^-a) = e^a, a = y - dS_b, because every estimate is
odd under the reversal (for block moves f(x + D) - f(x) with unchanged
neighbour channels is odd too).  So P(reverse path) / P(path) =
exp(-sum y + S_b(X') - S_b(X)), and the Metropolis-Hastings ratio of the
composite move, W(X') P(reverse) / (W(X) P(path)), is p_c.  For the reversed
schedule to be one the sampler itself may run, every sweep draws its
direction (Philox kind 7, shared by the chains of the sweep): forward, or
every step of the schedule in reverse order, with probability 1/2 each.

Visiting order: the paper does not fix one.  Points are visited by colour
classes (l mod 4, iy mod 2, ix mod 2), class after class; two points of one
class are never inside each other's patch (needs Nx even and L % 4 == 0), so
the moves of a class do not interact and their order within it is immaterial.

Block moves (paper: Global Updates, and the caption of its network figure).
A move shifts the whole column x[:, i] by D.  The convolutional network sees
three channels over the L slices of site i: the column itself and the means
of the four nearest and of the four diagonal next-nearest neighbours'
columns.  The paper fixes four layers, sigmoid hidden units and a linear
output, and leaves the first layer's stride and kernel open; here a circular
convolution along imaginary time (periodic in l) with 4 output channels,
kernel 4 and stride 2 (first hidden layer 4 x L/2 units), a dense layer of 32
units and the output.  Reading of how the move enters: the network is taken
as a site-local effective energy of the column, so its estimate of the
fermionic change of log W is y = f(x_i + D) - f(x_i) with the neighbour
channels unchanged.  Sites are visited by colour classes (iy mod 2, ix mod 2):
a site's inputs come from its 3 x 3 neighbourhood, which holds no other site
of its class.

A full forward sweep: n_u sweeps of network local moves, then n_u sweeps of
network block moves (if the block width is > 0); the reversed sweep takes the
same classes in the opposite order; then one cumulative accept with the sum
of every accepted y.

Parity: both forward passes are pinned against torch.nn.functional on the
same weights, the p_c algebra against log W from scratch, and the cumulative
ratio against the probabilities of the path and of its reverse evaluated
step by step (tests/test_oracle_nn.py).
"""
import math

import numpy as np

from . import philox
from .model import global_action_change, local_action_change
from .udt import green_and_logdet

N_IN, N_HID = 45, 64
N_WEIGHTS = N_HID * N_IN + N_HID + N_HID * N_HID + N_HID + N_HID + 1   # 7169

CNN_C, CNN_K, CNN_S, CNN_H = 4, 4, 2, 32     # conv channels, kernel, stride; dense units


def cnn_count(L):
    """Weights of the block-move network for L slices: 64 L + 117."""
    if L % CNN_S:
        raise ValueError("the block-move network needs L divisible by %d" % CNN_S)
    P = L // CNN_S
    return CNN_C * 3 * CNN_K + CNN_C + CNN_H * CNN_C * P + CNN_H + CNN_H + 1


def unpack_cnn(w, L):
    """Flat FP32 weights -> (Wc[C,3,K], bc[C], Wd[H, C*P], bd[H], Wo[H], bo) as float64.
    The dense layer reads the conv output flattened channel-major, index c * P + p."""
    w = np.asarray(w, dtype=np.float32).astype(np.float64)
    if w.size != cnn_count(L):
        raise ValueError("expected %d weights" % cnn_count(L))
    P = L // CNN_S
    o = 0
    Wc = w[o:o + CNN_C * 3 * CNN_K].reshape(CNN_C, 3, CNN_K); o += CNN_C * 3 * CNN_K
    bc = w[o:o + CNN_C]; o += CNN_C
    Wd = w[o:o + CNN_H * CNN_C * P].reshape(CNN_H, CNN_C * P); o += CNN_H * CNN_C * P
    bd = w[o:o + CNN_H]; o += CNN_H
    Wo = w[o:o + CNN_H]; o += CNN_H
    bo = w[o]
    return Wc, bc, Wd, bd, Wo, bo


def sigmoid(h):
    return 1.0 / (1.0 + np.exp(-h))


def cnn_forward(weights, inp):
    """Block-move network on inputs inp[3, L]: circular convolution along l
    (output position p reads slices S p .. S p + K - 1 mod L), sigmoid, dense
    sigmoid layer, linear output."""
    Wc, bc, Wd, bd, Wo, bo = weights
    L = inp.shape[1]
    P = L // CNN_S
    conv = np.empty((CNN_C, P))
    for c in range(CNN_C):
        for p in range(P):
            s = bc[c]
            for ch in range(3):
                for k in range(CNN_K):
                    s += Wc[c, ch, k] * inp[ch, (CNN_S * p + k) % L]
            conv[c, p] = s
    h1 = sigmoid(conv).reshape(-1)
    h2 = sigmoid(Wd @ h1 + bd)
    return float(Wo @ h2 + bo)


def cnn_inputs(nx, x, i):
    """The three input channels of site i: x[:, i], the mean over its four
    nearest neighbours and over its four diagonal next-nearest neighbours."""
    ix, iy = i % nx, i // nx
    site = lambda dx, dy: (ix + dx) % nx + nx * ((iy + dy) % nx)
    nn = [site(1, 0), site(-1, 0), site(0, 1), site(0, -1)]
    nnn = [site(1, 1), site(1, -1), site(-1, 1), site(-1, -1)]
    return np.stack([x[:, i], x[:, nn].mean(axis=1), x[:, nnn].mean(axis=1)])


def cnn_colour_order(nx):
    """Sites in visiting order: classes (iy mod 2, ix mod 2), then iy, ix."""
    if nx % 2:
        raise ValueError("network block moves need even Nx")
    return [ix + nx * iy for py in range(2) for px in range(2)
            for iy in range(py, nx, 2) for ix in range(px, nx, 2)]


def unpack(w):
    """Flat FP32 weights -> (W1[64,45], b1, W2[64,64], b2, W3[64], b3) as float64."""
    w = np.asarray(w, dtype=np.float32).astype(np.float64)
    if w.size != N_WEIGHTS:
        raise ValueError("expected %d weights" % N_WEIGHTS)
    o = 0
    W1 = w[o:o + N_HID * N_IN].reshape(N_HID, N_IN); o += N_HID * N_IN
    b1 = w[o:o + N_HID]; o += N_HID
    W2 = w[o:o + N_HID * N_HID].reshape(N_HID, N_HID); o += N_HID * N_HID
    b2 = w[o:o + N_HID]; o += N_HID
    W3 = w[o:o + N_HID]; o += N_HID
    b3 = w[o]
    return W1, b1, W2, b2, W3, b3


def activation(h, kind):
    if kind == 0:
        return np.maximum(h, 0.0)
    return np.logaddexp(0.0, h)          # softplus ln(1 + e^h)


def forward(weights, inp, kind=0):
    W1, b1, W2, b2, W3, b3 = weights
    h1 = activation(W1 @ inp + b1, kind)
    h2 = activation(W2 @ h1 + b2, kind)
    return float(W3 @ h2 + b3)


def patch(nx, x, l, i, d):
    """The 45 network inputs for a move of x[l, i] by d."""
    L = x.shape[0]
    ix, iy = i % nx, i // nx
    out = np.empty(N_IN)
    for dl in range(-2, 3):
        for dy in range(-1, 2):
            for dx in range(-1, 2):
                k = 9 * (dl + 2) + 3 * (dy + 1) + (dx + 1)
                j = (ix + dx) % nx + nx * ((iy + dy) % nx)
                out[k] = x[(l + dl) % L, j]
    out[22] = d
    return out


def local_classes(nx, L):
    """The 16 colour classes (l mod 4, iy mod 2, ix mod 2) of local moves, in
    forward order, each a list of (l, i)."""
    if nx % 2 or L % 4:
        raise ValueError("network sweep needs even Nx and L divisible by 4")
    out = []
    for cl in range(4):
        for py in range(2):
            for px in range(2):
                out.append([(l, ix + nx * iy) for l in range(cl, L, 4)
                            for iy in range(py, nx, 2) for ix in range(px, nx, 2)])
    return out


def colour_order(nx, L):
    """(l, i) in forward visiting order."""
    return [pt for cls in local_classes(nx, L) for pt in cls]


def block_classes(nx):
    """The 4 colour classes (iy mod 2, ix mod 2) of block moves, in forward order."""
    order = cnn_colour_order(nx)
    k = len(order) // 4
    return [order[j * k:(j + 1) * k] for j in range(4)]


def local_estimate(weights, nx, x, l, i, d, kind=0):
    """The network's estimate of the fermionic change of log W for x[l, i] += d:
    the odd part (f(d) - f(-d)) / 2 of the network output."""
    return 0.5 * (forward(weights, patch(nx, x, l, i, d), kind) - forward(weights, patch(nx, x, l, i, -d), kind))


def block_estimate(cnn, nx, x, i, d):
    """f(x_i + d) - f(x_i), the neighbour channels unchanged."""
    inp = cnn_inputs(nx, x, i)
    moved = inp.copy()
    moved[0] += d
    return cnn_forward(cnn, moved) - cnn_forward(cnn, inp)


def scan_reversed(seed, sweep):
    """Whether sweep `sweep` visits the schedule in reverse (Philox kind 7)."""
    u0, _ = philox.uniforms(seed, 0, sweep, 0, philox.KIND_SCAN)
    return u0 >= 0.5


class NNChain:
    """A chain driven by network proposals and exact cumulative accepts.
    cnn: flat block-move network weights (used when the chain's block width
    is > 0); nu: sweeps of each kind per cumulative accept.  After a sweep,
    `path` holds its steps in the order taken: (kind, u, points, x before the
    step) with points = [(l or None, i, d, accepted, y, dS_b)]."""

    def __init__(self, chain, weights_flat, kind=0, cnn=None, nu=1):
        self.c = chain                   # a dqmc.Chain: params, fields, G, log det, seed
        self.weights = unpack(weights_flat)
        self.kind = kind
        self.nu = nu
        self.cnn = unpack_cnn(cnn, chain.p.L) if cnn is not None else None
        self.inner_accepts = 0
        self.inner_proposals = 0
        self.block_accepts = 0
        self.block_proposals = 0
        self.cumulative_accepts = 0
        self.last_log_pc = 0.0
        self.last_sum_y = 0.0
        self.last_reversed = False
        self.decisions = []
        self.path = []

    def schedule(self):
        """The steps of one forward sweep: ("local", u, class) then ("block", u, class)."""
        p = self.c.p
        steps = [("local", u, cls) for u in range(self.nu) for cls in local_classes(p.nx, p.L)]
        if self.cnn is not None and p.global_width > 0:
            steps += [("block", u, cls) for u in range(self.nu) for cls in block_classes(p.nx)]
        return steps

    def _local_step(self, xp, u, cls):
        c, p = self.c, self.c.p
        L, n = p.L, p.n
        pts, y_acc = [], 0.0
        for l, i in cls:
            slot = u * L * n + l * n + i
            u0, u1 = philox.uniforms(c.seed, c.chain, c.sweep_index, slot, philox.KIND_NN)
            d = p.local_width * (2.0 * u0 - 1.0)
            y = local_estimate(self.weights, p.nx, xp, l, i, d, self.kind)
            ds = local_action_change(p, xp[l, i], xp[(l - 1) % L, i], xp[(l + 1) % L, i], d)
            R = math.exp(min(y - ds, 700.0))
            accept = u1 < R
            self.decisions.append((philox.KIND_NN, c.sweep_index, slot, accept,
                                   math.log(u1) - (y - ds) if u1 > 0 else -math.inf))
            self.inner_proposals += 1
            pts.append((l, i, d, accept, y, ds))
            if accept:
                y_acc += y
                self.inner_accepts += 1
        for l, i, d, accept, _, _ in pts:          # the points of a class do not interact
            if accept:
                xp[l, i] += d
        return pts, y_acc

    def _block_step(self, xp, u, cls):
        c, p = self.c, self.c.p
        L, n = p.L, p.n
        pts, y_acc = [], 0.0
        for i in cls:
            slot = u * n + i
            u0, u1 = philox.uniforms(c.seed, c.chain, c.sweep_index, slot, philox.KIND_NN_GLOBAL)
            d = p.global_width * (2.0 * u0 - 1.0)
            y = block_estimate(self.cnn, p.nx, xp, i, d)
            ds = global_action_change(p, float(np.sum(xp[:, i])), d, L)
            R = math.exp(min(y - ds, 700.0))
            accept = u1 < R
            self.decisions.append((philox.KIND_NN_GLOBAL, c.sweep_index, slot, accept,
                                   math.log(u1) - (y - ds) if u1 > 0 else -math.inf))
            self.block_proposals += 1
            pts.append((None, i, d, accept, y, ds))
            if accept:
                y_acc += y
                self.block_accepts += 1
        for _, i, d, accept, _, _ in pts:
            if accept:
                xp[:, i] += d
        return pts, y_acc

    def sweep(self):
        c, p = self.c, self.c.p
        xp = c.x.copy()
        sum_y = 0.0
        steps = self.schedule()
        rev = scan_reversed(c.seed, c.sweep_index)
        if rev:
            steps = steps[::-1]
        self.path = []
        for kind, u, cls in steps:
            before = xp.copy()
            if kind == "local":
                pts, y_acc = self._local_step(xp, u, cls)
            else:
                pts, y_acc = self._block_step(xp, u, cls)
            sum_y += y_acc
            self.path.append((kind, u, pts, before))
        g_new, ld_new = green_and_logdet(p, c.expk, xp, 0)
        log_pc = 2.0 * (ld_new - c.logdet) - sum_y
        uc, _ = philox.uniforms(c.seed, c.chain, c.sweep_index, 0, philox.KIND_CUMULATIVE)
        accept = uc < math.exp(min(log_pc, 700.0))
        self.decisions.append((philox.KIND_CUMULATIVE, c.sweep_index, 0, accept,
                               math.log(uc) - log_pc if uc > 0 else -math.inf))
        self.last_log_pc, self.last_sum_y, self.last_reversed = log_pc, sum_y, rev
        self.proposal = xp
        if accept:
            c.x, c.G, c.logdet = xp, g_new, ld_new
            self.cumulative_accepts += 1
        c.sweep_index += 1
        return accept
