"""Network-proposed local moves and the cumulative update (paper: Local
Updates; the p_c equation after Global Updates).

The fully connected network sees the proposed displacement and the fields
around the spacetime point (i, l): nearest and next-nearest neighbours in
space (a 3 x 3 patch) and in imaginary time (slices l-2 .. l+2), 45 inputs
in all.  Input p = 9 (dl + 2) + 3 (dy + 1) + (dx + 1) holds x at slice l+dl,
site (ix+dx, iy+dy), periodic in both, except the centre p = 22, which holds
the displacement d.  Two hidden layers of 64 units (ReLU, or the paper's
softplus), one linear output y: the network's estimate of the fermionic
change of log W, 2 log|r|.  The bosonic change is exact, so a proposal is
accepted inside the sweep iff u < exp(y - dS_b).

After the sweep the whole proposal X' is accepted with p_c:
    log p_c = [log W(X') - log W(X)] - [log W_NN(X') - log W_NN(X)]
            = 2 (log|det M(X')| - log|det M(X)|) - sum of accepted y,
the bosonic terms cancelling.  The determinant is from scratch in FP64.

Visiting order: the paper does not fix one.  Points are visited by colour
classes (l mod 4, iy mod 2, ix mod 2), class after class; two points of one
class are never inside each other's patch (needs Nx even and L % 4 == 0), so
the moves of a class do not interact and their order within it is immaterial.

Parity: the forward pass is pinned against torch.nn.functional on the same
weights, the p_c algebra against log W from scratch
(tests/test_oracle_nn.py).
"""
import math

import numpy as np

from . import philox
from .model import local_action_change
from .udt import green_and_logdet

N_IN, N_HID = 45, 64
N_WEIGHTS = N_HID * N_IN + N_HID + N_HID * N_HID + N_HID + N_HID + 1   # 7169


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


def colour_order(nx, L):
    """(l, i) in visiting order: classes (l mod 4, iy mod 2, ix mod 2), then l, iy, ix."""
    if nx % 2 or L % 4:
        raise ValueError("network sweep needs even Nx and L divisible by 4")
    order = []
    for cl in range(4):
        for py in range(2):
            for px in range(2):
                for l in range(cl, L, 4):
                    for iy in range(py, nx, 2):
                        for ix in range(px, nx, 2):
                            order.append((l, ix + nx * iy))
    return order


class NNChain:
    """A chain driven by network proposals and exact cumulative accepts."""

    def __init__(self, chain, weights_flat, kind=0):
        self.c = chain                   # a dqmc.Chain: params, fields, G, log det, seed
        self.weights = unpack(weights_flat)
        self.kind = kind
        self.inner_accepts = 0
        self.inner_proposals = 0
        self.cumulative_accepts = 0
        self.last_log_pc = 0.0
        self.last_sum_y = 0.0
        self.decisions = []

    def sweep(self):
        c, p = self.c, self.c.p
        L, n = p.L, p.n
        xp = c.x.copy()
        sum_y = 0.0
        for l, i in colour_order(p.nx, L):
            u0, u1 = philox.uniforms(c.seed, c.chain, c.sweep_index, l * n + i, philox.KIND_NN)
            d = p.local_width * (2.0 * u0 - 1.0)
            y = forward(self.weights, patch(p.nx, xp, l, i, d), self.kind)
            ds = local_action_change(p, xp[l, i], xp[(l - 1) % L, i], xp[(l + 1) % L, i], d)
            R = math.exp(min(y - ds, 700.0))
            accept = u1 < R
            self.decisions.append((philox.KIND_NN, c.sweep_index, l * n + i, accept,
                                   math.log(u1) - (y - ds) if u1 > 0 else -math.inf))
            self.inner_proposals += 1
            if accept:
                xp[l, i] += d
                sum_y += y
                self.inner_accepts += 1
        g_new, ld_new = green_and_logdet(p, c.expk, xp, 0)
        log_pc = 2.0 * (ld_new - c.logdet) - sum_y
        uc, _ = philox.uniforms(c.seed, c.chain, c.sweep_index, 0, philox.KIND_CUMULATIVE)
        accept = uc < math.exp(min(log_pc, 700.0))
        self.decisions.append((philox.KIND_CUMULATIVE, c.sweep_index, 0, accept,
                               math.log(uc) - log_pc if uc > 0 else -math.inf))
        self.last_log_pc, self.last_sum_y = log_pc, sum_y
        if accept:
            c.x, c.G, c.logdet = xp, g_new, ld_new
            self.cumulative_accepts += 1
        c.sweep_index += 1
        return accept
