"""Parity of the HIP path (through the C ABI) with the oracle, element by
element on the same seeded inputs.

Bars (the design notes derive them):
  * fields: bit-identical (both sides add the same exactly drawn displacement
    whenever they take the same decision);
  * decisions: identical (FP64); in mixed precision and for the FP32 network,
    identical outside a tie band |ln u - ln R| <= band where the GPU replays
    the oracle's decision, with zero disagreements outside the band;
  * G: max|dG| <= 1e-10 max|G| (FP64), <= 1e-5 max|G| (mixed: G is stored in FP32);
  * log|det M|: |d| <= 1e-10 max(1, |logdet|).
"""
import math
import sys

import numpy as np
import pytest

from oracle import dqmc, nnmc, philox
from oracle.model import Params
import workloads

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOL_MIXED = 1e-5
BAND_MIXED = 1e-4


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def hq():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1905_07440_amd import hq as mod
    mod.load()
    return mod


def params_of(gr, g=None):
    return Params(nx=gr["nx"], t=gr.get("t", 1.0), mu=gr.get("mu", 0.0), mass=gr.get("mass", 1.0),
                  omega=gr.get("omega", 1.0), g=gr.get("g", 1.0) if g is None else g,
                  beta=gr["beta"], dtau=gr.get("dtau", 0.1), n_stab=gr["n_stab"],
                  local_width=gr.get("local_width", 0.5), global_width=gr.get("global_width", 0.0))


def make_ctx(hq, groups, precision=0, seed=1, delay=0, record=True, activation=0):
    hg = [hq.make_group(gr["nx"], gr["chains"], t=gr.get("t", 1.0), mu=gr.get("mu", 0.0),
                        mass=gr.get("mass", 1.0), omega=gr.get("omega", 1.0), g=gr.get("g", 1.0),
                        g_range=gr.get("g_range"), beta=gr["beta"], dtau=gr.get("dtau", 0.1),
                        n_stab=gr["n_stab"], proposal=gr.get("proposal", 0),
                        local_width=gr.get("local_width", 0.5), global_width=gr.get("global_width", 0.0),
                        nn_sweeps=gr.get("nn_sweeps", 1))
          for gr in groups]
    return hq.Context(hg, precision=precision, seed=seed, delay=delay, record=record, activation=activation)


def rel_g(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def assert_state(ctx, c, ch, tol_g, tag):
    x = ctx.fields(c)
    G = ctx.green(c)
    st = ctx.stats(c)
    assert np.array_equal(x, ch.x), "%s: fields differ (max %g)" % (tag, np.max(np.abs(x - ch.x)))
    rg = rel_g(G, ch.G)
    assert rg <= tol_g, "%s: G rel diff %g" % (tag, rg)
    dl = abs(st["logdet"] - ch.logdet)
    assert dl <= TOL64 * max(1.0, abs(ch.logdet)), "%s: logdet diff %g" % (tag, dl)
    assert st["local_accepts"] == ch.local_accepts, tag
    assert st["global_accepts"] == ch.global_accepts, tag
    return st


def oracle_local_bits(ch, sweep):
    n_slots = ch.p.L * ch.p.n
    bits = np.zeros(n_slots, dtype=np.uint8)
    for d in ch.decisions:
        if d.kind == philox.KIND_LOCAL and d.sweep == sweep:
            bits[d.slot] = 1 if d.accept else 0
    return bits


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("nx,beta,ns,prec", [(2, 1.0, 5, 0), (4, 4.0, 10, 0), (8, 8.0, 8, 0),
                                             (10, 2.0, 10, 0), (12, 2.0, 10, 1), (6, 0.2, 1, 0),
                                             (4, 1.0, 10, 0)])
def test_initial_state(hq, nx, beta, ns, prec):
    """Fields, G and log det at creation against the oracle; the last case has
    one block per chain (L = n_stab) with two chains."""
    say("initial state nx=%d beta=%g ns=%d prec=%d" % (nx, beta, ns, prec))
    gr = dict(nx=nx, chains=2, g=1.1, beta=beta, n_stab=ns)
    ctx = make_ctx(hq, [gr], precision=prec, seed=7)
    for c in range(2):
        ch = dqmc.Chain(params_of(gr), 7, c)
        assert np.array_equal(ctx.fields(c), ch.x)
        assert rel_g(ctx.green(c), ch.G) <= (TOL_MIXED if prec else TOL64)
        assert abs(ctx.stats(c)["logdet"] - ch.logdet) <= TOL64 * max(1, abs(ch.logdet))
    ctx.close()


def test_holstein_4x4_all_sweeps(hq):
    """The whole 4x4 single-chain workload: 20 FP64 sweeps, every decision compared."""
    w = workloads.holstein_4x4_single()
    g = w.groups[0]
    say("4x4 single chain, %d sweeps" % w.sweeps)
    gr = dict(nx=g.nx, chains=1, g=g.g, beta=g.beta, n_stab=g.n_stab)
    ctx = make_ctx(hq, [gr], seed=w.seed)
    ch = dqmc.Chain(params_of(gr), w.seed, 0)
    for s in range(w.sweeps):
        ctx.sweep(1)
        ch.sweep()
        acc, margin = ctx.decisions(0, hq.KIND_LOCAL)
        assert np.array_equal(acc, oracle_local_bits(ch, s)), "sweep %d" % s
    st = assert_state(ctx, 0, ch, TOL64, "4x4")
    assert st["max_drift_green"] < 1e-10
    ctx.close()


@pytest.mark.parametrize("delay", [8, 16, 32])
def test_delay_depths_agree_with_oracle(hq, delay):
    say("8x8 delay=%d" % delay)
    gr = dict(nx=8, chains=2, g=1.2, beta=2.0, n_stab=4)
    ctx = make_ctx(hq, [gr], seed=11, delay=delay)
    ctx.sweep(2)
    for c in range(2):
        ch = dqmc.Chain(params_of(gr), 11, c)
        ch.sweep(); ch.sweep()
        assert_state(ctx, c, ch, TOL64, "delay %d chain %d" % (delay, c))
    ctx.close()


def test_block_moves_8x8(hq):
    """8x8 chains with one block move per site per sweep (the batched FP64 workload's moves)."""
    say("8x8 block moves")
    gr = dict(nx=8, chains=3, g=1.2, beta=1.6, n_stab=8, global_width=1.0)
    ctx = make_ctx(hq, [gr], seed=2)
    ctx.sweep(2)
    for c in range(3):
        ch = dqmc.Chain(params_of(gr), 2, c)
        ch.sweep(); ch.sweep()
        st = assert_state(ctx, c, ch, TOL64, "block chain %d" % c)
        acc, _ = ctx.decisions(c, hq.KIND_GLOBAL)
        obits = [d.accept for d in ch.decisions if d.kind == philox.KIND_GLOBAL and d.sweep == 1]
        assert list(acc.astype(bool)) == obits
        assert st["global_proposals"] == 2 * 64
    ctx.close()


def test_batched_8x8_full_size_sampled(hq):
    """64 chains of 8x8, L = 80, n_stab = 8 with block moves (full size); chains 0 and 63 vs the oracle."""
    w = workloads.holstein_8x8_batched_global()
    g = w.groups[0]
    say("8x8 x64 full size, one sweep")
    gr = dict(nx=g.nx, chains=g.n_chains, g=g.g, beta=g.beta, n_stab=g.n_stab, global_width=g.global_width)
    ctx = make_ctx(hq, [gr], seed=w.seed)
    ctx.sweep(1)
    for c in (0, 63):
        ch = dqmc.Chain(params_of(gr), w.seed, c)
        ch.sweep()
        assert_state(ctx, c, ch, TOL64, "8x8 chain %d" % c)
    ctx.close()


def _mixed_replay_case(hq, gr, chains_to_check, seed, sweeps=1, setup=None, delay=32, drift_gate=False):
    """Mixed-precision sweeps beside the oracle, the oracle's decisions replayed
    inside the tie band.  After each sweep: fields bit-identical, G and log det
    after the FP64 recompute, and the FP32-tracked G just before that recompute
    against the oracle's tracked G (1e-5 relative when drift_gate is set: the
    recompute interval then keeps the FP32 drift within the gate, which is
    also asserted)."""
    ctx = make_ctx(hq, [gr], precision=1, seed=seed, delay=delay)
    if setup is not None:
        setup(ctx)
    oracles = {c: dqmc.Chain(params_of(gr), seed, c) for c in chains_to_check}
    for s in range(sweeps):
        for c, ch in oracles.items():
            ch.sweep()
            ctx.set_replay(c, hq.KIND_LOCAL, oracle_local_bits(ch, s), BAND_MIXED)
        ctx.sweep(1)
        for c, ch in oracles.items():
            st = ctx.stats(c)
            assert st["replay_mismatches"] == 0, "chain %d: decision outside the tie band differs" % c
            assert np.array_equal(ctx.fields(c), ch.x), "sweep %d chain %d" % (s, c)
            assert rel_g(ctx.green(c), ch.G) <= TOL_MIXED
            assert abs(st["logdet"] - ch.logdet) <= TOL64 * max(1.0, abs(ch.logdet))
            assert st["local_accepts"] == ch.local_accepts
            gt, ldt = ctx.green_tracked(c)
            rt = rel_g(gt, ch.G_tracked)
            if drift_gate:
                assert st["max_drift_green"] <= TOL_MIXED, "chain %d: drift %g" % (c, st["max_drift_green"])
                assert rt <= TOL_MIXED, "sweep %d chain %d: tracked G rel %g" % (s, c, rt)
                assert abs(ldt - ch.logdet_tracked) <= TOL_MIXED * max(1.0, abs(ch.logdet_tracked))
            say("  sweep %d chain %d: overrides in band %d, max drift %.2e, tracked G rel %.2e"
                % (s, c, st["replay_overrides"], st["max_drift_green"], rt))
    ctx.close()


def test_mixed_one_block(hq):
    """Mixed precision with one block per chain (L = n_stab) and two chains:
    the recompute at the end of the only block, upward and downward."""
    say("mixed 6x6, L = n_stab")
    _mixed_replay_case(hq, dict(nx=6, chains=2, g=1.2, beta=1.0, n_stab=10), (0, 1), seed=21, sweeps=2, delay=16)


def test_mixed_delay8_streamed(hq):
    """Mixed precision with blocks of 8 sites (the streamed local form: the
    register form takes blocks of 16 and 32 only), two chains, both sweep
    directions."""
    say("mixed 8x8, delay 8")
    _mixed_replay_case(hq, dict(nx=8, chains=2, g=1.3, beta=1.2, n_stab=6), (0, 1), seed=23, sweeps=2, delay=8,
                       drift_gate=True)


def test_mixed_12x12_small(hq):
    say("12x12 mixed, beta=2")
    _mixed_replay_case(hq, dict(nx=12, chains=2, g=1.5, beta=2.0, n_stab=10), (0, 1), seed=3, sweeps=2)


@pytest.mark.parametrize("nx", [13, 15, 16])
def test_large_lattice_fp64(hq, nx):
    """N = 169 and 225 (panels with a ragged last one) and 256 in FP64, two
    chains: the streamed local form and the factorizations spread over
    several workgroups per matrix."""
    say("FP64 %dx%d" % (nx, nx))
    gr = dict(nx=nx, chains=2, g=1.1, beta=0.4, n_stab=2)
    ctx = make_ctx(hq, [gr], seed=12)
    ctx.sweep(2)
    for c in range(2):
        ch = dqmc.Chain(params_of(gr), 12, c)
        ch.sweep(); ch.sweep()
        assert_state(ctx, c, ch, TOL64, "%dx%d chain %d" % (nx, nx, c))
    ctx.close()


@pytest.mark.parametrize("nx", [13, 15])
def test_from_scratch_blocked_ragged(hq, nx):
    """From-scratch G and log det with 80 matrices at the first level of the
    pairwise UDT tree (8 chains x 10 blocks; the tree is what block-move
    proposals are scored with), so that level takes the QR with one
    workgroup per matrix through L2 and Q in a launch of its own, at N = 169
    and 225 (ragged last panel; the later levels spread over several
    workgroups per matrix).  At creation and after a recompute (an oracle
    sweep with block moves at this size takes minutes)."""
    say("from scratch, blocked QR, %dx%d" % (nx, nx))
    gr = dict(nx=nx, chains=8, g=1.1, beta=2.0, n_stab=2, global_width=0.5)
    ctx = make_ctx(hq, [gr], seed=31)
    chains = {c: dqmc.Chain(params_of(gr), 31, c) for c in (0, 7)}
    for c, ch in chains.items():
        assert_state(ctx, c, ch, TOL64, "%dx%d chain %d at creation" % (nx, nx, c))
    ctx.recompute()
    for c, ch in chains.items():
        assert_state(ctx, c, ch, TOL64, "%dx%d chain %d recomputed" % (nx, nx, c))
    ctx.close()


@pytest.mark.parametrize("ns", [9, 10])
def test_block_product_chunks_16x16(hq, ns):
    """N = 256 with n_stab slices per block above the 8 row-scale sets that
    one Kronecker chain launch holds: block products in two chunks (8 + 1,
    8 + 2) through the scratch buffer."""
    say("FP64 16x16 n_stab=%d" % ns)
    gr = dict(nx=16, chains=2, g=1.1, beta=0.1 * 2 * ns, n_stab=ns)
    ctx = make_ctx(hq, [gr], seed=19)
    ctx.sweep(2)
    for c in range(2):
        ch = dqmc.Chain(params_of(gr), 19, c)
        ch.sweep(); ch.sweep()
        assert_state(ctx, c, ch, TOL64, "16x16 n_stab=%d chain %d" % (ns, c))
    ctx.close()


@pytest.mark.parametrize("delay", [16, 32])
def test_mixed_16x16(hq, delay):
    """N = 256 in mixed precision, an upward and a downward sweep: at delay 16
    G lives in the accumulators of four waves (64 tiles each, the register
    form the 16x16 chains of the uneven batch take); at delay 32 it is
    streamed from global memory."""
    say("16x16 mixed, delay %d" % delay)
    _mixed_replay_case(hq, dict(nx=16, chains=2, g=1.2, beta=0.4, n_stab=2), (0, 1), seed=8, sweeps=2, delay=delay,
                       drift_gate=True)


@pytest.mark.parametrize("nx,delay", [(12, 16), (12, 32), (10, 16), (7, 16), (5, 32)])
def test_mixed_register_forms(hq, nx, delay):
    """The register-resident local-move kernel in FP32 for each tile-grid
    class (N = 25, 49, 144) and block size, an upward and a downward sweep,
    with the drift gate at a short recompute interval."""
    say("mixed register form nx=%d delay=%d" % (nx, delay))
    _mixed_replay_case(hq, dict(nx=nx, chains=2, g=1.5, beta=1.2, n_stab=6), (0, 1), seed=31, sweeps=2,
                       delay=delay, drift_gate=True)


@pytest.mark.parametrize("delay", [16, 32])
def test_fp64_12x12_register_form(hq, delay):
    """FP64 at N = 144 (the FP64 baseline's lattice): the register form at
    delay 16, the streamed form at delay 32 (its LDS panels do not fit)."""
    say("FP64 12x12 delay %d" % delay)
    gr = dict(nx=12, chains=2, g=1.5, beta=1.0, n_stab=5)
    ctx = make_ctx(hq, [gr], seed=33, delay=delay)
    ctx.sweep(2)
    for c in range(2):
        ch = dqmc.Chain(params_of(gr), 33, c)
        ch.sweep(); ch.sweep()
        assert_state(ctx, c, ch, TOL64, "12x12 FP64 delay %d chain %d" % (delay, c))
    ctx.close()


def golden(name):
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)
    with np.load(path) as z:
        return {k: z[k] for k in z.files}


def test_mixed_12x12_gate_full_size_golden(hq):
    """Exactly the benchmarked configuration: 128 chains of 12x12, L = 120,
    mixed precision, recompute every 6 slices, delay 16 (the register form
    local_regs_kernel<float, 16, 9>).  Chains 0 and 127 over one upward and
    one downward sweep against the oracle's stored results
    (tests/golden/make_golden.py): decisions replayed inside the tie band,
    fields bit-identical, G and log det after the recompute, and the
    FP32-tracked G and log det just before it, all within 1e-5."""
    w = workloads.ALL["c3-gate"]()
    g = w.groups[0]
    say("12x12 x128 mixed n_stab=6 delay 16, two sweeps against golden data")
    gr = dict(nx=g.nx, chains=g.n_chains, g=g.g, beta=g.beta, n_stab=g.n_stab)
    ref = {c: golden("c3gate_chain%d.npz" % c) for c in (0, 127)}
    ctx = make_ctx(hq, [gr], precision=1, seed=w.seed, delay=16)
    n_slots = g.nx ** 2 * round(g.beta / g.dtau)
    for s in range(2):
        for c, z in ref.items():
            ctx.set_replay(c, hq.KIND_LOCAL, np.unpackbits(z["bits%d" % s])[:n_slots], BAND_MIXED)
        ctx.sweep(1)
        for c, z in ref.items():
            st = ctx.stats(c)
            tag = "sweep %d chain %d" % (s, c)
            assert st["replay_mismatches"] == 0, tag
            assert st["local_accepts"] == int(z["accepts%d" % s]), tag
            assert np.array_equal(ctx.fields(c), z["x%d" % s]), tag
            Gref = z["G%d" % s].astype(np.float64)
            assert rel_g(ctx.green(c), Gref) <= TOL_MIXED, tag
            ld = float(z["logdet%d" % s])
            assert abs(st["logdet"] - ld) <= TOL64 * max(1.0, abs(ld)), tag
            gt, ldt = ctx.green_tracked(c)
            rt = rel_g(gt, z["Gtr%d" % s].astype(np.float64))
            assert rt <= TOL_MIXED, "%s: tracked G rel %g" % (tag, rt)
            ldr = float(z["logdet_tr%d" % s])
            assert abs(ldt - ldr) <= TOL_MIXED * max(1.0, abs(ldr)), tag
            assert st["max_drift_green"] <= TOL_MIXED, tag
            say("  %s: overrides %d, tracked G rel %.2e, drift %.2e" % (tag, st["replay_overrides"], rt,
                                                                       st["max_drift_green"]))
    ctx.close()


def test_mixed_12x12_full_size_sampled(hq):
    """128 chains of 12x12, L = 120 (the mixed workload at full size); chains 0 and 127 vs the oracle."""
    w = workloads.holstein_12x12_mixed()
    g = w.groups[0]
    say("12x12 x128 mixed full size")
    _mixed_replay_case(hq, dict(nx=g.nx, chains=g.n_chains, g=g.g, beta=g.beta, n_stab=g.n_stab),
                       (0, 127), seed=w.seed)


_TILE_CASE = dict(nx=10, chains=2, g=1.3, beta=2.0, n_stab=5)
_tile_oracle = {}


@pytest.mark.parametrize("tile", range(14))
def test_every_gemm_tile_fp64(hq, tile):
    """Each GEMM tile pinned in turn (N = 100: whole tiles plus a ragged edge
    for the 32, 48 and 64 tiles), an upward and a downward sweep in FP64."""
    say("FP64 sweeps with GEMM tile %s" % hq.tile_name(tile))
    gr = _TILE_CASE
    ctx = make_ctx(hq, [gr], seed=13)
    ctx.set_tuning(0, tile)
    assert ctx.tuning(0)["gemm_tile_fp64"] == hq.tile_name(tile)
    ctx.sweep(2)
    if not _tile_oracle:
        for c in range(2):
            ch = dqmc.Chain(params_of(gr), 13, c)
            ch.sweep(); ch.sweep()
            _tile_oracle[c] = ch
    for c in range(2):
        assert_state(ctx, c, _tile_oracle[c], TOL64, "tile %d chain %d" % (tile, c))
    ctx.close()


@pytest.mark.parametrize("tile", range(14))
def test_every_gemm_tile_mixed_wraps(hq, tile):
    """Each tile pinned for the FP32 wraps of a mixed-precision sweep."""
    say("mixed sweep with FP32 GEMM tile %s" % hq.tile_name(tile))
    _mixed_replay_case(hq, dict(_TILE_CASE, n_stab=4), (0,), seed=13,
                       sweeps=2, setup=lambda ctx: ctx.set_tuning(0, 0, tile))


@pytest.mark.parametrize("nx", [3, 8, 10, 12])
def test_fused_wrap_fp64(hq, nx):
    """Both wrap products in one launch (one instantiation per lattice-size
    class, ragged N = 9 and 100 included), an upward and a downward sweep;
    L = 9 and n_stab = 3 put the stabilisation points and the end of the sweep
    after odd numbers of wraps, where G sits in the other buffer."""
    say("FP64 fused wrap nx=%d" % nx)
    gr = dict(nx=nx, chains=2, g=1.2, beta=0.9, n_stab=3)
    ctx = make_ctx(hq, [gr], seed=15)
    ctx.set_tuning(0, 0, 0, wrap="fused")
    assert ctx.tuning(0)["wrap"] == "fused"
    ctx.sweep(2)
    for c in range(2):
        ch = dqmc.Chain(params_of(gr), 15, c)
        ch.sweep(); ch.sweep()
        assert_state(ctx, c, ch, TOL64, "fused wrap nx=%d chain %d" % (nx, c))
    ctx.close()


@pytest.mark.parametrize("nx", [5, 12])
def test_fused_wrap_mixed(hq, nx):
    say("mixed fused wrap nx=%d" % nx)
    _mixed_replay_case(hq, dict(nx=nx, chains=2, g=1.3, beta=0.9, n_stab=3), (0, 1), seed=16, sweeps=2,
                       setup=lambda ctx: ctx.set_tuning(0, 0, 0, wrap="fused"))


@pytest.mark.parametrize("nx", [2, 3, 5, 8, 12, 16])
def test_kron_wrap_fp64(hq, nx):
    """Wraps as Kronecker passes (each padded factor size 4, 8, 12, 16; strips
    of 16 that are ragged for N = 4, 9, 25), an upward and a downward sweep.
    Block products take the Kronecker form in every test."""
    say("FP64 Kronecker wrap nx=%d" % nx)
    gr = dict(nx=nx, chains=2, g=1.2, beta=0.9, n_stab=3)
    ctx = make_ctx(hq, [gr], seed=17)
    ctx.set_tuning(0, 0, 0, wrap="kron")
    assert ctx.tuning(0)["wrap"] == "kron"
    ctx.sweep(2)
    for c in range(2):
        ch = dqmc.Chain(params_of(gr), 17, c)
        ch.sweep(); ch.sweep()
        assert_state(ctx, c, ch, TOL64, "kron wrap nx=%d chain %d" % (nx, c))
    ctx.close()


@pytest.mark.parametrize("nx", [5, 12, 16])
def test_kron_wrap_mixed(hq, nx):
    say("mixed Kronecker wrap nx=%d" % nx)
    _mixed_replay_case(hq, dict(nx=nx, chains=2, g=1.3, beta=0.9, n_stab=3), (0, 1), seed=18, sweeps=2,
                       setup=lambda ctx: ctx.set_tuning(0, 0, 0, wrap="kron"))


@pytest.mark.parametrize("nx", [2, 3, 7, 10])
def test_kron_lds_wrap_fp64(hq, nx):
    """The four Kronecker passes in one launch with G in LDS (ragged 16-wide
    tiles for N = 4, 9, 49, 100); L = 9 with n_stab = 3 leaves G in the other
    buffer at stabilisation points and at the end of the sweep."""
    say("FP64 LDS Kronecker wrap nx=%d" % nx)
    gr = dict(nx=nx, chains=2, g=1.2, beta=0.9, n_stab=3)
    ctx = make_ctx(hq, [gr], seed=20)
    ctx.set_tuning(0, 0, 0, wrap="kron_lds")
    assert ctx.tuning(0)["wrap"] == "kron_lds"
    ctx.sweep(2)
    for c in range(2):
        ch = dqmc.Chain(params_of(gr), 20, c)
        ch.sweep(); ch.sweep()
        assert_state(ctx, c, ch, TOL64, "kron_lds wrap nx=%d chain %d" % (nx, c))
    ctx.close()


@pytest.mark.parametrize("nx", [5, 11, 12])
def test_kron_lds_wrap_mixed(hq, nx):
    say("mixed LDS Kronecker wrap nx=%d" % nx)
    _mixed_replay_case(hq, dict(nx=nx, chains=2, g=1.3, beta=0.9, n_stab=3), (0, 1), seed=21, sweeps=2,
                       setup=lambda ctx: ctx.set_tuning(0, 0, 0, wrap="kron_lds"))


def test_set_tuning_rejects_bad_tiles(hq):
    say("set_tuning errors")
    ctx = make_ctx(hq, [dict(nx=16, chains=1, beta=0.4, n_stab=2)])
    with pytest.raises(hq.HQError):
        ctx.set_tuning(0, hq.N_GEMM_TILES)
    with pytest.raises(hq.HQError):
        ctx.set_tuning(0, 0, 1)                 # FP64 wraps must use the FP64 tile
    with pytest.raises(hq.HQError):
        ctx.set_tuning(0, 10)                   # 32x32 prefetch holds K <= 160; here K = 256
    with pytest.raises(hq.HQError):
        ctx.set_tuning(1, 0)
    with pytest.raises(hq.HQError):
        ctx.set_tuning(0, 0, 0, wrap="fused")   # N = 256: no fused wrap
    with pytest.raises(hq.HQError):
        ctx.set_tuning(0, 0, 0, wrap="kron_lds")   # N = 256: G does not fit in LDS
    assert ctx._lib.hq_set_tuning(ctx._ctx, 0, 0, 0, 4) != 0   # no such wrap kind
    ctx.sweep(1)
    assert ctx.stats(0)["local_proposals"] == 256 * 4
    ctx.close()


def test_uneven_batch_full_size_sampled(hq):
    """The uneven batch at full size (6x6, 8x8, 10x10, 16x16 x 32 chains, L = 100,
    mixed, g per chain): the first chain of each of the three smaller lattices
    swept beside the oracle with the tie band replayed; the 16x16 lattice (an
    oracle sweep there takes most of a minute) through its initial state and,
    after the sweep, the oracle's from-scratch log|det| of the GPU's own
    fields, the recompute of G from those fields and the drift gate."""
    from oracle.model import chain_coupling
    from oracle.udt import green_and_logdet
    w = workloads.holstein_uneven_batch()
    say("uneven batch full size, one sweep")
    groups = [dict(nx=g.nx, chains=g.n_chains, beta=g.beta, n_stab=g.n_stab, g_range=g.g_range) for g in w.groups]
    ctx = make_ctx(hq, groups, precision=1, seed=w.seed, delay=w.delay)
    oracles = {}
    for k, gr in enumerate(groups[:3]):
        c = 32 * k
        oracles[c] = dqmc.Chain(params_of(gr, g=chain_coupling(w.seed, c, 0.8, 1.6)), w.seed, c)
    c16 = 96
    p16 = params_of(groups[3], g=chain_coupling(w.seed, c16, 0.8, 1.6))
    ch16 = dqmc.Chain(p16, w.seed, c16)
    assert np.array_equal(ctx.fields(c16), ch16.x)
    assert rel_g(ctx.green(c16), ch16.G) <= TOL_MIXED
    assert abs(ctx.stats(c16)["logdet"] - ch16.logdet) <= TOL64 * max(1.0, abs(ch16.logdet))
    for c, ch in oracles.items():
        ch.sweep()
        ctx.set_replay(c, hq.KIND_LOCAL, oracle_local_bits(ch, 0), BAND_MIXED)
    z = golden("c4n16_chain%d.npz" % c16)
    assert float(z["g"]) == p16.g
    ctx.set_replay(c16, hq.KIND_LOCAL, np.unpackbits(z["bits0"])[:p16.n * p16.L], BAND_MIXED)
    ctx.sweep(1)
    for c, ch in oracles.items():
        st = ctx.stats(c)
        assert st["replay_mismatches"] == 0, "chain %d" % c
        assert np.array_equal(ctx.fields(c), ch.x), "chain %d" % c
        assert rel_g(ctx.green(c), ch.G) <= TOL_MIXED, "chain %d" % c
        assert abs(st["logdet"] - ch.logdet) <= TOL64 * max(1.0, abs(ch.logdet)), "chain %d" % c
        assert st["local_accepts"] == ch.local_accepts, "chain %d" % c
    # the first 16x16 chain against the oracle's stored sweep
    st = ctx.stats(c16)
    assert st["replay_mismatches"] == 0
    assert st["local_accepts"] == int(z["accepts0"])
    assert np.array_equal(ctx.fields(c16), z["x0"])
    assert rel_g(ctx.green(c16), z["G0"].astype(np.float64)) <= TOL_MIXED
    assert abs(st["logdet"] - float(z["logdet0"])) <= TOL64 * max(1.0, abs(float(z["logdet0"])))
    gt, _ = ctx.green_tracked(c16)
    say("  16x16 chain: tracked G rel %.2e, drift %.2e" % (rel_g(gt, z["Gtr0"].astype(np.float64)),
                                                           st["max_drift_green"]))
    assert rel_g(gt, z["Gtr0"].astype(np.float64)) <= TOL_MIXED
    st = ctx.stats(c16)
    x16 = ctx.fields(c16)
    _, ld = green_and_logdet(p16, ch16.expk, x16, 0)
    assert abs(st["logdet"] - ld) <= TOL64 * max(1.0, abs(ld))
    assert st["max_drift_green"] <= TOL_MIXED
    assert 0 < st["local_accepts"] < st["local_proposals"] == 256 * 100
    G_swept = ctx.green(c16)
    ctx.recompute()
    assert rel_g(G_swept, ctx.green(c16)) <= TOL_MIXED
    ctx.close()


def test_network_full_size_sampled(hq):
    """The network workload at full size (64 chains of 16x16, L = 160) with the
    trained network: chains 0 and 63 swept beside the oracle's network sweep,
    inner decisions replayed inside the tie band, cumulative accept, fields,
    log det and G compared."""
    w = workloads.holstein_16x16_network()
    g = w.groups[0]
    say("network 16x16 x64 full size, one sweep")
    gr = dict(nx=g.nx, chains=g.n_chains, g=g.g, beta=g.beta, n_stab=g.n_stab, proposal=1)
    from paper_1905_07440_amd import train
    net = train.load_weights("local")          # the trained network: cumulative updates are accepted
    ctx = make_ctx(hq, [gr], seed=w.seed)
    ctx.set_network(net)
    p = params_of(gr)
    nets = {c: nnmc.NNChain(dqmc.Chain(p, w.seed, c), net) for c in (0, 63)}
    for c, nn in nets.items():
        nn.sweep()
        bits = np.zeros(p.L * p.n, dtype=np.uint8)
        cum = np.zeros(1, dtype=np.uint8)
        for kind, sw, slot, acc, _ in nn.decisions:
            if kind == philox.KIND_NN:
                bits[slot] = acc
            if kind == philox.KIND_CUMULATIVE:
                cum[0] = acc
        ctx.set_replay(c, hq.KIND_NN, bits, BAND_MIXED)
        ctx.set_replay(c, hq.KIND_CUMULATIVE, cum, BAND_MIXED)
    ctx.sweep(1)
    for c, nn in nets.items():
        st = ctx.stats(c)
        assert st["replay_mismatches"] == 0, "chain %d" % c
        assert np.array_equal(ctx.fields(c), nn.c.x), "chain %d" % c
        assert abs(st["logdet"] - nn.c.logdet) <= TOL64 * max(1.0, abs(nn.c.logdet)), "chain %d" % c
        assert rel_g(ctx.green(c), nn.c.G) <= TOL64, "chain %d" % c
        assert st["cumulative_accepts"] == nn.cumulative_accepts
        assert st["nn_accepts"] == nn.inner_accepts
    ctx.close()


def test_uneven_groups_per_chain_coupling(hq):
    """Two lattice sizes in one context, g per chain from U(0.8, 1.6)."""
    say("uneven groups 4x4 + 6x6")
    groups = [dict(nx=4, chains=2, beta=2.0, n_stab=10, g_range=(0.8, 1.6)),
              dict(nx=6, chains=2, beta=2.0, n_stab=10, g_range=(0.8, 1.6))]
    ctx = make_ctx(hq, groups, seed=4)
    ctx.sweep(1)
    chain = 0
    for gr in groups:
        for _ in range(gr["chains"]):
            from oracle.model import chain_coupling
            gc = chain_coupling(4, chain, 0.8, 1.6)
            ch = dqmc.Chain(params_of(gr, g=gc), 4, chain)
            ch.sweep()
            st = assert_state(ctx, chain, ch, TOL64, "uneven chain %d" % chain)
            assert st["g"] == gc
            chain += 1
    ctx.close()


def test_uneven_groups_shapes_and_directions(hq):
    """Three lattice groups of different N, L and n_stab (one block per chain,
    three blocks, four blocks) as parallel branches of one captured sweep, an
    upward and a downward sweep, every chain against the oracle."""
    say("uneven groups 4x4 / 6x6 / 3x3, mixed shapes")
    groups = [dict(nx=4, chains=2, beta=1.0, n_stab=10, g=1.2),
              dict(nx=6, chains=3, beta=1.2, n_stab=4, g=1.1),
              dict(nx=3, chains=2, beta=0.8, n_stab=2, g=1.3)]
    ctx = make_ctx(hq, groups, seed=9)
    ctx.sweep(2)
    chain = 0
    for gr in groups:
        for _ in range(gr["chains"]):
            ch = dqmc.Chain(params_of(gr), 9, chain)
            ch.sweep(); ch.sweep()
            assert_state(ctx, chain, ch, TOL64, "group nx=%d chain %d" % (gr["nx"], chain))
            chain += 1
    ctx.close()


@pytest.mark.parametrize("case", ["atomic", "free", "nx2", "two_slices", "one_block", "one_block_global",
                                  "three_blocks_global", "phonon_params"])
def test_edge_cases(hq, case):
    """Degenerate lattices and slicings, every chain against the oracle after
    an upward and a downward sweep (one_block: L = n_stab, a single block per
    chain, with three chains; one_block_global: the same with block moves,
    whose determinants come from scratch; three_blocks_global: a pairwise
    tree with an unpaired block; phonon_params: mass, frequency, chemical
    potential, time step and move widths away from their defaults)."""
    say("edge case %s" % case)
    gr = {"atomic": dict(nx=3, chains=1, t=0.0, beta=1.0, n_stab=5, g=1.3),
          "free": dict(nx=4, chains=1, g=0.0, beta=2.0, n_stab=5),
          "nx2": dict(nx=2, chains=2, beta=2.0, n_stab=4, g=1.0, mu=0.3),
          "two_slices": dict(nx=4, chains=2, beta=0.2, n_stab=1, g=1.0),
          "one_block": dict(nx=3, chains=3, beta=1.0, n_stab=10, g=1.2),
          "one_block_global": dict(nx=3, chains=2, beta=1.0, n_stab=10, g=1.2, global_width=1.0),
          "three_blocks_global": dict(nx=4, chains=2, beta=0.6, n_stab=2, g=1.2, global_width=1.0),
          "phonon_params": dict(nx=4, chains=2, beta=1.0, n_stab=4, g=0.9, mass=2.0, omega=0.5, mu=-0.4,
                                dtau=0.125, local_width=0.8, global_width=0.7)}[case]
    ctx = make_ctx(hq, [gr], seed=5)
    ctx.sweep(2)
    for c in range(gr["chains"]):
        ch = dqmc.Chain(params_of(gr), 5, c)
        ch.sweep(); ch.sweep()
        assert_state(ctx, c, ch, TOL64, "%s chain %d" % (case, c))
    ctx.close()


def test_batched_observables_match_per_chain(hq):
    """hq_read_observables over two lattice groups (FP64 and a mixed context)
    gives each chain's five values exactly as hq_read_stats does."""
    say("batched observables")
    for prec in (0, 1):
        groups = [dict(nx=4, chains=3, beta=1.0, n_stab=5, g=1.2), dict(nx=6, chains=2, beta=1.0, n_stab=5, g=1.1)]
        ctx = make_ctx(hq, groups, precision=prec, seed=3)
        ctx.sweep(1)
        ob = ctx.observables()
        assert ob.shape == (5, 5)
        for c in range(5):
            st = ctx.stats(c)
            ref = [st["density"], st["double_occupancy"], st["s_cdw"], st["x_mean"], st["x2_mean"]]
            assert np.array_equal(ob[c], np.array(ref)), "precision %d chain %d" % (prec, c)
        with pytest.raises(hq.HQError):
            ctx._check(ctx._lib.hq_read_observables(ctx._ctx, ob.ctypes.data, 24))
        ctx.close()


def test_observables_match_oracle(hq):
    say("observables")
    gr = dict(nx=4, chains=1, g=1.0, beta=2.0, n_stab=5)
    ctx = make_ctx(hq, [gr], seed=9)
    ctx.sweep(1)
    ch = dqmc.Chain(params_of(gr), 9, 0)
    ch.sweep()
    st = ctx.stats(0)
    ob = ch.observables()
    for k_gpu, k_or in [("density", "density"), ("double_occupancy", "double_occupancy"),
                        ("s_cdw", "s_cdw"), ("x_mean", "x_mean"), ("x2_mean", "x2_mean")]:
        assert abs(st[k_gpu] - ob[k_or]) <= 1e-10 * max(1.0, abs(ob[k_or])), k_gpu
    ctx.close()


def test_set_fields_and_recompute(hq):
    say("set_fields")
    gr = dict(nx=6, chains=2, g=1.2, beta=2.0, n_stab=10)
    p = params_of(gr)
    x = workloads.random_fields(123, p.L, p.n, scale=0.7)
    ctx = make_ctx(hq, [gr], seed=1)
    ctx.set_fields(1, x)
    ch = dqmc.Chain(p, 1, 1, x=x)
    assert np.array_equal(ctx.fields(1), x)
    assert rel_g(ctx.green(1), ch.G) <= TOL64
    ctx.sweep(1)
    ch.sweep()
    assert_state(ctx, 1, ch, TOL64, "after set_fields")
    G_before = ctx.green(1)
    ctx.recompute()
    assert rel_g(ctx.green(1), G_before) <= TOL64
    ctx.close()


@pytest.mark.parametrize("nx,precision,extra", [(8, 0, dict(global_width=0.5)), (12, 1, {})])
def test_bitwise_deterministic(hq, nx, precision, extra):
    """The same seed and the same kernel choices give the same bits.  The
    autotuner picks GEMM tiles and the delayed-update block from timings, and
    different tiles or blocks sum in different orders, so both contexts are
    pinned to one choice, with G recomputed under it, before the sweeps."""
    say("determinism nx=%d precision=%d" % (nx, precision))
    gr = dict(nx=nx, chains=2, g=1.2, beta=2.0, n_stab=4, **extra)
    out = []
    for _ in range(2):
        ctx = make_ctx(hq, [gr], seed=21, precision=precision, delay=16)
        ctx.set_tuning(0, 0, 0)        # 64x64 tiles for every product, two-pass wrap
        ctx.recompute()
        ctx.sweep(2)
        out.append((ctx.fields(1), ctx.green(1), ctx.stats(1)["logdet"]))
        ctx.close()
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])
    assert out[0][2] == out[1][2]


def test_invalid_arguments(hq):
    say("invalid arguments")
    gr = dict(nx=4, chains=1, beta=2.0, n_stab=5)
    ctx = make_ctx(hq, [gr])
    with pytest.raises(hq.HQError):
        ctx.set_fields(0, np.zeros(7))
    bad = np.zeros((20, 16))
    bad[3, 3] = np.nan
    with pytest.raises(hq.HQError):
        ctx.set_fields(0, bad)
    with pytest.raises(hq.HQError):
        ctx.green(5)
    with pytest.raises(hq.HQError):
        ctx.set_network(np.zeros(10, dtype=np.float32))
    ctx.sweep(1)                       # the context is still usable
    assert ctx.stats(0)["local_proposals"] == 16 * 20
    ctx.close()
    with pytest.raises(hq.HQError):
        make_ctx(hq, [dict(nx=4, chains=1, beta=2.0, n_stab=5, proposal=1)]).sweep(1)   # no network loaded


@pytest.mark.parametrize("nu", [1, 2])
def test_network_block_moves_and_inner_sweeps(hq, nu):
    """Network local moves and network block moves (the convolutional network
    over the column and its neighbour means), n_u sweeps of each per
    cumulative accept, on 4x4 (L = 8): inner decisions of both kinds replayed
    inside the tie band, fields, log det and every counter against the oracle."""
    say("network block moves 4x4 n_u=%d" % nu)
    gr = dict(nx=4, chains=2, g=1.2, beta=0.8, n_stab=4, proposal=1, global_width=0.4, nn_sweeps=nu)
    p = params_of(gr)
    w = workloads.random_network(17, scale=0.1)
    cw = (0.2 * np.random.default_rng(23).standard_normal(nnmc.cnn_count(p.L))).astype(np.float32)
    ctx = make_ctx(hq, [gr], seed=6)
    ctx.set_network(w)
    with pytest.raises(hq.HQError):
        ctx.sweep(1)                                   # block moves need their network first
    with pytest.raises(hq.HQError):
        ctx.set_block_network(cw[:-1], p.L)
    ctx.set_block_network(cw, p.L)
    nets = [nnmc.NNChain(dqmc.Chain(p, 6, c), w, cnn=cw, nu=nu) for c in range(2)]
    for s in range(3):
        for c, nn in enumerate(nets):
            nn.sweep()
            bits = {philox.KIND_NN: np.zeros(nu * p.L * p.n, dtype=np.uint8),
                    philox.KIND_NN_GLOBAL: np.zeros(nu * p.n, dtype=np.uint8),
                    philox.KIND_CUMULATIVE: np.zeros(1, dtype=np.uint8)}
            for kind, sw, slot, acc, _ in nn.decisions:
                if sw == s:
                    bits[kind][slot] = acc
            ctx.set_replay(c, hq.KIND_NN, bits[philox.KIND_NN], BAND_MIXED)
            ctx.set_replay(c, hq.KIND_NN_GLOBAL, bits[philox.KIND_NN_GLOBAL], BAND_MIXED)
            ctx.set_replay(c, hq.KIND_CUMULATIVE, bits[philox.KIND_CUMULATIVE], BAND_MIXED)
        ctx.sweep(1)
        for c, nn in enumerate(nets):
            st = ctx.stats(c)
            assert st["replay_mismatches"] == 0
            assert np.array_equal(ctx.fields(c), nn.c.x), "sweep %d chain %d" % (s, c)
            assert abs(st["logdet"] - nn.c.logdet) <= TOL64 * max(1.0, abs(nn.c.logdet))
            assert rel_g(ctx.green(c), nn.c.G) <= TOL64, "sweep %d chain %d" % (s, c)
            assert st["cumulative_accepts"] == nn.cumulative_accepts
            assert st["nn_proposals"] == nn.inner_proposals and st["nn_accepts"] == nn.inner_accepts
            assert st["global_proposals"] == nn.block_proposals and st["global_accepts"] == nn.block_accepts
            acc, margin = ctx.decisions(c, hq.KIND_NN_GLOBAL)
            assert acc.size == nu * p.n and np.all(np.isfinite(margin))
    assert sum(nn.block_accepts for nn in nets) > 0
    ctx.close()


@pytest.mark.parametrize("kind,nx,beta,extra", [(0, 4, 0.8, {}), (1, 4, 0.8, {}), (0, 2, 0.4, {}), (0, 4, 1.2, {}),
                                                 (0, 4, 0.8, dict(mass=1.5, omega=0.7, mu=0.2, local_width=0.9))])
def test_network_proposals_and_cumulative_update(hq, kind, nx, beta, extra):
    """Network-proposed sweeps on 4x4 (L = 8), ReLU and softplus networks, on
    2x2 with L = 4 (every patch wraps around in space and time, one block per
    chain), on 4x4 with L = 12 (three blocks: a tree with an unpaired one), and
    with non-default phonon mass, frequency, chemical potential and width: inner
    decisions replayed inside the tie band (FP32 network vs the oracle's FP64
    forward), cumulative accepts compared."""
    say("network proposals %dx%d, activation %d" % (nx, nx, kind))
    gr = dict(nx=nx, chains=2, g=1.2, beta=beta, n_stab=4, proposal=1, **extra)
    w = workloads.random_network(17, scale=0.1)
    ctx = make_ctx(hq, [gr], seed=6, activation=kind)
    ctx.set_network(w)
    nets = [nnmc.NNChain(dqmc.Chain(params_of(gr), 6, c), w, kind=kind) for c in range(2)]
    p = params_of(gr)
    for s in range(3):
        for c, nn in enumerate(nets):
            nn.sweep()
            bits = np.zeros(p.L * p.n, dtype=np.uint8)
            cum = np.zeros(1, dtype=np.uint8)
            for kind, sw, slot, acc, _ in nn.decisions:
                if sw == s and kind == philox.KIND_NN:
                    bits[slot] = acc
                if sw == s and kind == philox.KIND_CUMULATIVE:
                    cum[0] = acc
            ctx.set_replay(c, hq.KIND_NN, bits, BAND_MIXED)
            ctx.set_replay(c, hq.KIND_CUMULATIVE, cum, BAND_MIXED)
        ctx.sweep(1)
        for c, nn in enumerate(nets):
            st = ctx.stats(c)
            assert st["replay_mismatches"] == 0
            assert np.array_equal(ctx.fields(c), nn.c.x), "sweep %d chain %d" % (s, c)
            assert abs(st["logdet"] - nn.c.logdet) <= TOL64 * max(1.0, abs(nn.c.logdet))
            assert rel_g(ctx.green(c), nn.c.G) <= TOL64, "sweep %d chain %d" % (s, c)
            assert st["cumulative_accepts"] == nn.cumulative_accepts
            assert st["nn_accepts"] == nn.inner_accepts
    ctx.close()
