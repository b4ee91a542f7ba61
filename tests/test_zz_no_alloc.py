"""hq_create_static (the entry point that allocates no device memory: the
library's static device array is the workspace) against hq_create with a
caller-owned workspace, on the same seeded chains: two contexts in a row, the
second smaller than the first, so the second reuses the array the first
left behind."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL64 = 1e-10


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


def run(hq, static, gr, seed, sweeps):
    group = hq.make_group(gr["nx"], gr["chains"], g=gr["g"], beta=gr["beta"], n_stab=gr["n_stab"],
                          global_width=gr.get("global_width", 0.0))
    ctx = hq.Context([group], precision=0, seed=seed, record=True, static=static)
    if static:
        t = ctx.tuning(0)
        assert (t["gemm_tile_fp64"], t["wrap"]) == (hq.tile_name(0), "kron")
    else:
        ctx.set_tuning(0, 0, 0, wrap="kron")     # the static context's fixed choices
    ctx.sweep(sweeps)
    out = [(ctx.fields(c), ctx.green(c), ctx.stats(c), ctx.decisions(c, hq.KIND_LOCAL)[0])
           for c in range(gr["chains"])]
    return ctx, out


@pytest.mark.parametrize("gr,seed", [
    (dict(nx=8, chains=3, g=1.2, beta=1.6, n_stab=4, global_width=0.8), 41),   # the larger context first
    (dict(nx=4, chains=2, g=1.0, beta=0.8, n_stab=4), 42),                     # then a smaller one
])
def test_static_workspace_matches_caller_workspace(hq, gr, seed):
    say("static workspace: %dx%d x%d chains, L = %d" % (gr["nx"], gr["nx"], gr["chains"], round(gr["beta"] / 0.1)))
    ctx_s, got = run(hq, True, gr, seed, 2)
    # a second static context on the same GPU would share the array: refused while this one lives
    with pytest.raises(hq.HQError) as e:
        hq.Context([hq.make_group(4, 1, beta=0.8, n_stab=4)], static=True)
    assert e.value.status == hq.HQ_ESTATE
    ctx_s.close()
    ctx_w, ref = run(hq, False, gr, seed, 2)
    ctx_w.close()
    for c, ((x, G, st, acc), (xr, Gr, sr, accr)) in enumerate(zip(got, ref)):
        assert np.array_equal(acc, accr), "chain %d: decisions" % c
        assert np.array_equal(x, xr), "chain %d: fields" % c
        assert np.max(np.abs(G - Gr)) <= TOL64 * np.max(np.abs(Gr)), "chain %d: G" % c
        assert abs(st["logdet"] - sr["logdet"]) <= TOL64 * max(1.0, abs(sr["logdet"])), "chain %d" % c
        assert st["local_accepts"] == sr["local_accepts"] and st["global_accepts"] == sr["global_accepts"]


def test_static_workspace_limits(hq):
    say("static workspace limits")
    big = hq.make_group(12, 16, beta=2.4, n_stab=6)          # about 100 MB of workspace
    with pytest.raises(hq.HQError) as e:
        hq.Context([big], precision=1, static=True)
    assert e.value.status == hq.HQ_ENOMEM and "static workspace holds" in str(e.value)
    two = [hq.make_group(4, 1, beta=0.8, n_stab=4), hq.make_group(6, 1, beta=0.8, n_stab=4)]
    with pytest.raises(hq.HQError) as e:
        hq.Context(two, static=True)
    assert e.value.status == hq.HQ_EINVAL
    ctx = hq.Context([hq.make_group(4, 1, beta=0.8, n_stab=4)], static=True)   # the failures left it free
    ctx.sweep(1)
    assert ctx.stats(0)["local_proposals"] == 16 * 8
    ctx.close()
