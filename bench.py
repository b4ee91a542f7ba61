"""Benchmark: phonon-field updates per second of the Holstein DQMC sweep on one
MI355X, all chains together.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c3]

A step is one full sweep of every chain (wraps, local moves with delayed
updates, FP64 stabilisation every n_stab slices, and the block moves or
network proposals the workload has).  An update is one proposal, accepted or
not.  Inputs are synthetic: seeded Gaussian initial fields and the model
parameters of the workload; the chains live in HBM before timing starts.

Prints one JSON line.  Besides the throughput it carries the mixed-precision
accuracy (max |G_mixed - G_FP64| at stabilisation points and the log-weight
error), the roofline of the dominant kernel (per-launch duration from HIP
events on the library's stream, in a profiling pass right after the timed
sweeps), and the oracle timed on host cores on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

MI355X_PEAK = {"fp64": 78.6e12, "fp32": 157.3e12, "hbm": 8.0e12}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-chains", type=int, default=0)
    return ap.parse_args()


def proposals_per_sweep(w):
    total = 0
    for g in w.groups:
        L = round(g.beta / g.dtau)
        n = g.nx * g.nx
        total += g.n_chains * n * L
        if g.global_width > 0 and g.proposal == 0:
            total += g.n_chains * n
    return total


def phase_flops(w, phase, accept_rate):
    """Algorithmic flops of one launch-region of a phase, summed over chains."""
    fl = 0.0
    for g in w.groups:
        n = g.nx * g.nx
        if phase == "wrap":          # G <- D e^{-dtau K} G e^{+dtau K} D^-1: two N^3 products
            fl += g.n_chains * 2 * 2.0 * n ** 3
        elif phase == "local":       # one slice: a rank-1 update of N^2 per accepted move
            fl += g.n_chains * accept_rate * n * 2.0 * n * n
    return fl


def cpu_baseline(w, max_chains):
    """The oracle, as it stands, on a bounded sample: one sweep of up to P chains,
    P worker processes with one BLAS thread each."""
    import multiprocessing as mp
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    os.environ["OMP_NUM_THREADS"] = "1"
    os.environ["MKL_NUM_THREADS"] = "1"
    g = w.groups[0]
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    P = max(1, min(16, cores, g.n_chains, max_chains or 16))
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(P) as pool:
        res = pool.map(_oracle_one_sweep, [(w.name, c) for c in range(P)])
    wall = time.perf_counter() - t0
    props = sum(r[0] for r in res)
    busy = max(r[1] for r in res)
    return {"value": props / busy, "unit": "updates/s", "cores": P, "kind": "oracle",
            "sample": "one sweep of %d of the %d chains of %s, one process per chain "
                      "(single-threaded BLAS); rate = proposals / slowest worker's sweep time "
                      "(%.1f s wall incl. start-up)" % (P, g.n_chains, w.name, wall)}


def _oracle_one_sweep(arg):
    name, chain = arg
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    import workloads
    from oracle import dqmc
    from oracle.model import Params
    w = {v().name: v for v in workloads.ALL.values()}[name]()
    g = w.groups[0]
    p = Params(nx=g.nx, t=g.t, mu=g.mu, mass=g.mass, omega=g.omega, g=g.g, beta=g.beta, dtau=g.dtau,
               n_stab=g.n_stab, local_width=g.local_width, global_width=g.global_width)
    ch = dqmc.Chain(p, w.seed, chain)
    t0 = time.perf_counter()
    ch.sweep()
    dt = time.perf_counter() - t0
    return ch.local_proposals + ch.global_proposals, dt


def main():
    a = parse()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the chains of this workload are independent and the "
              "library has no multi-GPU path (see the sharding paragraph of the design notes).",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import workloads
    from paper_1905_07440_amd import hq

    w = workloads.ALL[a.workload]()
    ctx = hq.Context(hq.groups_from_workload(w), precision=w.precision, seed=w.seed, delay=w.delay)
    stream = ctx._stream
    ctx.sweep(a.warmup)
    ctx.synchronize()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    ctx.sweep(a.steps)
    e1.record(stream)
    ctx.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / a.steps
    value = proposals_per_sweep(w) / (ms * 1e-3)

    stats = [ctx.stats(c) for c in range(ctx.n_chains)]
    acc = sum(s["local_accepts"] for s in stats) / max(1, sum(s["local_proposals"] for s in stats))
    max_dg = max(s["max_drift_green"] for s in stats)
    max_dl = max(s["max_drift_logdet"] for s in stats)

    # profiling pass: per-phase device time from HIP events on the library stream
    ctx.set_profiling(True)
    ctx.sweep(1)
    phases = {}
    for ph in ("wrap", "local", "stab", "global", "network"):
        t, k = ctx.phase_time(ph)
        if k:
            phases[ph] = {"ms_per_sweep": t, "launch_regions": k, "us_per_region": 1e3 * t / k}
    ctx.set_profiling(False)
    dominant = max(phases, key=lambda p: phases[p]["ms_per_sweep"])
    roof_phase = dominant if dominant in ("wrap", "local") else max(
        ("wrap", "local"), key=lambda p: phases.get(p, {"ms_per_sweep": 0})["ms_per_sweep"])
    per = phases[roof_phase]["us_per_region"] * 1e-6
    flops = phase_flops(w, roof_phase, acc)
    peak = MI355X_PEAK["fp32" if w.precision else "fp64"]
    roofline = {"bound": "mfma", "achieved": flops / per / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                "frac": flops / per / peak, "traffic": None, "kernel": roof_phase,
                "note": "dominant phase by device time: %s" % dominant}

    cpu = None
    if not a.no_cpu_baseline:
        cpu = cpu_baseline(w, a.cpu_sample_chains)

    g0 = w.groups[0]
    out = {
        "metric": "phonon-field updates/s (all chains), mixed vs FP64 at |G-G_FP64|<=1e-5",
        "value": value, "unit": "updates/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if w.precision else "f64", "data": "synthetic",
        "config": {"workload": w.name, "chains": w.n_chains, "nx": [g.nx for g in w.groups],
                   "L": [round(g.beta / g.dtau) for g in w.groups], "n_stab": g0.n_stab,
                   "precision": "mixed" if w.precision else "fp64", "delay": w.delay or 16,
                   "parallelism": "independent chains, one GPU"},
        "accuracy": {"max_abs_G_minus_fp64": max_dg, "max_logdet_err": max_dl,
                     "log_weight_err": 2 * max_dl, "gate_1e-5": max_dg <= 1e-5},
        "local_acceptance": acc,
        "phases": phases,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "wall_s": wall,
    }
    print(json.dumps(out))
    ctx.close()


if __name__ == "__main__":
    main()
