"""Benchmark of the TUfRG flow right-hand side on one MI355X.

A step is one full right-hand side (loops, projections, products) of the
t' = -0.25, n = 0.85, N_ff = 13, 24x24 transfer / 96x96 fine-grid workload
with its inputs resident in HBM.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-flow] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "flow-RHS evals/sec and full-flow time vs plain FP64 GPU at Λ_c err ≤1%"
PEAK_FP64_TFLOPS = 78.6     # MI355X FP64 vector peak (256 CUs x 64 lanes x 2 flops x 2.4 GHz)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-flow", action="store_true", help="skip the full-flow timing")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(point, seconds):
    """The FP64 CPU oracle, untuned, on a bounded sample of the same workload."""
    import numpy as np

    import synth
    from oracle.lattice import FormFactors
    from oracle.rhs import rhs as oracle_rhs
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = 1
    ff = FormFactors(point.shells)
    X = synth.random_channels(point.nq, ff.nff, seed=7, scale=1.0)
    Ts = [0.5, 0.05, 0.01, 0.2]
    n, t0 = 0, time.perf_counter()
    while True:
        oracle_rhs(point, Ts[n % len(Ts)], X, ff)
        n += 1
        el = time.perf_counter() - t0
        log(f"[cpu] oracle rhs {n} done, {el:.1f} s")
        if el >= seconds or n >= 50:
            break
    return {"value": n / el, "unit": "RHS evals/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} full right-hand sides of the same workload (oracle, FP64, numpy)"}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the right-hand side would shard over transfer momenta; see DESIGN.md)",
              file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1604_06296_amd as tf
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    w = synth.cfg2()
    pt = w.points[0]
    pt.mu = tf.mu_from_filling(pt.t, pt.tp, pt.filling, pt.mu_T, pt.mu_L)
    ctx = tf.Context([pt])
    nff = 13
    X = torch.from_numpy(synth.random_channels(pt.nq, nff, seed=5, scale=1.0).reshape(3, -1)).cuda()
    out = ctx.empty(3)
    dchi = ctx.empty(2)
    # temperatures spread over the flow range
    Ts = [math.exp(math.log(10.0) + (math.log(1e-3) - math.log(10.0)) * i / 63) for i in range(64)]
    log(f"[bench] workload {w.name}: Nq={pt.nq} Nk={pt.Lk ** 2} Nff={nff} mu={pt.mu:.6f}")

    for i in range(args.warmup):
        ctx.rhs(Ts[i % 64], X, out)
    torch.cuda.synchronize()
    log("[bench] warmup done")
    t0 = time.perf_counter()
    for i in range(args.steps):
        ctx.rhs(Ts[i % 64], X, out)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms = 1e3 * el / args.steps
    log(f"[bench] {args.steps} rhs in {el:.4f} s ({ms:.4f} ms each)")

    # dominant kernel (loops): live HIP-event timing on the context's stream
    nb = max(args.steps, 20)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ctx.bubbles(Ts[0], dchi)
    ev0.record()
    for i in range(nb):
        ctx.bubbles(Ts[i % 64], dchi)
    ev1.record()
    torch.cuda.synchronize()
    loop_ms = ev0.elapsed_time(ev1) / nb
    flops = ctx.flop_count()
    achieved = flops["loops"] / (loop_ms * 1e-3) / 1e12
    log(f"[bench] loop kernel {loop_ms * 1e3:.2f} us/launch, {achieved:.2f} TFLOP/s")

    flow_info = None
    if not args.no_flow:
        Xf = ctx.empty(3).zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = ctx.flow(Xf, tf.FlowOptions(T0=w.T0, Tmin=w.Tmin, Xmax=w.Xmax, scheme="dopri5",
                                        rtol=w.rtol, atol=w.atol))[0]
        fl = time.perf_counter() - t0
        flow_info = {"flow_time_s": fl, "status": r.status, "Tc": r.Tc, "channel": r.channel,
                     "q_index": r.q_index, "irrep": r.irrep, "n_rhs": r.n_rhs, "n_steps": r.n_steps}
        log(f"[bench] flow {fl:.3f} s: {flow_info}")

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(pt, args.cpu_seconds)

    line = {
        "metric": METRIC,
        "value": args.steps / el,
        "unit": "RHS evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "Lq": pt.Lq, "Lk": pt.Lk, "nff": nff, "t": pt.t,
                   "tp": pt.tp, "filling": pt.filling, "mu": pt.mu, "U": pt.U,
                   "flow": flow_info, "flops_per_rhs": flops},
        "roofline": {"bound": "alu", "kernel": "k_loops", "achieved": achieved,
                     "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                     "traffic": None, "launch_us": loop_ms * 1e3},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
