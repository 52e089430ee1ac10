"""Benchmark of the TUfRG flow right-hand side on one MI355X.

A step is one full right-hand side (loops, projections, products) of the
t' = -0.25, n = 0.85, N_ff = 13, 24x24 transfer / 96x96 fine-grid workload
with its inputs resident in HBM; `value` is right-hand sides per second.
Further legs measure the other rows against the plain FP64 GPU path:
  mixed      N_ff = 21, 48x48 / 128x128: FP64 vs mixed precision, per-result errors
  batched    64 uneven points in one context: batched RK4 flow, eager vs graph
  surrogate  N_ff = 21, 64x64 / 160x160: flow with and without the learned loops
Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-flow] [--no-cpu]
                    [--no-mixed] [--no-batched] [--no-surrogate]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "flow-RHS evals/sec and full-flow time vs plain FP64 GPU at Λ_c err ≤1%"
PEAK_FP64_TFLOPS = 78.6     # MI355X FP64 vector peak (256 CUs x 64 lanes x 2 flops x 2.4 GHz); FP64 MFMA the same
PEAK_FP32_TFLOPS = 157.3    # MI355X FP32 vector (and FP32 MFMA) peak
PEAK_BF16_TFLOPS = 2500.0   # MI355X dense BF16 MFMA peak

# HBM bytes per launch of the loop kernel at the headline workload (default
# geometry), from two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) scaled by
# the counters of a plain 64 MiB device copy; valid only for the kernel
# sources they were taken with (loops.hip, loop_body.h, loop_math.h;
# profiles/loop_kernel_traffic_*.md).
LOOP_TRAFFIC = {"sources_sha256": "3102942e7854bb619e9476afc61f552e07e8a62fabfcaf87aa2aabe346318ac4",
                "bytes": 584064}


def loop_flops_algorithmic(Lq, Lk, n_harm, c_pair=157.0):
    """Algorithmic flops of one loop-kernel launch on a uniform Lq x Lq grid:
    per (q, p) pair (q over the point-group orbit representatives, p over the
    half fine grid) the loop-derivative flops c_pair (the kernel's measured
    FP64 count per pair) plus 4 N_S' for projecting both channels onto the
    N_S' harmonics (a multiply-add each).  The kernel executes the projection
    in separable form (fewer flops); the count credits the direct one."""
    nirr = (Lq // 2 + 1) * (Lq // 2 + 2) // 2
    pairs = nirr * Lk * (Lk // 2 + 1)
    return pairs * (c_pair + 4.0 * n_harm)


def loop_kernel_sources_sha():
    h = hashlib.sha256()
    for f in ("loops.hip", "loop_body.h", "loop_math.h"):
        with open(os.path.join(ROOT, "paper_1604_06296_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-flow", action="store_true", help="skip the full-flow timing")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--no-omega", action="store_true")
    ap.add_argument("--no-wedge", action="store_true")
    ap.add_argument("--no-dense", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--train-steps", type=int, default=8000)
    ap.add_argument("--probe-loops", type=int, default=0,
                    help="counter probe only: one 64 MiB device copy (calibration), then this many "
                         "loop steps of the headline workload; prints no JSON")
    ap.add_argument("--probe-projections", type=int, default=0,
                    help="counter probe only: this many projection steps (tufrg_project) of the "
                         "headline workload (FP64) and of the N_ff=21, 48x48 workload (FP64, then "
                         "mixed); prints no JSON")
    ap.add_argument("--probe-wedge", type=int, default=0,
                    help="trace probe only: this many right-hand sides of the N_ff=21, 48x48 workload "
                         "(FP64) per momentum, one fill kernel as a marker, then as many with "
                         "symmetric states; prints no JSON")
    return ap.parse_args()


def probe_loops(n):
    """Fixed kernel sequence for hardware-counter runs (rocprofv3 --pmc)."""
    import torch

    import paper_1604_06296_amd as tf
    import synth
    words = 64 * 1024 * 1024 // 8
    a = torch.ones(words, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)                                    # 64 MiB read + 64 MiB written
    torch.cuda.synchronize()
    w = synth.cfg2()
    pt = w.points[0]
    pt.mu = tf.mu_from_filling(pt.t, pt.tp, pt.filling, pt.mu_T, pt.mu_L)
    ctx = tf.Context([pt])
    d = ctx.empty(2)
    for _ in range(n):
        ctx.bubbles(0.05, d)
    torch.cuda.synchronize()
    log(f"[probe] copy of {2 * words * 8} bytes, {n} loop steps, geometry {ctx.geometry(0)}")


def probe_projections(n):
    """Fixed projection sequence for hardware-counter runs (rocprofv3 --pmc)."""
    import torch

    import paper_1604_06296_amd as tf
    import synth
    for w, prec in ((synth.cfg2(), "fp64"), (synth.cfg3(), "fp64"), (synth.cfg3(), "mixed")):
        pt = w.points[0]
        if pt.mu is None:
            pt.mu = tf.mu_from_filling(pt.t, pt.tp, pt.filling, pt.mu_T, pt.mu_L)
        ctx = tf.Context([pt], precision=prec)
        X = torch.from_numpy(synth.random_channels(pt.nq, pt.nff, seed=5).reshape(3, -1)).cuda()
        V = ctx.empty(3)
        for _ in range(n):
            ctx.project(X, V)
        torch.cuda.synchronize()
        log(f"[probe] {w.name} {prec}: {n} projection steps")
        ctx.close()


def probe_wedge(n):
    """Fixed right-hand-side sequence for a kernel trace of the symmetric-state mode."""
    import torch

    import paper_1604_06296_amd as tf
    import synth
    pt = synth.cfg3().points[0]
    for sym in (False, True):
        ctx = tf.Context([pt], symmetric_state=sym)
        X = ctx.empty(3).zero_()
        out = ctx.empty(3)
        for _ in range(n):
            ctx.rhs(0.05, X, out)
        torch.cuda.synchronize()
        log(f"[probe] {n} right-hand sides, symmetric_state={sym}")
        ctx.close()
        if not sym:
            torch.zeros(1, device="cuda").fill_(1.0)    # marker between the two runs
            torch.cuda.synchronize()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def _cpu_chunk(args):
    """One worker's share of an oracle right-hand side: the momenta of one chunk."""
    point, T, X, q_index = args
    from oracle.lattice import FormFactors
    from oracle.rhs import rhs as oracle_rhs
    return oracle_rhs(point, T, X, FormFactors(point.shells), q_index=q_index)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(point, seconds):
    """The FP64 CPU oracle, untuned, on a bounded sample of the same workload.

    The oracle's right-hand side is evaluated per transfer momentum (its
    q_index argument), so one right-hand side is split into one chunk of
    momenta per worker process (one process per core this process may run
    on, BLAS limited to one thread each) and the chunks are put back
    together in order.  Runs before the GPU is touched: the workers are
    fresh interpreters started by the spawn method."""
    import multiprocessing as mp

    import numpy as np

    import synth
    from oracle.lattice import mu_from_filling
    if point.mu is None:
        point.mu = mu_from_filling(point.filling, point.t, point.tp, point.mu_T, point.mu_L)
    cores = len(os.sched_getaffinity(0))
    saved = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in saved:
        os.environ[k] = "1"
    X = synth.random_channels(point.nq, point.nff, seed=7, scale=1.0)
    chunks = [c for c in np.array_split(np.arange(point.nq), cores) if c.size]
    Ts = [0.5, 0.05, 0.01, 0.2]
    try:
        with mp.get_context("spawn").Pool(processes=len(chunks)) as pool:
            pool.map(_cpu_chunk, [(point, Ts[0], X, c) for c in chunks[:1]])   # start-up of every worker
            n, t0 = 0, time.perf_counter()
            while True:
                parts = pool.map(_cpu_chunk, [(point, Ts[n % len(Ts)], X, c) for c in chunks])
                dX = np.concatenate(parts, axis=1)
                assert dX.shape == X.shape
                n += 1
                el = time.perf_counter() - t0
                log(f"[cpu] oracle rhs {n} done, {el:.1f} s")
                if el >= seconds or n >= 200:
                    break
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    return {"value": n / el, "unit": "RHS evals/s", "cores": len(chunks), "kind": "oracle",
            "cpu_model": _cpu_model(), "cores_available": cores, "blas_threads_per_worker": 1,
            "sample": f"{n} full right-hand sides of the same workload (oracle, FP64, numpy), each split "
                      f"over {len(chunks)} worker processes by transfer momentum"}


def _sync():
    import torch
    torch.cuda.synchronize()


def time_rhs(ctx, T, X, out, n=50):
    for _ in range(5):
        ctx.rhs(T, X, out)
    _sync()
    t0 = time.perf_counter()
    for _ in range(n):
        ctx.rhs(T, X, out)
    _sync()
    return (time.perf_counter() - t0) / n


def timed_flow(ctx, X, opts):
    X.zero_()
    _sync()
    t0 = time.perf_counter()
    res = ctx.flow(X, opts)
    _sync()
    return res, time.perf_counter() - t0


def kernel_table(ctx, T, X, out, reps, precision):
    """Each projection kernel and the products timed alone (the library's HIP events on the
    context's stream): microseconds per launch, algorithmic TFLOP/s, and its fraction of the
    peak of the unit that computes it.  The split-precision transforms execute three BF16
    products (hi.hi, hi.lo, lo.hi) per algorithmic multiply-add: executed = 3 x algorithmic."""
    mixed = precision == "mixed"
    units = {"forward_transform": ("bf16 mfma", PEAK_BF16_TFLOPS, 3) if mixed else ("fp64 mfma", PEAK_FP64_TFLOPS, 1),
             "bond_basis": ("fp64 valu", PEAK_FP64_TFLOPS, 1),
             "gather": ("fp64 valu", PEAK_FP64_TFLOPS, 1),
             "products": ("fp32", PEAK_FP32_TFLOPS, 1) if mixed else ("fp64", PEAK_FP64_TFLOPS, 1)}
    units["inverse_transform"] = units["forward_transform"]
    table = {}
    for k, (us, fl) in ctx.kernel_times(T, X, out, reps=reps).items():
        unit, peak, ex = units[k]
        tfl = fl / (us * 1e-6) / 1e12
        table[k] = {"us": us, "flops": fl, "tflops": tfl, "unit": unit, "peak": peak, "frac": tfl / peak,
                    "executed_per_algorithmic": ex}
    return table


def leg_mixed(tf, synth):
    """cfg3: plain FP64 against the mixed-precision form, per result."""
    import torch
    w = synth.cfg3()
    pt = w.points[0]
    out = {"workload": w.name}
    X = torch.from_numpy(synth.random_channels(pt.nq, pt.nff, seed=5).reshape(3, -1)).cuda()
    ctxs = {p: tf.Context([pt], precision=p, autotune=True) for p in ("fp64", "mixed")}
    opts = tf.FlowOptions(T0=w.T0, Tmin=w.Tmin, Xmax=w.Xmax, scheme="rk4", nsteps=w.nsteps, use_graph=True)
    res = {}
    for p, ctx in ctxs.items():
        o = ctx.empty(3)
        out[f"rhs_ms_{p}"] = 1e3 * time_rhs(ctx, 0.05, X, o)
        out[f"kernels_{p}"] = kernel_table(ctx, 0.05, X, o, 20, p)
        log(f"[mixed] {p} kernels (us): " + ", ".join(f"{k} {v['us']:.2f}" for k, v in out[f"kernels_{p}"].items()))
        Xf = ctx.empty(3)
        r, el = timed_flow(ctx, Xf, opts)
        V = ctx.project(Xf)
        res[p] = (r[0], el, Xf, V)
        out[f"flow_s_{p}"] = el
        log(f"[mixed] {p}: rhs {out[f'rhs_ms_{p}']:.3f} ms, flow {el:.3f} s, {r[0]}")
    # a diverging flow for the critical scale: the cfg2 point, RK4 in both precisions
    w2 = synth.cfg2()
    p2 = w2.points[0]
    p2.mu = tf.mu_from_filling(p2.t, p2.tp, p2.filling, p2.mu_T, p2.mu_L)
    o2 = tf.FlowOptions(T0=w2.T0, Tmin=w2.Tmin, Xmax=w2.Xmax, scheme="rk4", nsteps=400, use_graph=True)
    c2 = {}
    for p in ("fp64", "mixed"):
        cx = tf.Context([p2], precision=p, autotune=True)
        r, el = timed_flow(cx, cx.empty(3), o2)
        c2[p] = (r[0], el)
    a, b = c2["fp64"][0], c2["mixed"][0]
    out["diverging_flow"] = {
        "workload": w2.name + " (rk4, 400 steps)", "status": [a.status, b.status], "Tc": [a.Tc, b.Tc],
        "Tc_rel_err": (abs(b.Tc / a.Tc - 1) if (a.Tc and b.Tc) else None),
        "leading": [[a.channel, a.q_index, a.irrep], [b.channel, b.q_index, b.irrep]],
        "flow_s": [c2["fp64"][1], c2["mixed"][1]]}
    log(f"[mixed] cfg2 rk4: {out['diverging_flow']}")
    r64, rmx = res["fp64"][0], res["mixed"][0]
    maxV = [float(res[p][3].abs().max()) for p in ("fp64", "mixed")]
    out.update({
        "rhs_speedup": out["rhs_ms_fp64"] / out["rhs_ms_mixed"],
        "flow_speedup": out["flow_s_fp64"] / out["flow_s_mixed"],
        "status": [r64.status, rmx.status],
        "Tc": [r64.Tc, rmx.Tc],
        "Tc_rel_err": (abs(rmx.Tc / r64.Tc - 1) if (r64.Tc and rmx.Tc) else None),
        "leading": [[r64.channel, r64.q_index, r64.irrep], [rmx.channel, rmx.q_index, rmx.irrep]],
        "max_abs_X": [r64.max_abs_X, rmx.max_abs_X],
        "max_abs_X_rel_err": abs(rmx.max_abs_X / r64.max_abs_X - 1),
        "max_abs_V": maxV,
        "max_abs_V_rel_err": abs(maxV[1] / maxV[0] - 1),
        "X_end_rel_err": float((res["mixed"][2] - res["fp64"][2]).abs().max() / res["fp64"][2].abs().max()),
    })
    return out


def leg_batched(tf, synth):
    """cfg4: 64 uneven points, one context, RK4 flow eagerly and graph-replayed."""
    w = synth.cfg4()
    for p in w.points:
        p.mu = tf.mu_from_filling(p.t, p.tp, p.filling, p.mu_T, p.mu_L)
    ctx = tf.Context(w.points, autotune=True)
    out = {"workload": w.name, "points": len(w.points), "S": ctx.S,
           "loop_launch_form": "persistent queue" if ctx.geometry(0)[3] else "one block per item"}
    X = ctx.empty(3)
    Ts = [0.05] * len(w.points)
    o = ctx.empty(3)
    out["rhs_ms"] = 1e3 * time_rhs(ctx, Ts, X.zero_(), o, n=10)
    opts = dict(T0=w.T0, Tmin=w.Tmin, Xmax=w.Xmax, scheme="rk4", nsteps=w.nsteps)
    r_e, t_e = timed_flow(ctx, X, tf.FlowOptions(use_graph=False, **opts))
    r_g, t_g = timed_flow(ctx, X, tf.FlowOptions(use_graph=True, **opts))
    out.update({"flow_s_eager": t_e, "flow_s_graph": t_g, "graph_equals_eager": r_e == r_g,
                "diverged": sum(r.status == "diverged" for r in r_g),
                "rhs_total": sum(r.n_rhs for r in r_g)})
    log(f"[batched] rhs {out['rhs_ms']:.3f} ms, flow eager {t_e:.2f} s, graph {t_g:.2f} s")
    ctx.close()
    # the same batch with symmetric states (every flow starts at zero): one
    # momentum per orbit in the loop expansion, inverse transform and products
    sym = tf.Context(w.points, autotune=True, symmetric_state=True)
    Xs, os_ = sym.empty(3), sym.empty(3)
    rhs_ms = 1e3 * time_rhs(sym, Ts, Xs.zero_(), os_, n=10)
    r_s, t_s = timed_flow(sym, Xs, tf.FlowOptions(use_graph=True, **opts))
    same = all(a.status == b.status and a.n_steps == b.n_steps and a.channel == b.channel and a.irrep == b.irrep
               and (a.Tc is None or abs(a.Tc / b.Tc - 1) < 1e-8) for a, b in zip(r_s, r_g))
    out["symmetric_state"] = {"rhs_ms": rhs_ms, "flow_s_graph": t_s, "same_outcomes": same}
    log(f"[batched] symmetric states: rhs {rhs_ms:.3f} ms, flow graph {t_s:.2f} s, same outcomes {same}")
    sym.close()
    return out


def leg_omega(tf, synth, steps):
    """The benchmark point with the Omega cutoff at zero temperature: right-hand
    sides over the flow's range of Omega, the loop kernel alone, and the
    adaptive flow (Omega 800 -> 1e-3, stop at max|X| > 80) to its critical Omega."""
    import torch
    w = synth.cfg2_omega()
    pt = w.points[0]
    pt.mu = tf.mu_from_filling(pt.t, pt.tp, pt.filling, pt.mu_T, pt.mu_L)
    ctx = tf.Context([pt], regulator="omega")
    X = torch.from_numpy(synth.random_channels(pt.nq, pt.nff, seed=5, scale=1.0).reshape(3, -1)).cuda()
    o = ctx.empty(3)
    Oms = [math.exp(math.log(w.T0) + (math.log(w.Tmin) - math.log(w.T0)) * i / 63) for i in range(64)]
    for i in range(20):
        ctx.rhs(Oms[i % 64], X, o)
    _sync()
    t0 = time.perf_counter()
    for i in range(steps):
        ctx.rhs(Oms[i % 64], X, o)
    _sync()
    el = time.perf_counter() - t0
    loop_us, loop_flops = ctx.loop_kernel_time(0.05, reps=max(steps, 20))
    alg = loop_flops_algorithmic(pt.Lq, pt.Lk, ctx.harmonics(0)[0], c_pair=58.0)
    tflops = alg / (loop_us * 1e-6) / 1e12
    r, fl = timed_flow(ctx, ctx.empty(3), tf.FlowOptions(T0=w.T0, Tmin=w.Tmin, Xmax=w.Xmax, scheme="dopri5",
                                                         rtol=w.rtol, atol=w.atol))
    r = r[0]
    out = {"workload": w.name, "regulator": "omega", "rhs_per_s": steps / el, "ms_per_rhs": 1e3 * el / steps,
           "loop_kernel_us": loop_us, "loop_kernel_flops": alg, "loop_kernel_executed_flops": loop_flops,
           "loop_kernel_tflops": tflops,
           "loop_kernel_frac_fp64_peak": tflops / PEAK_FP64_TFLOPS,
           "flow": {"flow_time_s": fl, "status": r.status, "Omega_c": r.Tc, "channel": r.channel,
                    "q_index": r.q_index, "irrep": r.irrep, "n_rhs": r.n_rhs, "n_steps": r.n_steps}}
    log(f"[omega] rhs {out['ms_per_rhs']:.4f} ms, loop kernel {loop_us:.2f} us ({tflops:.2f} TFLOP/s), "
        f"flow {fl:.3f} s: {out['flow']}")
    return out


def leg_wedge(tf, synth, steps, Tc_ref):
    """Symmetric states (one momentum per C4v orbit in the inverse transform and the
    products): the benchmark point's adaptive flow from zero and right-hand sides of
    its end state over the flow's temperatures; the 48x48 / 128x128, N_ff = 21
    point's right-hand side at the flow's start (X = 0) against the per-momentum path."""
    import torch
    w = synth.cfg2()
    pt = w.points[0]
    pt.mu = tf.mu_from_filling(pt.t, pt.tp, pt.filling, pt.mu_T, pt.mu_L)
    ctx = tf.Context([pt], symmetric_state=True)
    X = ctx.empty(3)
    r, fl = timed_flow(ctx, X, tf.FlowOptions(T0=w.T0, Tmin=w.Tmin, Xmax=w.Xmax, scheme="dopri5",
                                              rtol=w.rtol, atol=w.atol))
    r = r[0]
    o = ctx.empty(3)
    Ts = [math.exp(math.log(10.0) + (math.log(1e-3) - math.log(10.0)) * i / 63) for i in range(64)]
    for i in range(20):
        ctx.rhs(Ts[i % 64], X, o)
    _sync()
    t0 = time.perf_counter()
    for i in range(steps):
        ctx.rhs(Ts[i % 64], X, o)
    _sync()
    el = time.perf_counter() - t0
    out = {"workload": w.name + "_symmetric_state", "rhs_per_s": steps / el, "ms_per_rhs": 1e3 * el / steps,
           "flow": {"flow_time_s": fl, "status": r.status, "Tc": r.Tc, "channel": r.channel,
                    "q_index": r.q_index, "irrep": r.irrep, "n_rhs": r.n_rhs, "n_steps": r.n_steps},
           "Tc_rel_vs_per_momentum": (abs(r.Tc / Tc_ref - 1) if (r.Tc and Tc_ref) else None)}
    w3 = synth.cfg3()
    p3 = w3.points[0]
    big = {"workload": w3.name}
    for prec in ("fp64", "mixed"):
        for sym in (False, True):
            c3 = tf.Context([p3], precision=prec, symmetric_state=sym)
            X3 = c3.empty(3).zero_()
            big[f"rhs_ms_{prec}_{'wedge' if sym else 'per_momentum'}"] = 1e3 * time_rhs(c3, 0.05, X3, c3.empty(3))
            c3.close()
            torch.cuda.empty_cache()
    out["large"] = big
    log(f"[wedge] rhs {out['ms_per_rhs']:.4f} ms, flow {fl:.3f} s: {out['flow']}; 48x48: {big}")
    return out


def leg_dense(tf, synth, steps):
    """The dense projection operator against the factored projections at small
    sizes (the precomputed-projection-data option of the paper): projection
    and right-hand side times, and the operator's size."""
    import torch
    out = {}
    for name, pt in (("q8_nff1", synth.Point(t=1.0, tp=0.0, U=3.0, Lq=8, Lk=32, shells=0, mu=0.0)),
                     ("q16_nff1", synth.Point(t=1.0, tp=0.0, U=3.0, Lq=16, Lk=64, shells=0, mu=0.0)),
                     ("q8_nff5", synth.cfg1().points[0])):
        X = torch.from_numpy(synth.random_channels(pt.nq, pt.nff, seed=5).reshape(3, -1)).cuda()
        row = {"N": 3 * pt.nq * pt.nff ** 2, "operator_MB": 8e-6 * (3 * pt.nq * pt.nff ** 2) ** 2}
        for form, dense in (("factored", False), ("dense", True)):
            ctx = tf.Context([pt], dense_projection=dense)
            o = ctx.empty(3)
            for _ in range(10):
                ctx.project(X, o)
            _sync()
            t0 = time.perf_counter()
            for _ in range(steps):
                ctx.project(X, o)
            _sync()
            row[f"project_us_{form}"] = 1e6 * (time.perf_counter() - t0) / steps
            row[f"rhs_us_{form}"] = 1e6 * time_rhs(ctx, 0.05, X, o, n=steps)
            ctx.close()
        out[name] = row
        log(f"[dense] {name}: {row}")
    return out


def leg_surrogate(tf, synth, train_steps):
    """cfg5: surrogate trained on 2M exact samples; flow with and without it."""
    import torch

    from paper_1604_06296_amd import surrogate as sur
    out = {}
    pts = synth.surrogate_training_points(64)
    temps = synth.surrogate_training_temperatures(64, 9)
    t0 = time.perf_counter()
    x, y = sur.make_training_set(pts, temps[:8], 262144, seed=500)
    xv, yv = sur.make_training_set(pts, temps[8:], 65536, seed=900)
    _sync()
    out["data_s"] = time.perf_counter() - t0
    out["train_samples"] = int(x.shape[0])
    nets = sur.train_ensemble(x, y, steps=train_steps, batch=4096, lr=2e-3)
    out["train_steps"] = train_steps
    out["train_s"] = [t for _, _, t in nets]
    out["final_loss"] = [float(h[-50:].mean()) for _, h, _ in nets]
    out["validation"] = [sur.validation_error(n, xv, yv) for n, _, _ in nets]
    log(f"[surrogate] data {out['data_s']:.2f} s, train {out['train_s']}, val {out['validation']}")
    del x, y, xv, yv
    w = synth.cfg5()
    pt = w.points[0]
    out["workload"] = w.name
    opts = tf.FlowOptions(T0=w.T0, Tmin=w.Tmin, Xmax=w.Xmax, scheme="rk4", nsteps=w.nsteps, use_graph=True)
    exact = tf.Context([pt], autotune=True)
    Xe = exact.empty(3)
    re, te = timed_flow(exact, Xe, opts)
    ctx = tf.Context([pt], autotune=True)
    ctx.attach_surrogate(nets[0][0], nets[1][0], tol=1e-3, check_stride=8)
    Xs = ctx.empty(3)
    rs, ts = timed_flow(ctx, Xs, opts)
    st = ctx.surrogate_stats()
    # one network (half the inference) at the same tolerance and at a looser one
    single = {}
    for tol in (1e-3, 2e-2):
        c1 = tf.Context([pt], autotune=True)
        c1.attach_surrogate(nets[0][0], None, tol=tol, check_stride=8)
        X1 = c1.empty(3)
        r1, t1 = timed_flow(c1, X1, opts)
        s1 = c1.surrogate_stats()
        single[f"tol_{tol:g}"] = {
            "flow_s": t1, "flow_speedup": te / t1, "exact_fraction": s1["exact_q"] / max(s1["queried_q"], 1),
            "failed_checks": s1["failed_checks"], "status": r1[0].status, "Tc": r1[0].Tc,
            "Tc_rel_err": (abs(r1[0].Tc / re[0].Tc - 1) if (re[0].Tc and r1[0].Tc) else None),
            "X_end_rel_err": float((X1 - Xe).abs().max() / Xe.abs().max())}
        log(f"[surrogate] one network, tol {tol:g}: {single[f'tol_{tol:g}']}")
        c1.close()
    out["single_network"] = single
    X = torch.from_numpy(synth.random_channels(pt.nq, pt.nff, seed=5).reshape(3, -1)).cuda()
    o = exact.empty(3)
    out.update({
        "flow_s_exact": te, "flow_s_surrogate": ts, "flow_speedup": te / ts,
        "rhs_ms_exact": 1e3 * time_rhs(exact, 0.05, X, o, n=20),
        "rhs_ms_surrogate": 1e3 * time_rhs(ctx, 0.05, X, o, n=20),
        "exact_fraction": st["exact_q"] / max(st["queried_q"], 1), "failed_checks": st["failed_checks"],
        "status": [re[0].status, rs[0].status], "Tc": [re[0].Tc, rs[0].Tc],
        "Tc_rel_err": (abs(rs[0].Tc / re[0].Tc - 1) if (re[0].Tc and rs[0].Tc) else None),
        "leading": [[re[0].channel, re[0].q_index, re[0].irrep], [rs[0].channel, rs[0].q_index, rs[0].irrep]],
        "max_abs_X": [re[0].max_abs_X, rs[0].max_abs_X],
        "X_end_rel_err": float((Xs - Xe).abs().max() / Xe.abs().max()),
    })
    log(f"[surrogate] flow exact {te:.3f} s, surrogate {ts:.3f} s, exact fraction {out['exact_fraction']:.3f}")
    return out


def main():
    args = parse()
    if args.probe_loops > 0 or args.probe_projections > 0 or args.probe_wedge > 0:
        if args.probe_wedge > 0:
            probe_wedge(args.probe_wedge)
        if args.probe_loops > 0:
            probe_loops(args.probe_loops)
        if args.probe_projections > 0:
            probe_projections(args.probe_projections)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(the right-hand side would shard over transfer momenta, with one all-reduce of the "
              "forward transform's partial sums per right-hand side)",
              file=sys.stderr)
        sys.exit(2)
    import synth

    # the oracle's baseline first, before the native library is loaded or
    # anything touches the GPU (its workers are fresh interpreters); the
    # oracle solves the workload's mu(n) itself
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(synth.cfg2().points[0], args.cpu_seconds)

    import torch

    import paper_1604_06296_amd as tf
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    w = synth.cfg2()
    pt = w.points[0]
    pt.mu = tf.mu_from_filling(pt.t, pt.tp, pt.filling, pt.mu_T, pt.mu_L)
    ctx = tf.Context([pt])          # default (deterministic) loop geometry
    nff = pt.nff
    X = torch.from_numpy(synth.random_channels(pt.nq, nff, seed=5, scale=1.0).reshape(3, -1)).cuda()
    out = ctx.empty(3)
    # temperatures spread over the flow range
    Ts = [math.exp(math.log(10.0) + (math.log(1e-3) - math.log(10.0)) * i / 63) for i in range(64)]
    log(f"[bench] workload {w.name}: Nq={pt.nq} Nk={pt.Lk ** 2} Nff={nff} mu={pt.mu:.6f} "
        f"loop geometry {ctx.geometry(0)}")

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

    # dominant kernel (the loop kernel): HIP events recorded by the library on
    # the context's stream around back-to-back launches of that kernel alone
    loop_us, loop_flops = ctx.loop_kernel_time(0.05, reps=max(args.steps, 20))
    alg_flops = loop_flops_algorithmic(pt.Lq, pt.Lk, ctx.harmonics(0)[0])
    achieved = alg_flops / (loop_us * 1e-6) / 1e12
    flops = ctx.flop_count()
    log(f"[bench] loop kernel {loop_us:.2f} us/launch, {achieved:.2f} TFLOP/s")
    traffic = LOOP_TRAFFIC["bytes"] if LOOP_TRAFFIC["sources_sha256"] == loop_kernel_sources_sha() else None
    # the projection kernels and the products, each alone (outside the timed region)
    kernels = kernel_table(ctx, 0.05, X, out, max(args.steps, 20), "fp64")
    log("[bench] kernels (us): " + ", ".join(f"{k} {v['us']:.2f}" for k, v in kernels.items()))

    flow_info = None
    if not args.no_flow:
        Xf = ctx.empty(3)
        fopts = tf.FlowOptions(T0=w.T0, Tmin=w.Tmin, Xmax=w.Xmax, scheme="dopri5", rtol=w.rtol, atol=w.atol)
        # the first flow of a context also allocates its flow buffers; the
        # second is the steady-state time
        _, fl_first = timed_flow(ctx, Xf, fopts)
        r, fl = timed_flow(ctx, Xf, fopts)
        r = r[0]
        flow_info = {"flow_time_s": fl, "first_flow_time_s": fl_first,
                     "rhs_time_share": r.n_rhs * ms * 1e-3 / fl, "status": r.status, "Tc": r.Tc, "channel": r.channel,
                     "q_index": r.q_index, "irrep": r.irrep, "n_rhs": r.n_rhs, "n_steps": r.n_steps}
        log(f"[bench] flow {fl:.3f} s: {flow_info}")

    legs = {}
    Tc_ref = flow_info["Tc"] if flow_info else None
    for name, skip, fn in (("omega", args.no_omega, lambda: leg_omega(tf, synth, args.steps)),
                           ("wedge", args.no_wedge, lambda: leg_wedge(tf, synth, args.steps, Tc_ref)),
                           ("dense", args.no_dense, lambda: leg_dense(tf, synth, args.steps)),
                           ("mixed", args.no_mixed, lambda: leg_mixed(tf, synth)),
                           ("batched", args.no_batched, lambda: leg_batched(tf, synth)),
                           ("surrogate", args.no_surrogate, lambda: leg_surrogate(tf, synth, args.train_steps))):
        if not skip:
            log(f"[bench] leg {name}")
            legs[name] = fn()
            torch.cuda.empty_cache()

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
                   "loop_geometry": list(ctx.geometry(0)),
                   "flow": flow_info, "flops_per_rhs": flops, "kernels": kernels, **legs},
        "roofline": {"bound": "alu", "kernel": "k_loops", "achieved": achieved,
                     "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                     "traffic": traffic, "launch_us": loop_us, "flops_per_launch": alg_flops,
                     "executed_flops_per_launch": loop_flops},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
