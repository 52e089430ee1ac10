"""Batched launches: many uneven points per launch, device-side stopping,
HIP-graph replay of the RK4 step, and the loop-geometry autotuner.

Every point of a batch must give its own single-point result (up to the
summation order of the px contraction, which follows the block size shared
by the batch: 1e-12 normwise), the oracle's result (1e-10 normwise), and the
graph-replayed flow must equal the eagerly launched one bit for bit.
"""
import os

import numpy as np
import pytest

import synth
from oracle import rhs as orhs
from oracle.lattice import FormFactors

pytestmark = pytest.mark.gpu
TOL = 1e-10


@pytest.fixture(scope="module")
def tf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1604_06296_amd as tf
    tf.load_library()
    return tf


def _torch():
    import torch
    return torch


def _normwise(got, ref, tol, what=""):
    for c in range(ref.shape[0]):
        scale = np.abs(ref[c]).max()
        err = np.abs(got[c] - ref[c]).max()
        assert err <= tol * max(scale, 1e-300), f"{what} channel {c}: err {err:.3e} scale {scale:.3e}"


def _pack(ctx, Xs):
    torch = _torch()
    Xd = torch.zeros((3, ctx.S), dtype=torch.float64, device="cuda")
    for i, X in enumerate(Xs):
        ctx.view(Xd, i).copy_(torch.from_numpy(np.ascontiguousarray(X)))
    return Xd


# uneven points: every truncation, ragged grids, different fillings and U
BATCH = [
    synth.Point(t=1.0, tp=-0.30, U=3.0, Lq=10, Lk=24, shells=4, mu=-0.9),
    synth.Point(t=1.0, tp=-0.10, U=2.2, Lq=6, Lk=12, shells=1, mu=-0.2),
    synth.Point(t=1.0, tp=0.00, U=3.4, Lq=8, Lk=20, shells=0, mu=0.0),
    synth.Point(t=1.0, tp=-0.25, U=2.8, Lq=12, Lk=36, shells=3, mu=-0.7),
    synth.Point(t=1.0, tp=-0.20, U=2.5, Lq=8, Lk=14, shells=2, mu=-0.4),
    synth.Point(t=1.0, tp=-0.15, U=3.8, Lq=6, Lk=32, shells=1, mu=-0.1),
]


def test_batch_rhs_matches_single_and_oracle(tf):
    print("[batch] rhs of 6 uneven points", flush=True)
    ctx = tf.Context(BATCH)
    Ts = [0.4, 0.05, 2.0, 0.011, 0.13, 0.9]
    Xs = [synth.random_channels(p.nq, FormFactors(p.shells).nff, seed=70 + i) for i, p in enumerate(BATCH)]
    Xd = _pack(ctx, Xs)
    d = ctx.rhs(Ts, Xd).cpu()
    V = ctx.project(Xd).cpu()
    b = ctx.bubbles(Ts).cpu()
    for i, p in enumerate(BATCH):
        ff = FormFactors(p.shells)
        ref, refV, refb = orhs.rhs(p, Ts[i], Xs[i], ff, return_parts=True)
        _normwise(ctx.view(d, i).numpy(), ref, TOL, f"pt{i} rhs")
        _normwise(ctx.view(V, i).numpy(), refV, TOL, f"pt{i} V")
        _normwise(ctx.view(b, i).numpy(), refb, TOL, f"pt{i} bubbles")
        one = tf.Context([p])
        Xo = _pack(one, [Xs[i]])
        _normwise(ctx.view(d, i).numpy(), one.view(one.rhs(Ts[i], Xo)).cpu().numpy(), 1e-12,
                  f"pt{i} batch vs single")
        one.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_loop_queue_form_identical(tf, precision):
    """Persistent work-queue launch and one block per item: the same bits."""
    print(f"[batch] loop launch forms, {precision}", flush=True)
    a = tf.Context(BATCH, precision=precision)
    b = tf.Context(BATCH, precision=precision, loop_queue=True)
    assert not a.geometry(0)[3] and b.geometry(0)[3]
    Ts = [0.4, 0.05, 2.0, 0.011, 0.13, 0.9]
    Xs = [synth.random_channels(p.nq, FormFactors(p.shells).nff, seed=80 + i) for i, p in enumerate(BATCH)]
    torch = _torch()
    for rep in range(3):        # the queue resets itself between launches
        assert torch.equal(a.bubbles(Ts), b.bubbles(Ts))
        assert torch.equal(a.rhs(Ts, _pack(a, Xs)), b.rhs(Ts, _pack(b, Xs)))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_fused_and_two_stream_forms_identical(tf, precision):
    """A small context runs the right-hand side in fused launches on one stream
    (loops with the forward transform, loop expansion with the bond basis);
    with fuse=False the loops run on a second stream beside the projection
    chain.  Same bits, for right-hand sides and for a graph-replayed RK4 flow."""
    print(f"[batch] fused vs two-stream, {precision}", flush=True)
    torch = _torch()
    a = tf.Context(BATCH, precision=precision)
    b = tf.Context(BATCH, precision=precision, fuse=False)
    assert a.S <= 1 << 18
    Ts = [0.4, 0.05, 2.0, 0.011, 0.13, 0.9]
    Xs = [synth.random_channels(p.nq, FormFactors(p.shells).nff, seed=90 + i) for i, p in enumerate(BATCH)]
    for rep in range(2):
        assert torch.equal(a.rhs(Ts, _pack(a, Xs)), b.rhs(Ts, _pack(b, Xs)))
    assert torch.equal(a.project(_pack(a, Xs)), b.project(_pack(b, Xs)))
    opts = tf.FlowOptions(T0=10.0, Tmin=0.05, Xmax=20.0, scheme="rk4", nsteps=30, use_graph=True)
    Xa, Xb = a.empty(3).zero_(), b.empty(3).zero_()
    ra, rb = a.flow(Xa, opts), b.flow(Xb, opts)
    assert ra == rb
    assert torch.equal(Xa, Xb)


def test_fused_form_with_more_points_than_passed_by_value(tf):
    """A small context of 70 points runs fused, but its temperatures (one per
    point) are more than the fused launch takes by value: they are stored by a
    separate launch first.  Same bits as the two-stream form, and every point
    keeps its own temperature."""
    print("[batch] fused, 70 points", flush=True)
    torch = _torch()
    pts = [synth.Point(t=1.0, tp=-0.05 * (i % 5), U=2.0 + 0.02 * i, Lq=6, Lk=12 + 4 * (i % 3), shells=i % 2,
                       mu=-0.1 * (i % 7)) for i in range(70)]
    a = tf.Context(pts)
    b = tf.Context(pts, fuse=False)
    assert a.S <= 1 << 18
    Ts = [0.05 + 0.01 * i for i in range(70)]
    Xs = [synth.random_channels(p.nq, FormFactors(p.shells).nff, seed=300 + i) for i, p in enumerate(pts)]
    ra = a.rhs(Ts, _pack(a, Xs))
    assert torch.equal(ra, b.rhs(Ts, _pack(b, Xs)))
    for i in (0, 37, 69):
        one = tf.Context([pts[i]])
        ref = one.view(one.rhs(Ts[i], _pack(one, [Xs[i]]))).cpu().numpy()
        _normwise(a.view(ra, i).cpu().numpy(), ref, 1e-12, f"pt{i} batch vs single")
        one.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_point_group_reduction_matches_full_grid(tf, precision):
    """Loops on one representative per C4v orbit equal the loops at every
    transfer momentum: 1e-12 normwise in FP64 (summation order only); in
    mixed precision the two sides round their FP32 sums independently, so
    twice the mixed loop bound of 2e-6."""
    torch = _torch()
    print(f"[batch] point-group reduction, {precision}", flush=True)
    full = tf.Context(BATCH, precision=precision, no_symmetry=True)
    red = tf.Context(BATCH, precision=precision)
    Ts = [0.4, 0.05, 2.0, 0.011, 0.13, 0.9]
    a, b = full.bubbles(Ts).cpu().numpy(), red.bubbles(Ts).cpu().numpy()
    tol = 1e-12 if precision == "fp64" else 4e-6
    for i in range(len(BATCH)):
        _normwise(red.view(torch.from_numpy(b), i).numpy(), full.view(torch.from_numpy(a), i).numpy(), tol,
                  f"pt{i}")


def _flow_opts(tf, graph, nsteps=80):
    return tf.FlowOptions(T0=10.0, Tmin=0.01, Xmax=20.0, scheme="rk4", nsteps=nsteps, use_graph=graph)


def test_batch_flow_stops_each_point(tf):
    """Batched RK4: each point stops at its own step, as in its own flow."""
    print("[batch] rk4 flow of 6 points, eager", flush=True)
    ctx = tf.Context(BATCH)
    X = ctx.empty(3).zero_()
    res = ctx.flow(X, _flow_opts(tf, False))
    Xh = X.cpu()
    steps = set()
    for i, p in enumerate(BATCH):
        one = tf.Context([p])
        Xo = one.empty(3).zero_()
        r1 = one.flow(Xo, _flow_opts(tf, False))[0]
        r = res[i]
        print(f"  pt{i}: {r.status} Tc={r.Tc} {r.channel} q={r.q_index} {r.irrep} steps={r.n_steps}",
              flush=True)
        assert r.status == r1.status and r.n_steps == r1.n_steps and r.n_rhs == 4 * r.n_steps
        assert (r.channel, r.q_index, r.irrep) == (r1.channel, r1.q_index, r1.irrep)
        if r.status == "diverged":
            assert abs(r.Tc / r1.Tc - 1) < 1e-8
        _normwise(ctx.view(Xh, i).numpy(), one.view(Xo).cpu().numpy(), 1e-8, f"pt{i} X at stop")
        steps.add(r.n_steps)
        one.close()
    assert len(steps) > 1, "the batch should stop its points at different steps"


def test_graph_replay_equals_eager(tf):
    print("[batch] rk4 flow: graph replay vs eager", flush=True)
    ctx = tf.Context(BATCH, loop_queue=True)
    Xa = ctx.empty(3).zero_()
    Xb = ctx.empty(3).zero_()
    ra = ctx.flow(Xa, _flow_opts(tf, False))
    rb = ctx.flow(Xb, _flow_opts(tf, True))
    assert ra == rb
    assert _torch().equal(Xa, Xb)
    # a second replay set on the same context (state reset) is identical too
    Xc = ctx.empty(3).zero_()
    assert ctx.flow(Xc, _flow_opts(tf, True)) == ra and _torch().equal(Xa, Xc)


def test_graph_reached_tmin(tf):
    """No point diverges: every step runs and the graph path reports REACHED_TMIN."""
    pts = [synth.Point(t=1.0, tp=-0.1, U=0.5, Lq=6, Lk=12, shells=1, mu=-0.3),
           synth.Point(t=1.0, tp=-0.2, U=0.4, Lq=8, Lk=16, shells=0, mu=-0.5)]
    ctx = tf.Context(pts)
    X = ctx.empty(3).zero_()
    res = ctx.flow(X, tf.FlowOptions(T0=10.0, Tmin=0.5, Xmax=20.0, scheme="rk4", nsteps=12,
                                     use_graph=True))
    assert all(r.status == "reached_tmin" and r.n_steps == 12 and r.n_rhs == 48 for r in res)


def test_autotune_geometry_and_cache(tf, tmp_path):
    cache = tmp_path / "tune.txt"
    os.environ["TUFRG_TUNE_CACHE"] = str(cache)
    try:
        pts = BATCH[:4]
        print("[autotune] 4 points", flush=True)
        tuned = tf.Context(pts, autotune=True)
        plain = tf.Context(pts)
        lines = cache.read_text().split()
        # one line per distinct point shape, and one for the batch's row-slice factor
        assert len(lines) == 3 * (len({(p.nq, p.Lk, FormFactors(p.shells).nff) for p in pts}) + 1)
        assert sum(1 for w in lines if w.startswith("batch_")) == 1
        for i, p in enumerate(pts):
            ns, nc, th, _ = tuned.geometry(i)
            assert ns >= 1 and nc >= 1 and p.Lk * nc <= th <= 512
        Ts = [0.3, 0.02, 1.0, 0.07]
        Xs = [synth.random_channels(p.nq, FormFactors(p.shells).nff, seed=90 + i) for i, p in enumerate(pts)]
        a = tuned.rhs(Ts, _pack(tuned, Xs)).cpu()
        b = plain.rhs(Ts, _pack(plain, Xs)).cpu()
        for i in range(len(pts)):
            _normwise(tuned.view(a, i).numpy(), plain.view(b, i).numpy(), 1e-12, f"pt{i} tuned")
        # the cache is read back: same choices, nothing appended
        again = tf.Context(pts, autotune=True)
        assert [again.geometry(i) for i in range(4)] == [tuned.geometry(i) for i in range(4)]
        assert cache.read_text().split() == lines
    finally:
        del os.environ["TUFRG_TUNE_CACHE"]


def test_cfg4_full_batch_sampled(tf):
    """The 64-point sweep in one context: sampled points and momenta against the oracle."""
    w = synth.cfg4()
    for p in w.points:
        p.mu = tf.mu_from_filling(p.t, p.tp, p.filling, p.mu_T, p.mu_L)
    print("[cfg4] 64 points, S =", end=" ", flush=True)
    ctx = tf.Context(w.points)
    print(ctx.S, flush=True)
    rng = np.random.default_rng(4404)
    Ts = list(np.exp(rng.uniform(np.log(0.01), np.log(10.0), len(w.points))))
    Xs = [synth.random_channels(p.nq, FormFactors(p.shells).nff, seed=400 + i) for i, p in enumerate(w.points)]
    d = ctx.rhs(Ts, _pack(ctx, Xs)).cpu()
    for i in (0, 17, 63) + tuple(int(k) for k in rng.choice(64, 2, replace=False)):
        p = w.points[i]
        ff = FormFactors(p.shells)
        qi = list(synth.sample_indices(p.nq, 3, seed=i)) + [p.nq - 1]
        ref = orhs.rhs(p, Ts[i], Xs[i], ff, q_index=qi)
        _normwise(ctx.view(d, i).numpy()[:, qi], ref, TOL, f"cfg4 pt{i} (Nff={ff.nff}, Lq={p.Lq})")


def test_batched_dopri5_equals_single_point_flows(tf):
    """The adaptive flow of a batch of uneven points (each with its own step
    size and stop on the device) gives every point its single-point flow:
    same status and instability, critical scale and state within the flow's
    tolerances (the batch sums the loops in the batch's block order, so the
    step sequence may differ by rounding); graph-replayed = eager bit for bit."""
    import torch
    pts = BATCH[:4]
    print("[batch] dopri5 batch vs single points", flush=True)
    opts = dict(T0=10.0, Tmin=0.01, Xmax=20.0, scheme="dopri5", rtol=1e-7, atol=1e-9)
    ctx = tf.Context(pts)
    Xg, Xe = ctx.empty(3).zero_(), ctx.empty(3).zero_()
    rg = ctx.flow(Xg, tf.FlowOptions(use_graph=True, **opts))
    re = ctx.flow(Xe, tf.FlowOptions(use_graph=False, **opts))
    assert rg == re and torch.equal(Xg, Xe)
    for i, p in enumerate(pts):
        one = tf.Context([p])
        X1 = one.empty(3).zero_()
        r1 = one.flow(X1, tf.FlowOptions(**opts))[0]
        a = rg[i]
        assert (a.status, a.channel, a.q_index, a.irrep) == (r1.status, r1.channel, r1.q_index, r1.irrep), (i, a, r1)
        assert abs(a.n_steps - r1.n_steps) <= 1, (i, a, r1)
        if r1.Tc:
            assert abs(a.Tc / r1.Tc - 1) < 1e-5
        _normwise(ctx.view(Xg, i).cpu().numpy(), one.view(X1).cpu().numpy(), 1e-5, f"point {i}")


def test_dopri5_step_budget_and_step_sign(tf):
    """A flow that uses up max_steps says so; a first step pointing away from
    Tmin is rejected."""
    from paper_1604_06296_amd.binding import TufrgError
    ctx = tf.Context([BATCH[1]])
    r = ctx.flow(ctx.empty(3).zero_(), tf.FlowOptions(T0=10.0, Tmin=0.01, Xmax=20.0, scheme="dopri5",
                                                      rtol=1e-7, atol=1e-9, max_steps=3))[0]
    assert r.status == "max_steps" and r.n_steps <= 3 and r.n_rhs == 1 + 6 * 3
    with pytest.raises(TufrgError, match="h0"):
        ctx.flow(ctx.empty(3).zero_(), tf.FlowOptions(T0=10.0, Tmin=0.01, Xmax=20.0, scheme="dopri5",
                                                      rtol=1e-7, atol=1e-9, h0=0.05))
