"""The Omega-cutoff regulator at zero temperature (named in Sec. 3; start and stop
values of Sec. 4) on the GPU
against the FP64 CPU oracle.

Only the loops change with the regulator; every entry point is compared:
  loops and right-hand sides (FP64) normwise within 1e-10, as for the
  temperature flow; mixed precision within the same 2e-6 loop bound (FP32
  rational pair function, compensated sums); flows with the same critical
  scale and leading instability as the oracle's; the launch forms with the
  same bits.
"""
import json
import os

import numpy as np
import pytest

import synth
from oracle import bubbles as obub
from oracle import flow as oflow
from oracle import rhs as orhs
from oracle.lattice import FormFactors, mu_from_filling

pytestmark = pytest.mark.gpu
TOL = 1e-10
OMEGAS = (800.0, 3.0, 0.21, 0.013, 1.1e-3)


@pytest.fixture(scope="module")
def tf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1604_06296_amd as tf
    tf.load_library()
    return tf


def _to_dev(ctx, arrs, point=0, nch=3):
    import torch
    out = torch.zeros((nch, ctx.S), dtype=torch.float64, device="cuda")
    ctx.view(out, point).copy_(torch.from_numpy(np.ascontiguousarray(arrs)))
    return out


def _host(ctx, dev, point=0):
    return ctx.view(dev, point).cpu().numpy()


def _assert_normwise(got, ref, tol=TOL, what=""):
    for c in range(ref.shape[0]):
        scale = np.abs(ref[c]).max()
        err = np.abs(got[c] - ref[c]).max()
        assert err <= tol * max(scale, 1e-300), f"{what} channel {c}: err {err:.3e} scale {scale:.3e}"


POINTS = [(0, 6, 12), (1, 8, 34), (2, 10, 16), (3, 10, 24), (4, 14, 40)]


def _pt(shells, Lq, Lk, tp=-0.27, mu=-0.61, U=2.7):
    return synth.Point(t=1.0, tp=tp, U=U, Lq=Lq, Lk=Lk, shells=shells, mu=mu)


@pytest.mark.parametrize("shells,Lq,Lk", POINTS)
def test_omega_bubbles_small(tf, shells, Lq, Lk):
    pt = _pt(shells, Lq, Lk)
    print(f"[omega bubbles] shells={shells} Lq={Lq} Lk={Lk}", flush=True)
    ctx = tf.Context([pt], regulator="omega")
    for Om in OMEGAS:
        ref = obub.bubbles(pt, Om, "dot", regulator="omega")
        _assert_normwise(_host(ctx, ctx.bubbles(Om)), ref, what=f"bubbles Om={Om}")


@pytest.mark.parametrize("shells,Lq,Lk", POINTS[1:4])
def test_omega_rhs_small(tf, shells, Lq, Lk):
    pt = _pt(shells, Lq, Lk)
    print(f"[omega rhs] shells={shells} Lq={Lq} Lk={Lk}", flush=True)
    ff = FormFactors(shells)
    ctx = tf.Context([pt], regulator="omega")
    X = synth.random_channels(pt.nq, ff.nff, seed=31 + shells, scale=1.5)
    for Om in (2.0, 0.05):
        ref = orhs.rhs(pt, Om, X, ff, regulator="omega")
        _assert_normwise(_host(ctx, ctx.rhs(Om, _to_dev(ctx, X))), ref, what=f"rhs Om={Om}")


def test_omega_cfg2_full(tf):
    """The benchmark workload (N_ff = 13, 24x24 / 96x96) with the Omega cutoff, in full."""
    print("[omega] cfg2 full", flush=True)
    pt = synth.cfg2_omega().points[0]
    pt.mu = tf.mu_from_filling(pt.t, pt.tp, pt.filling, pt.mu_T, pt.mu_L)
    ff = FormFactors(pt.shells)
    ctx = tf.Context([pt], regulator="omega")
    X = synth.random_channels(pt.nq, ff.nff, seed=12, scale=1.5)
    Om = 0.037
    ref_rhs, _, ref_chi = orhs.rhs(pt, Om, X, ff, return_parts=True, regulator="omega")
    Xd = _to_dev(ctx, X)
    _assert_normwise(_host(ctx, ctx.bubbles(Om)), ref_chi, what="cfg2 omega bubbles")
    _assert_normwise(_host(ctx, ctx.rhs(Om, Xd)), ref_rhs, what="cfg2 omega rhs")


@pytest.mark.parametrize("which", ["cfg3", "cfg5"])
def test_omega_full_size_sampled(tf, which):
    """N_ff = 21 at 48x48/128x128 and 64x64/160x160 with the Omega cutoff: loops and
    right-hand sides on sampled momenta."""
    w = synth.cfg3() if which == "cfg3" else synth.cfg5()
    pt = w.points[0]
    print(f"[omega] {which} sampled", flush=True)
    ff = FormFactors(pt.shells)
    ctx = tf.Context([pt], regulator="omega")
    X = synth.random_channels(pt.nq, ff.nff, seed=14, scale=1.0)
    qi = list(synth.sample_indices(pt.nq, 4, seed=19)) + [0, pt.nq - 1]
    Om = 0.023
    ref_rhs, _, ref_chi = orhs.rhs(pt, Om, X, ff, return_parts=True, q_index=qi, regulator="omega")
    Xd = _to_dev(ctx, X)
    _assert_normwise(_host(ctx, ctx.bubbles(Om))[:, qi], ref_chi, what=f"{which} omega bubbles")
    _assert_normwise(_host(ctx, ctx.rhs(Om, Xd))[:, qi], ref_rhs, what=f"{which} omega rhs")


def test_omega_multi_point_and_full_grid(tf):
    """Uneven points in one context, and the point-group reduction off: same results."""
    pts = [_pt(1, 8, 20), _pt(3, 10, 24, tp=-0.1, mu=-0.3), _pt(0, 6, 12, tp=0.0, mu=0.0)]
    print("[omega] multi-point", flush=True)
    ctx = tf.Context(pts, regulator="omega")
    full = tf.Context(pts, regulator="omega", no_symmetry=True)
    Oms = [0.4, 0.02, 5.0]
    d, f = ctx.bubbles(Oms).cpu(), full.bubbles(Oms).cpu()
    for i, pt in enumerate(pts):
        ref = obub.bubbles(pt, Oms[i], "dot", regulator="omega")
        _assert_normwise(ctx.view(d, i).numpy(), ref, what=f"pt{i}")
        _assert_normwise(full.view(f, i).numpy(), ref, what=f"pt{i} full grid")


@pytest.mark.parametrize("shells,Lq,Lk", [(4, 10, 22), (1, 8, 32), (3, 24, 96)])
def test_omega_mixed_loops(tf, shells, Lq, Lk):
    pt = _pt(shells, Lq, Lk, tp=-0.25, mu=-0.9)
    print(f"[omega mixed] shells={shells} Lq={Lq} Lk={Lk}", flush=True)
    ctx = tf.Context([pt], precision="mixed", regulator="omega")
    for Om in (2.0, 0.05, 2e-3):
        ref = obub.bubbles(pt, Om, "dot", regulator="omega")
        _assert_normwise(_host(ctx, ctx.bubbles(Om)), ref, tol=2e-6, what=f"mixed Om={Om}")


def test_omega_launch_forms_identical(tf):
    """Fused and two-stream right-hand sides, the loop queue, and graph-replayed
    and eager flows give the same bits with the Omega cutoff."""
    import torch
    pts = [_pt(1, 8, 20), _pt(3, 10, 24, tp=-0.1, mu=-0.3)]
    print("[omega] launch forms", flush=True)
    a = tf.Context(pts, regulator="omega")
    b = tf.Context(pts, regulator="omega", fuse=False)
    c = tf.Context(pts, regulator="omega", loop_queue=True)
    Xs = [synth.random_channels(p.nq, FormFactors(p.shells).nff, seed=50 + i) for i, p in enumerate(pts)]

    def pack(ctx):
        Xd = torch.zeros((3, ctx.S), dtype=torch.float64, device="cuda")
        for i, X in enumerate(Xs):
            ctx.view(Xd, i).copy_(torch.from_numpy(np.ascontiguousarray(X)))
        return Xd

    Oms = [0.3, 0.04]
    ra = a.rhs(Oms, pack(a))
    assert torch.equal(ra, b.rhs(Oms, pack(b)))
    assert torch.equal(ra, c.rhs(Oms, pack(c)))
    res = []
    for ctx, graph in ((a, True), (a, False), (b, True)):
        X = ctx.empty(3).zero_()
        r = ctx.flow(X, tf.FlowOptions(T0=100.0, Tmin=0.05, Xmax=20.0, scheme="rk4", nsteps=40,
                                       use_graph=graph))
        res.append((r, X.clone()))
    assert res[0][0] == res[1][0] == res[2][0]
    assert torch.equal(res[0][1], res[1][1]) and torch.equal(res[0][1], res[2][1])


def test_omega_flow_small_dopri5(tf):
    """Half filling, t' = 0: adaptive Omega flow against the oracle's (critical
    scale within 1e-3, same channel, momentum and irrep)."""
    pt = _pt(1, 6, 16, tp=0.0, mu=0.0, U=3.0)
    print("[omega] small dopri5 flow", flush=True)
    ctx = tf.Context([pt], regulator="omega")
    X = ctx.empty(3).zero_()
    r = ctx.flow(X, tf.FlowOptions(T0=800.0, Tmin=1e-3, Xmax=80.0, scheme="dopri5", rtol=1e-7,
                                   atol=1e-9))[0]
    ref = oflow.flow_dopri5(pt, 800.0, 1e-3, 80.0, rtol=1e-7, atol=1e-9, regulator="omega")
    print("gpu", r, "oracle", ref.Tc, ref.channel, ref.q_index, ref.irrep, flush=True)
    assert r.status == "diverged" and ref.status == oflow.STATUS_DIVERGED
    assert abs(r.Tc / ref.Tc - 1) < 1e-3
    assert (r.channel, r.q_index, r.irrep) == (ref.channel, ref.q_index, ref.irrep)


def test_omega_flow_no_cross_is_rpa(tf):
    """Decoupled Omega flow = RPA ladder of the oracle's Omega-regulated loop values."""
    pt = _pt(0, 6, 16, tp=-0.1, mu=-0.2, U=2.0)
    print("[omega] decoupled flow", flush=True)
    ctx = tf.Context([pt], no_cross=True, regulator="omega")
    X = ctx.empty(3).zero_()
    r = ctx.flow(X, tf.FlowOptions(T0=50.0, Tmin=0.2, Xmax=1e9, scheme="rk4", nsteps=200))[0]
    assert r.status == "reached_tmin"
    b0 = obub.bubbles(pt, 50.0, "value", regulator="omega")
    b1 = obub.bubbles(pt, 0.2, "value", regulator="omega")
    dph = b1[1, :, 0, 0] - b0[1, :, 0, 0]
    dpp = b1[0, :, 0, 0] - b0[0, :, 0, 0]
    Xh = _host(ctx, X)
    np.testing.assert_allclose(2.0 + Xh[1, :, 0, 0], 2.0 / (1 + 2.0 * dph), rtol=2e-8)
    np.testing.assert_allclose(2.0 - Xh[0, :, 0, 0], 2.0 / (1 + 2.0 * dpp), rtol=2e-8)


def test_omega_flow_cfg2_against_oracle_golden(tf):
    """The benchmark point flowed with the Omega cutoff (Omega 800 -> 1e-3, stop at
    max|X| > 80): critical Omega within 1e-3 of the oracle's (stored by
    tests/golden/make_flow_cfg2_omega.py) and the same leading instability."""
    with open(os.path.join(os.path.dirname(__file__), "golden", "flow_cfg2_omega_dopri5_oracle.json")) as fh:
        ref = json.load(fh)
    w = synth.cfg2_omega()
    pt = w.points[0]
    pt.mu = tf.mu_from_filling(pt.t, pt.tp, pt.filling, pt.mu_T, pt.mu_L)
    assert abs(pt.mu - ref["point"]["mu"]) < 1e-12
    print(f"[omega] cfg2 dopri5 vs oracle golden Omega_c={ref['Omega_c']}", flush=True)
    ctx = tf.Context([pt], regulator="omega")
    X = ctx.empty(3).zero_()
    r = ctx.flow(X, tf.FlowOptions(T0=w.T0, Tmin=w.Tmin, Xmax=w.Xmax, scheme="dopri5",
                                   rtol=w.rtol, atol=w.atol))[0]
    print("gpu", r, flush=True)
    assert r.status == ref["status"] == "diverged"
    assert abs(r.Tc / ref["Omega_c"] - 1) < 1e-3
    assert (r.channel, r.q_index, r.irrep) == (ref["channel"], ref["q_index"], ref["irrep"])


def test_omega_surrogate_rejected(tf):
    pt = _pt(1, 6, 12)
    ctx = tf.Context([pt], regulator="omega")
    a, b = tf.MLP([9, 16, 4], max_rows=64), tf.MLP([9, 16, 4], max_rows=64, seed=1)
    with pytest.raises(tf.TufrgError, match="EUNSUPPORTED"):
        ctx.attach_surrogate(a, b, tol=1e-3)
