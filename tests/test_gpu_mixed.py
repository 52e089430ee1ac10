"""Mixed precision (FP32 loops with compensated sums, BF16-split MFMA transforms,
FP32 products, FP64 ODE state) against the FP64 CPU oracle.

Bounds (normwise per channel, derived from the arithmetic):
  loops        2e-6: FP32 pair math (unit roundoff 6e-8, amplified <= ~4x by
               the divided differences and the FP32 rounding of eps/T-scaled
               exponents), blocked Neumaier-compensated row sums;
  projections  1e-5: operands split into two BF16 terms (about 2^-17 relative
               residual each), three MFMA passes, FP32 accumulation over the
               transfer grid;
  rhs          1e-5: projections and loops above, products in FP32.
"""
import numpy as np
import pytest

import synth
from oracle import bubbles as obub
from oracle import flow as oflow
from oracle import projections as oproj
from oracle import rhs as orhs
from oracle.lattice import FormFactors

pytestmark = pytest.mark.gpu
TOL_LOOPS, TOL_PROJ, TOL_RHS = 2e-6, 1e-5, 1e-5


@pytest.fixture(scope="module")
def tf():
    import torch
    assert torch.cuda.is_available()
    import paper_1604_06296_amd as tf
    return tf


def _nw(got, ref):
    return max(np.abs(got[c] - ref[c]).max() / np.abs(ref[c]).max() for c in range(ref.shape[0]))


def _dev(ctx, X):
    import torch
    out = torch.zeros((3, ctx.S), dtype=torch.float64, device="cuda")
    ctx.view(out).copy_(torch.from_numpy(X))
    return out


CASES = [
    (synth.Point(t=1.0, tp=-0.27, U=2.7, Lq=10, Lk=22, shells=4, mu=-0.61), None),
    (synth.Point(t=1.0, tp=0.0, U=3.0, Lq=8, Lk=32, shells=1, mu=0.0), None),
    (synth.Point(t=1.0, tp=-0.2, U=3.0, Lq=6, Lk=12, shells=0, mu=-0.4), None),
    (synth.Point(t=1.0, tp=-0.25, U=3.0, Lq=24, Lk=96, shells=3, mu=-0.9000355875840214), None),
    # the mixed-precision workload at full size, sampled momenta
    ("cfg3", [0, 47, 777, 1200, 2303]),
]


def _case(c):
    pt, qi = c
    if pt == "cfg3":
        pt = synth.cfg3().points[0]
    return pt, qi


@pytest.mark.parametrize("case", range(len(CASES)))
def test_mixed_loops_projections_rhs(tf, case):
    pt, qi = _case(CASES[case])
    ff = FormFactors(pt.shells)
    print(f"[mixed] Lq={pt.Lq} Lk={pt.Lk} nff={ff.nff}", flush=True)
    ctx = tf.Context([pt], precision="mixed")
    X = synth.random_channels(pt.nq, ff.nff, seed=3 + case, scale=1.0)
    Xd = _dev(ctx, X)
    sel = (lambda a: a) if qi is None else (lambda a: a[:, qi])
    for T in (5.0, 0.2, 0.02, 0.002):
        e = _nw(sel(ctx.view(ctx.bubbles(T)).cpu().numpy()), obub.bubbles(pt, T, "dot", ff, q_index=qi))
        print(f"  loops T={T}: {e:.2e}", flush=True)
        assert e <= TOL_LOOPS
    e = _nw(sel(ctx.view(ctx.project(Xd)).cpu().numpy()), oproj.project(pt, X, ff, l_index=qi))
    print(f"  projections: {e:.2e}", flush=True)
    assert e <= TOL_PROJ
    for T in (0.2, 0.02):
        e = _nw(sel(ctx.view(ctx.rhs(T, Xd)).cpu().numpy()), orhs.rhs(pt, T, X, ff, q_index=qi))
        print(f"  rhs T={T}: {e:.2e}", flush=True)
        assert e <= TOL_RHS


def test_mixed_no_cross(tf):
    pt = synth.small_point(Lq=8, Lk=16, shells=2)
    ff = FormFactors(2)
    ctx = tf.Context([pt], precision="mixed", no_cross=True)
    X = synth.random_channels(pt.nq, ff.nff, seed=5)
    Xd = _dev(ctx, X)
    assert _nw(ctx.view(ctx.project(Xd)).cpu().numpy(), oproj.project(pt, X, ff, no_cross=True)) < 1e-6
    assert _nw(ctx.view(ctx.rhs(0.1, Xd)).cpu().numpy(), orhs.rhs(pt, 0.1, X, ff, no_cross=True)) < TOL_RHS


def test_mixed_flow_matches_oracle_flow(tf):
    """Flow with an FP64 state and mixed-precision increments: critical scale
    within 1% of the FP64 oracle flow, same leading instability."""
    w = synth.cfg1()
    pt = w.points[0]
    ctx = tf.Context([pt], precision="mixed")
    X = ctx.empty(3).zero_()
    r = ctx.flow(X, tf.FlowOptions(T0=w.T0, Tmin=w.Tmin, Xmax=w.Xmax, scheme="rk4", nsteps=w.nsteps))[0]
    ref = oflow.flow_rk4(pt, w.T0, w.Tmin, w.nsteps, w.Xmax)
    print(f"mixed Tc {r.Tc} oracle {ref.Tc} rel {abs(r.Tc / ref.Tc - 1):.2e}", flush=True)
    assert r.status == "diverged"
    assert abs(r.Tc / ref.Tc - 1) < 0.01
    assert (r.channel, r.q_index, r.irrep) == (ref.channel, ref.q_index, ref.irrep)


def test_mixed_flow_full_size_against_fp64_gpu(tf):
    """The mixed-precision workload (N_ff = 21, 48x48, 128x128): critical scale
    within 1% of the FP64 path (itself oracle-checked) and same instability."""
    w = synth.cfg3()
    pt = w.points[0]
    res = {}
    for prec in ("fp64", "mixed"):
        ctx = tf.Context([pt], precision=prec)
        X = ctx.empty(3).zero_()
        res[prec] = ctx.flow(X, tf.FlowOptions(T0=w.T0, Tmin=w.Tmin, Xmax=w.Xmax, scheme="rk4",
                                                nsteps=w.nsteps))[0]
        print(prec, res[prec], flush=True)
    a, b = res["fp64"], res["mixed"]
    assert a.status == b.status
    if a.status == "diverged":
        assert abs(b.Tc / a.Tc - 1) < 0.01
        assert (a.channel, a.q_index, a.irrep) == (b.channel, b.q_index, b.irrep)
