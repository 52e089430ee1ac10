"""C4v-symmetric states (TUFRG_SYMMETRIC_STATE) on the GPU against the FP64 CPU oracle.

With the flag, the inverse transform and the products run at one transfer
momentum per point-group orbit and the increments are copied to the other
members by the form factors' signed permutations (the covariance law pinned
in tests/test_oracle_symmetry.py).  Checked here:
  right-hand sides and projected vertices of symmetrised states against the
  oracle's full evaluation (FP64 normwise 1e-10, mixed 1e-5, both
  regulators, every truncation, ragged fine grids);
  at the full bench and 48x48 sizes against the library's own per-momentum
  path (bit-identical at the representatives, 1e-11 elsewhere);
  every orbit member an exact signed copy of its representative, for any
  input (the representatives themselves obey their stabilisers' part of the
  law up to rounding);
  flows started at zero with the oracle's critical scale and instability;
  a batch of uneven points against their single-point per-momentum results.
"""
import json
import os

import numpy as np
import pytest

import synth
from oracle import flow as oflow
from oracle import projections as oproj
from oracle import rhs as orhs
from oracle import symmetry as osym
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


def _to_dev(ctx, arrs, point=0, out=None):
    import torch
    if out is None:
        out = torch.zeros((3, ctx.S), dtype=torch.float64, device="cuda")
    ctx.view(out, point).copy_(torch.from_numpy(np.ascontiguousarray(arrs)))
    return out


def _host(ctx, dev, point=0):
    return ctx.view(dev, point).cpu().numpy()


def _assert_normwise(got, ref, tol=TOL, what=""):
    for c in range(ref.shape[0]):
        scale = np.abs(ref[c]).max()
        err = np.abs(got[c] - ref[c]).max()
        assert err <= tol * max(scale, 1e-300), f"{what} channel {c}: err {err:.3e} scale {scale:.3e}"


def _pt(shells, Lq, Lk, tp=-0.27, mu=-0.61, U=2.7):
    return synth.Point(t=1.0, tp=tp, U=U, Lq=Lq, Lk=Lk, shells=shells, mu=mu)


def _sym_state(pt, seed, scale=1.0):
    ff = FormFactors(pt.shells)
    X = synth.random_channels(pt.Lq * pt.Lq, ff.nff, seed=seed, scale=scale)
    return osym.symmetrize(X, ff, pt.Lq)


POINTS = [(0, 6, 12), (1, 8, 34), (2, 10, 16), (3, 10, 24), (4, 14, 40), (2, 12, 18), (1, 6, 14)]


@pytest.mark.parametrize("shells,Lq,Lk", POINTS)
@pytest.mark.parametrize("reg", ["T", "omega"])
def test_rhs_of_symmetric_state_matches_oracle(tf, shells, Lq, Lk, reg):
    pt = _pt(shells, Lq, Lk)
    ff = FormFactors(shells)
    Xs = _sym_state(pt, seed=7 + shells)
    T = 0.07 if reg == "T" else 0.3
    print(f"[wedge] rhs shells={shells} Lq={Lq} Lk={Lk} reg={reg}", flush=True)
    ctx = tf.Context([pt], regulator=reg, symmetric_state=True)
    got = _host(ctx, ctx.rhs(T, _to_dev(ctx, Xs)))
    ref = orhs.rhs(pt, T, Xs, ff, regulator=reg)
    _assert_normwise(got, ref, what="rhs")
    assert osym.defect(got, ff, Lq) <= 1e-13 * np.abs(got).max()
    _assert_orbit_copies(got, ff, Lq)


@pytest.mark.parametrize("shells,Lq,Lk", [(2, 10, 16), (4, 14, 40)])
def test_mixed_rhs_of_symmetric_state_matches_oracle(tf, shells, Lq, Lk):
    pt = _pt(shells, Lq, Lk)
    ff = FormFactors(shells)
    Xs = _sym_state(pt, seed=3)
    ctx = tf.Context([pt], precision="mixed", symmetric_state=True)
    got = _host(ctx, ctx.rhs(0.07, _to_dev(ctx, Xs)))
    ref = orhs.rhs(pt, 0.07, Xs, ff)
    _assert_normwise(got, ref, tol=1e-5, what="mixed rhs")   # the mixed form's RHS bound
    _assert_orbit_copies(got, ff, Lq)


@pytest.mark.parametrize("shells,Lq,Lk", [(1, 8, 16), (3, 10, 24), (2, 12, 18)])
def test_projection_of_symmetric_state_matches_oracle(tf, shells, Lq, Lk):
    pt = _pt(shells, Lq, Lk)
    ff = FormFactors(shells)
    Xs = _sym_state(pt, seed=5)
    ctx = tf.Context([pt], symmetric_state=True)
    got = _host(ctx, ctx.project(_to_dev(ctx, Xs)))
    ref = oproj.project(pt, Xs, ff)
    _assert_normwise(got, ref, what="V")


def _reps(Lq):
    return sorted({min(osym.image(Lq, h, q)[0] for h in osym.C4V_OPS) for q in range(Lq * Lq)})


def _assert_orbit_copies(Y, ff, Lq):
    """Every momentum holds T Y(r) T^T of its representative r exactly, for one of
    the operations that map it there."""
    laws = osym.law(ff, Lq)
    reps = set(_reps(Lq))
    for q in range(Lq * Lq):
        cands = [(q2, T) for row in laws for (q2, T) in [row[q]] if q2 in reps and q2 == min(
            osym.image(Lq, h, q)[0] for h in osym.C4V_OPS)]
        assert any(np.array_equal(Y[:, q], T @ Y[:, q2] @ T.T) for q2, T in cands), f"q={q}"


def test_output_is_copied_by_the_law_for_any_state(tf):
    """For a state that breaks the law the result is the representatives' increments
    copied by it, equal to the per-momentum path at the representatives."""
    pt = _pt(2, 10, 16)
    ff = FormFactors(2)
    X = synth.random_channels(100, ff.nff, seed=9)
    ctx = tf.Context([pt], symmetric_state=True)
    got = _host(ctx, ctx.rhs(0.1, _to_dev(ctx, X)))
    _assert_orbit_copies(got, ff, pt.Lq)
    full = tf.Context([pt])
    ref = _host(full, full.rhs(0.1, _to_dev(full, X)))
    reps = _reps(pt.Lq)
    np.testing.assert_array_equal(got[:, reps], ref[:, reps])


@pytest.mark.parametrize("which", ["cfg2", "cfg3"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_full_size_against_per_momentum_path(tf, which, precision):
    """Bench sizes: the same bits at the representatives, 1e-11 (mixed: 1e-5) elsewhere."""
    w = getattr(synth, which)()
    pt = w.points[0]
    if pt.mu is None:
        pt.mu = tf.mu_from_filling(pt.t, pt.tp, pt.filling, pt.mu_T, pt.mu_L)
    ff = FormFactors(pt.shells)
    Xs = _sym_state(pt, seed=21, scale=0.5)
    print(f"[wedge] full size {which} {precision}", flush=True)
    wedge = tf.Context([pt], precision=precision, symmetric_state=True)
    full = tf.Context([pt], precision=precision)
    a = _host(wedge, wedge.rhs(0.05, _to_dev(wedge, Xs)))
    b = _host(full, full.rhs(0.05, _to_dev(full, Xs)))
    reps = _reps(pt.Lq)
    np.testing.assert_array_equal(a[:, reps], b[:, reps])
    _assert_normwise(a, b, tol=1e-11 if precision == "fp64" else 1e-5, what=which)
    # the representatives obey their stabilisers' part of the law to the
    # precision's rounding; every other member is an exact copy
    assert osym.defect(a, ff, pt.Lq) <= (1e-13 if precision == "fp64" else 1e-6) * np.abs(a).max()
    _assert_orbit_copies(a, ff, pt.Lq)


def test_flow_cfg1_rk4_matches_oracle(tf):
    w = synth.cfg1()
    pt = w.points[0]
    ctx = tf.Context([pt], symmetric_state=True)
    X = ctx.empty(3).zero_()
    r = ctx.flow(X, tf.FlowOptions(T0=w.T0, Tmin=w.Tmin, Xmax=w.Xmax, scheme="rk4", nsteps=w.nsteps))[0]
    ref = oflow.flow_rk4(pt, w.T0, w.Tmin, w.nsteps, w.Xmax)
    print("gpu", r, "oracle", ref.Tc, ref.channel, ref.q_index, ref.irrep, flush=True)
    assert r.status == "diverged" and ref.status == oflow.STATUS_DIVERGED
    assert abs(r.Tc / ref.Tc - 1) < 1e-6
    assert (r.channel, r.q_index, r.irrep) == (ref.channel, ref.q_index, ref.irrep)
    _assert_normwise(_host(ctx, X), ref.X, tol=1e-8, what="X at stop")


@pytest.mark.parametrize("reg", ["T", "omega"])
def test_flow_cfg2_dopri5_against_oracle_golden(tf, reg):
    name = "flow_cfg2_dopri5_oracle.json" if reg == "T" else "flow_cfg2_omega_dopri5_oracle.json"
    with open(os.path.join(os.path.dirname(__file__), "golden", name)) as fh:
        ref = json.load(fh)
    w = synth.cfg2() if reg == "T" else synth.cfg2_omega()
    pt = w.points[0]
    pt.mu = tf.mu_from_filling(pt.t, pt.tp, pt.filling, pt.mu_T, pt.mu_L)
    print(f"[wedge] cfg2 dopri5 flow reg={reg}", flush=True)
    ctx = tf.Context([pt], regulator=reg, symmetric_state=True)
    X = ctx.empty(3).zero_()
    r = ctx.flow(X, tf.FlowOptions(T0=w.T0, Tmin=w.Tmin, Xmax=w.Xmax, scheme="dopri5",
                                   rtol=w.rtol, atol=w.atol))[0]
    print("gpu", r, flush=True)
    key = "Tc" if "Tc" in ref else "Omega_c"
    assert r.status == ref["status"] == "diverged"
    assert abs(r.Tc / ref[key] - 1) < 1e-3
    assert (r.channel, r.q_index, r.irrep) == (ref["channel"], ref["q_index"], ref["irrep"])


def test_batch_of_uneven_points(tf):
    pts = [_pt(1, 8, 16), _pt(3, 10, 24, tp=-0.1, mu=-0.3), _pt(2, 12, 18, tp=-0.35, mu=-1.1)]
    states = [_sym_state(p, seed=30 + i) for i, p in enumerate(pts)]
    ctx = tf.Context(pts, symmetric_state=True)
    import torch
    X = torch.zeros((3, ctx.S), dtype=torch.float64, device="cuda")
    for i, s in enumerate(states):
        _to_dev(ctx, s, point=i, out=X)
    out = ctx.rhs(0.08, X)
    for i, (p, s) in enumerate(zip(pts, states)):
        single = tf.Context([p])
        ref = _host(single, single.rhs(0.08, _to_dev(single, s)))
        _assert_normwise(_host(ctx, out, i), ref, tol=1e-11, what=f"point {i}")


def test_bubbles_entry_point_still_covers_every_momentum(tf):
    """The right-hand side expands the loops at the representatives only; the
    loops entry point still returns chi' of every momentum, bit for bit."""
    pt = _pt(3, 10, 24)
    a = tf.Context([pt], symmetric_state=True)
    b = tf.Context([pt])
    ga = _host(a, a.bubbles(0.09))
    gb = _host(b, b.bubbles(0.09))
    np.testing.assert_array_equal(ga, gb)


def _rep_of(Lq, q):
    return min(osym.image(Lq, h, q)[0] for h in osym.C4V_OPS)


def test_batched_rk4_flow_graph_and_eager(tf):
    """A batch of uneven points flowed from zero with symmetric states: the HIP-graph
    replay equals the eager flow bit for bit, and every point matches the
    per-momentum batch (critical scale 1e-8, same steps and channel, the ordering
    vector in the same orbit: members of an orbit are exact copies here, so the
    classification's first maximum may be another member)."""
    import torch
    pts = [_pt(1, 8, 16, tp=-0.1, mu=-0.2, U=3.0), _pt(2, 10, 20, tp=-0.3, mu=-1.0, U=2.5),
           _pt(3, 12, 24, tp=-0.2, mu=-0.6, U=2.8), _pt(0, 6, 12, tp=0.0, mu=0.0, U=3.2)]
    opts = lambda g: tf.FlowOptions(T0=10.0, Tmin=0.01, Xmax=20.0, scheme="rk4", nsteps=60, use_graph=g)
    print("[wedge] batched rk4 flow, graph vs eager", flush=True)
    ctx = tf.Context(pts, symmetric_state=True, loop_queue=True)
    Xa, Xb = ctx.empty(3).zero_(), ctx.empty(3).zero_()
    ra = ctx.flow(Xa, opts(False))
    rb = ctx.flow(Xb, opts(True))
    assert ra == rb and torch.equal(Xa, Xb)
    ref = tf.Context(pts, loop_queue=True)
    Xr = ref.empty(3).zero_()
    rr = ref.flow(Xr, opts(False))
    for i, (a, r) in enumerate(zip(ra, rr)):
        print(f"  pt{i}: {a.status} Tc={a.Tc} {a.channel} q={a.q_index} {a.irrep} / {r.Tc} q={r.q_index}",
              flush=True)
        assert a.status == r.status and a.n_steps == r.n_steps and a.channel == r.channel
        if a.status == "diverged":
            assert abs(a.Tc / r.Tc - 1) < 1e-8
            assert _rep_of(pts[i].Lq, a.q_index) == _rep_of(pts[i].Lq, r.q_index)
        _assert_normwise(_host(ctx, Xa, i), _host(ref, Xr, i), tol=1e-8, what=f"pt{i} X at stop")


def test_singleton_orbits_give_the_per_momentum_bits(tf):
    """With the point-group reduction off every momentum is its own representative:
    the symmetric-state path is then the per-momentum path, bit for bit."""
    pt = _pt(3, 10, 24)
    ff = FormFactors(3)
    X = synth.random_channels(100, ff.nff, seed=12)
    a = tf.Context([pt], no_symmetry=True, symmetric_state=True)
    b = tf.Context([pt], no_symmetry=True)
    np.testing.assert_array_equal(_host(a, a.rhs(0.06, _to_dev(a, X))), _host(b, b.rhs(0.06, _to_dev(b, X))))
    np.testing.assert_array_equal(_host(a, a.project(_to_dev(a, X))), _host(b, b.project(_to_dev(b, X))))


def test_mixed_precision_flow(tf):
    """Mixed precision along a whole RK4 flow from zero: the same outcome as the
    per-momentum mixed flow (critical scale within the mixed form's 1e-5)."""
    w = synth.cfg1()
    pt = w.points[0]
    opts = tf.FlowOptions(T0=w.T0, Tmin=w.Tmin, Xmax=w.Xmax, scheme="rk4", nsteps=w.nsteps)
    a = tf.Context([pt], precision="mixed", symmetric_state=True)
    b = tf.Context([pt], precision="mixed")
    ra = a.flow(a.empty(3).zero_(), opts)[0]
    rb = b.flow(b.empty(3).zero_(), opts)[0]
    print("wedge", ra, "per momentum", rb, flush=True)
    assert ra.status == rb.status == "diverged" and ra.n_steps == rb.n_steps
    assert abs(ra.Tc / rb.Tc - 1) < 1e-5
    assert ra.channel == rb.channel and ra.irrep == rb.irrep
    assert _rep_of(pt.Lq, ra.q_index) == _rep_of(pt.Lq, rb.q_index)


def test_symmetry_defect_detects_non_symmetric_states(tf):
    """tufrg_symmetry_defect: ~0 for a symmetrised state (and its flow
    increment), O(1) for a random state; a symmetric-state flow rejects a
    non-symmetric initial state with EINVAL instead of a silent answer."""
    import torch
    from paper_1604_06296_amd.binding import TufrgError
    pt = synth.Point(t=1.0, tp=-0.25, U=3.0, Lq=12, Lk=24, shells=3, mu=-0.8)
    ff = FormFactors(pt.shells)
    ctx = tf.Context([pt], symmetric_state=True)
    X = synth.random_channels(pt.nq, ff.nff, seed=41)
    Xs = osym.symmetrize(X, ff, pt.Lq)
    print("[wedge] symmetry defect", flush=True)
    assert ctx.symmetry_defect(_to_dev(ctx, X)) > 1e-2
    assert ctx.symmetry_defect(_to_dev(ctx, Xs)) <= 1e-14
    assert ctx.symmetry_defect(ctx.rhs(0.1, _to_dev(ctx, Xs))) <= 1e-12
    assert ctx.symmetry_defect(torch.zeros((3, ctx.S), dtype=torch.float64, device="cuda")) == 0.0
    opts = tf.FlowOptions(T0=10.0, Tmin=0.1, Xmax=20.0, scheme="rk4", nsteps=10)
    with pytest.raises(TufrgError, match="not C4v-symmetric"):
        ctx.flow(_to_dev(ctx, X), opts)
    r = ctx.flow(_to_dev(ctx, 1e-3 * Xs), opts)
    assert r[0].status in ("reached_tmin", "diverged")
