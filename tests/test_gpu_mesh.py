"""Non-uniform transfer meshes (Sec. 4: the exchange propagators on an
adaptively dense set of momenta) on the GPU against the FP64 CPU oracle.

The meshes refine the uniform grid by 3 x 3 around q = 0 and (pi, pi) (the
regions where the pairing and magnetic propagators peak), so the momenta are
genuinely non-uniform with two cell sizes; the oracle's mesh path is pinned
in tests/test_oracle_mesh.py.  FP64 parity is normwise 1e-10 per channel,
mixed precision 1e-5.
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
CENTERS = [(0.0, 0.0), (np.pi, np.pi)]


@pytest.fixture(scope="module")
def tf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1604_06296_amd as tf
    tf.load_library()
    return tf


def _point(Lq, Lk, shells, radius, **kw):
    p = synth.Point(t=1.0, tp=kw.get("tp", -0.25), U=kw.get("U", 3.0), Lq=Lq, Lk=Lk, shells=shells,
                    mu=kw.get("mu", -0.8))
    p.mesh = synth.refined_mesh(Lq, 3, CENTERS, radius)
    return p


def _dev(X):
    import torch
    return torch.from_numpy(np.ascontiguousarray(X.reshape(X.shape[0], -1))).cuda()


def _normwise(got, ref, tol, what=""):
    for c in range(ref.shape[0]):
        scale = np.abs(ref[c]).max()
        err = np.abs(got[c] - ref[c]).max()
        assert err <= tol * max(scale, 1e-300), f"{what} channel {c}: err {err:.3e} scale {scale:.3e}"


@pytest.mark.parametrize("shells,Lq,Lk", [(0, 6, 16), (1, 8, 20), (2, 8, 24), (3, 10, 22), (4, 10, 24)])
def test_mesh_rhs_loops_projections_match_oracle(tf, shells, Lq, Lk):
    pt = _point(Lq, Lk, shells, radius=1)
    ff = FormFactors(shells)
    print(f"[mesh] shells={shells} Lq={Lq} Lk={Lk} nq={pt.nq}", flush=True)
    ctx = tf.Context([pt])
    assert ctx.layouts[0][1] == pt.nq
    X = synth.random_channels(pt.nq, ff.nff, seed=60 + shells)
    T = 0.07
    _normwise(ctx.view(ctx.bubbles(T)).cpu().numpy(), obub.bubbles(pt, T, "dot", ff), 1e-10, "loops")
    _normwise(ctx.view(ctx.project(_dev(X))).cpu().numpy(), oproj.project(pt, X, ff), 1e-10, "projections")
    _normwise(ctx.view(ctx.rhs(T, _dev(X))).cpu().numpy(), orhs.rhs(pt, T, X, ff), 1e-10, "rhs")


def test_mesh_mixed_precision_rhs(tf):
    pt = _point(10, 24, 4, radius=1)
    ff = FormFactors(4)
    ctx = tf.Context([pt], precision="mixed")
    X = synth.random_channels(pt.nq, ff.nff, seed=71)
    _normwise(ctx.view(ctx.rhs(0.1, _dev(X))).cpu().numpy(), orhs.rhs(pt, 0.1, X, ff), 1e-5, "mixed rhs")


def test_mesh_with_976_momenta_on_sampled_q(tf):
    """The uniform 24 x 24 grid refined 3 x 3 within two cells of q = 0 and
    (pi, pi): 976 momenta (the paper's pairing mesh has 992), N_ff = 13,
    96 x 96 fine grid, against the oracle at sampled momenta of both cell
    sizes."""
    pt = _point(24, 96, 3, radius=2)
    assert pt.nq == 976
    ff = FormFactors(3)
    ctx = tf.Context([pt])
    X = synth.random_channels(pt.nq, ff.nff, seed=72)
    T = 0.02
    got = ctx.view(ctx.rhs(T, _dev(X))).cpu().numpy()
    w = pt.mesh.w
    idx = np.concatenate([synth.sample_indices(pt.nq, 6, seed=1),
                          np.flatnonzero(w < w.max())[:3], np.flatnonzero(w == w.max())[:3]])
    idx = np.unique(idx)
    ref = orhs.rhs(pt, T, X, ff, q_index=idx)
    _normwise(got[:, idx], ref, 1e-10, "rhs at sampled momenta")


def test_mesh_flows(tf):
    """RK4 and adaptive flows on a mesh: the oracle's critical scale and
    leading instability; graph-replayed RK4 = eager bit for bit."""
    import torch
    pt = _point(8, 24, 1, radius=1, tp=0.0, mu=0.0)
    ctx = tf.Context([pt])
    ref = oflow.flow_rk4(pt, 10.0, 0.01, 80, 20.0)
    Xe, Xg = ctx.empty(3).zero_(), ctx.empty(3).zero_()
    re = ctx.flow(Xe, tf.FlowOptions(T0=10.0, Tmin=0.01, Xmax=20.0, scheme="rk4", nsteps=80))[0]
    rg = ctx.flow(Xg, tf.FlowOptions(T0=10.0, Tmin=0.01, Xmax=20.0, scheme="rk4", nsteps=80, use_graph=True))[0]
    assert re == rg and torch.equal(Xe, Xg)
    assert re.status == "diverged" and ref.status == oflow.STATUS_DIVERGED
    assert abs(re.Tc / ref.Tc - 1) < 1e-6
    assert (re.channel, re.q_index, re.irrep) == (ref.channel, ref.q_index, ref.irrep)
    rd = ctx.flow(ctx.empty(3).zero_(), tf.FlowOptions(T0=10.0, Tmin=0.01, Xmax=20.0, scheme="dopri5",
                                                      rtol=1e-7, atol=1e-9))[0]
    assert rd.status == "diverged" and abs(rd.Tc / ref.Tc - 1) < 1e-2
