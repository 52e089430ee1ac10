"""Flows that take the loops of the stage before at an equal temperature.

RK4's second and third stages share one temperature, so do RK4's first stage
and the last stage of the step before (its table temperature is the same
expression), and so do the sixth and seventh stages of Dormand-Prince; the
loops depend on the temperature alone, so by default the second of each pair
takes the loops its predecessor left in the workspace.  Checked here: every
flow equals, bit for bit, the same flow with the loops evaluated at every
stage (TUFRG_NO_LOOP_REUSE), in the fused single-stream form and in the
two-stream form, eager and graph-replayed, for one point and for a batch of
uneven points, in FP64 and in the mixed precision form.
"""
import pytest

import synth

pytestmark = pytest.mark.gpu

PTS = [
    synth.Point(t=1.0, tp=-0.25, U=2.8, Lq=12, Lk=36, shells=3, mu=-0.7),
    synth.Point(t=1.0, tp=-0.10, U=2.2, Lq=6, Lk=12, shells=1, mu=-0.2),
    synth.Point(t=1.0, tp=-0.30, U=3.0, Lq=10, Lk=24, shells=4, mu=-0.9),
]


@pytest.fixture(scope="module")
def tf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1604_06296_amd as tf
    tf.load_library()
    return tf


def _opts(tf, scheme, graph):
    if scheme == "rk4":
        return tf.FlowOptions(T0=10.0, Tmin=0.01, Xmax=20.0, scheme="rk4", nsteps=60, use_graph=graph)
    return tf.FlowOptions(T0=10.0, Tmin=0.01, Xmax=20.0, scheme="dopri5", rtol=1e-7, atol=1e-9,
                          use_graph=graph)


def _both(tf, pts, opts, **kw):
    import torch
    out = []
    for reuse in (True, False):
        ctx = tf.Context(pts, loop_reuse=reuse, **kw)
        X = ctx.empty(3).zero_()
        res = ctx.flow(X, opts)
        torch.cuda.synchronize()
        out.append((res, X.cpu()))
        ctx.close()
    return out


@pytest.mark.parametrize("scheme", ["rk4", "dopri5"])
@pytest.mark.parametrize("fuse", [True, False])
def test_reuse_is_bit_identical_single_point(tf, scheme, fuse):
    import torch
    print(f"[reuse] {scheme} fuse={fuse}", flush=True)
    (ra, Xa), (rb, Xb) = _both(tf, PTS[:1], _opts(tf, scheme, graph=False), fuse=fuse)
    assert ra == rb
    assert torch.equal(Xa, Xb)
    assert ra[0].n_rhs > 1


@pytest.mark.parametrize("scheme", ["rk4", "dopri5"])
def test_reuse_is_bit_identical_batch_graph(tf, scheme):
    import torch
    print(f"[reuse] batch {scheme} graph", flush=True)
    (ra, Xa), (rb, Xb) = _both(tf, PTS, _opts(tf, scheme, graph=True))
    assert ra == rb
    assert torch.equal(Xa, Xb)


def test_reuse_is_bit_identical_mixed(tf):
    import torch
    print("[reuse] mixed dopri5", flush=True)
    (ra, Xa), (rb, Xb) = _both(tf, PTS[:1], _opts(tf, "dopri5", graph=False), precision="mixed")
    assert ra == rb
    assert torch.equal(Xa, Xb)


@pytest.mark.parametrize("fuse", [True, False])
def test_reuse_is_bit_identical_rk4_graph_single_point(tf, fuse):
    """The RK4 graph holds a step after the first; the first step runs eagerly."""
    import torch
    print(f"[reuse] rk4 graph fuse={fuse}", flush=True)
    (ra, Xa), (rb, Xb) = _both(tf, PTS[:1], _opts(tf, "rk4", graph=True), fuse=fuse)
    assert ra == rb
    assert torch.equal(Xa, Xb)


def test_reuse_is_bit_identical_mixed_rk4(tf):
    import torch
    print("[reuse] mixed rk4 graph", flush=True)
    (ra, Xa), (rb, Xb) = _both(tf, PTS[:1], _opts(tf, "rk4", graph=True), precision="mixed")
    assert ra == rb
    assert torch.equal(Xa, Xb)
