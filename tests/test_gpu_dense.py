"""The dense projection operator (TUFRG_DENSE_PROJECTION): the projections'
cross terms precomputed as one matrix per point and applied as one operator
product, against the factored path (same linear map: 1e-12 normwise) and
the oracle (1e-10)."""
import numpy as np
import pytest

import synth
from oracle import projections as oproj
from oracle import rhs as orhs
from oracle.lattice import FormFactors

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1604_06296_amd as tf
    tf.load_library()
    return tf


def _dev(X):
    import torch
    return torch.from_numpy(np.ascontiguousarray(X.reshape(3, -1))).cuda()


def _normwise(got, ref, tol, what=""):
    for c in range(ref.shape[0]):
        scale = np.abs(ref[c]).max()
        err = np.abs(got[c] - ref[c]).max()
        assert err <= tol * max(scale, 1e-300), f"{what} channel {c}: err {err:.3e} scale {scale:.3e}"


CASES = [dict(Lq=8, Lk=16, shells=0), dict(Lq=8, Lk=32, shells=1), dict(Lq=6, Lk=12, shells=1),
         dict(Lq=10, Lk=20, shells=0)]


@pytest.mark.parametrize("case", CASES)
def test_dense_operator_equals_factored_and_oracle(tf, case):
    pt = synth.Point(t=1.0, tp=-0.2, U=2.6, mu=-0.5, **case)
    ff = FormFactors(pt.shells)
    print(f"[dense] {case}", flush=True)
    dense, fact = tf.Context([pt], dense_projection=True), tf.Context([pt])
    for seed, T in ((81, 0.3), (82, 0.02)):
        X = synth.random_channels(pt.nq, ff.nff, seed=seed)
        Xd = _dev(X)
        vd = dense.view(dense.project(Xd)).cpu().numpy()
        _normwise(vd, fact.view(fact.project(Xd)).cpu().numpy(), 1e-12, "project vs factored")
        _normwise(vd, oproj.project(pt, X, ff), 1e-10, "project vs oracle")
        rd = dense.view(dense.rhs(T, Xd)).cpu().numpy()
        _normwise(rd, fact.view(fact.rhs(T, Xd)).cpu().numpy(), 1e-12, "rhs vs factored")
        _normwise(rd, orhs.rhs(pt, T, X, ff), 1e-10, "rhs vs oracle")


def test_dense_operator_on_a_mesh_and_in_flows(tf):
    """A refined mesh (any linear map of the state is a matrix) and the RK4
    and adaptive flows: the factored flows' outcome."""
    pt = synth.Point(t=1.0, tp=0.0, U=3.0, Lq=6, Lk=24, shells=1, mu=0.0)
    pt.mesh = synth.refined_mesh(6, 3, [(0.0, 0.0), (np.pi, np.pi)], radius=0)
    ff = FormFactors(1)
    dense, fact = tf.Context([pt], dense_projection=True), tf.Context([pt])
    X = synth.random_channels(pt.nq, ff.nff, seed=83)
    _normwise(dense.view(dense.rhs(0.1, _dev(X))).cpu().numpy(), orhs.rhs(pt, 0.1, X, ff), 1e-10, "mesh rhs")
    for opts in (tf.FlowOptions(T0=10.0, Tmin=0.01, Xmax=20.0, scheme="rk4", nsteps=60),
                 tf.FlowOptions(T0=10.0, Tmin=0.01, Xmax=20.0, scheme="dopri5", rtol=1e-7, atol=1e-9)):
        a, b = dense.flow(dense.empty(3).zero_(), opts)[0], fact.flow(fact.empty(3).zero_(), opts)[0]
        assert (a.status, a.channel, a.q_index, a.irrep) == (b.status, b.channel, b.q_index, b.irrep)
        if b.Tc:
            assert abs(a.Tc / b.Tc - 1) < 1e-8


def test_dense_operator_rejects_large_points(tf):
    from paper_1604_06296_amd.binding import TufrgError
    pt = synth.Point(t=1.0, tp=-0.2, U=2.6, mu=-0.5, Lq=8, Lk=16, shells=2)   # 3 * 64 * 81 > 8192
    with pytest.raises(TufrgError, match="dense projection operator needs"):
        tf.Context([pt], dense_projection=True)
