"""Pins of the oracle's projections (eqns. proj_VP/VC/VD) against brute force."""
import numpy as np
import pytest

import synth
from brute_force import TrigPropagator, channel_function, project_brute
from oracle.lattice import FormFactors, q_grid
from oracle.projections import cross_projections, project

PAIRS = {"P[C]": ("P", "C"), "P[D]": ("P", "D"), "C[P]": ("C", "SC"),
         "C[D]": ("C", "D"), "D[P]": ("D", "SC"), "D[C]": ("D", "C")}


def _state(ff, Lq, wmax, seed):
    props = {k: TrigPropagator(ff, wmax, seed=seed + i) for i, k in enumerate("PCD")}
    qx, qy = q_grid(Lq)
    X = np.stack([props[k](qx, qy) for k in "PCD"])
    return props, X


@pytest.mark.parametrize("shells,Lq,wmax,Lf,nl", [(0, 4, 1, 6, 16), (1, 6, 2, 10, 6),
                                                   (2, 6, 2, 10, 4), (3, 10, 2, 12, 2),
                                                   (4, 10, 2, 12, 2)])
def test_cross_projections_equal_double_momentum_sums(shells, Lq, wmax, Lf, nl):
    """Each of the six cross projections equals the literal double integral of
    the projection rule applied to the channel decomposition."""
    ff = FormFactors(shells)
    props, X = _state(ff, Lq, wmax, seed=100 + shells)
    pt = synth.small_point(Lq=Lq, Lk=8, shells=shells)
    kp = cross_projections(pt, X, ff)
    src = {"SC": props["P"], "C": props["C"], "D": props["D"]}
    qx, qy = q_grid(Lq)
    idx = synth.sample_indices(qx.size, nl, seed=shells)
    for key, (onto, kind) in PAIRS.items():
        for i in idx:
            b = project_brute(ff, src[kind], onto, kind, qx[i], qy[i], Lf)
            assert np.abs(b - kp[key][i]).max() <= 1e-13 * max(1.0, np.abs(b).max()), (key, i)


def test_trig_propagator_gives_periodic_vertex():
    """The half-bond phase of the test propagators is what makes V periodic in
    every fermion momentum (shifting k1 and k4 by a reciprocal vector)."""
    ff = FormFactors(2)
    prop = TrigPropagator(ff, 2, seed=7)
    rng = np.random.default_rng(1)
    k1, k2, k3 = ((rng.uniform(-3, 3, 20), rng.uniform(-3, 3, 20)) for _ in range(3))
    for kind in ("SC", "C", "D"):
        a = channel_function(ff, prop, kind, k1, k2, k3)
        for G in ((2 * np.pi, 0.0), (0.0, 2 * np.pi)):
            b = channel_function(ff, prop, kind, (k1[0] + G[0], k1[1] + G[1]), k2, k3)
            c = channel_function(ff, prop, kind, k1, (k2[0] + G[0], k2[1] + G[1]), k3)
            np.testing.assert_allclose(a, b, atol=1e-12)
            np.testing.assert_allclose(a, c, atol=1e-12)


def test_onsite_limit_is_bz_average():
    """N_ff = 1: every cross projection is the BZ mean of the other channel."""
    pt = synth.small_point(Lq=6, Lk=8, shells=0, U=2.0)
    X = synth.random_channels(36, 1, seed=5)
    V = project(pt, X)
    P, C, D = X[:, :, 0, 0]
    np.testing.assert_allclose(V[0, :, 0, 0], 2.0 - P + C.mean() + D.mean(), atol=1e-14)
    np.testing.assert_allclose(V[1, :, 0, 0], 2.0 - P.mean() + C + D.mean(), atol=1e-14)
    np.testing.assert_allclose(V[2, :, 0, 0], 2.0 - P.mean() + C.mean() + D, atol=1e-14)


def test_bare_and_self_projection():
    pt = synth.small_point(Lq=6, Lk=8, shells=1, U=3.0)
    V = project(pt, np.zeros((3, 36, 5, 5)))
    ref = np.zeros((36, 5, 5))
    ref[:, 0, 0] = 3.0
    for c in range(3):
        np.testing.assert_array_equal(V[c], ref)
    X = synth.random_channels(36, 5, seed=9)
    Vd = project(pt, X, no_cross=True)
    np.testing.assert_allclose(Vd[0], ref - X[0])
    np.testing.assert_allclose(Vd[1], ref + X[1])
    np.testing.assert_allclose(Vd[2], ref + X[2])


def test_vanishing_bond_length_bound():
    """Appendix B: the projection vanishes once the bond length of f_n exceeds
    the summed bond lengths of f_m and of the propagator's form factors.
    Input only in the onsite component -> row m=0 (bond length 0) of every
    cross term has only the n=0 entry."""
    pt = synth.small_point(Lq=10, Lk=8, shells=4)
    ff = FormFactors(4)
    X = np.zeros((3, 100, 21, 21))
    X[:, :, 0, 0] = synth.random_channels(100, 1, seed=2)[:, :, 0, 0]
    kp = cross_projections(pt, X, ff)
    for key, val in kp.items():
        assert np.abs(val[:, 0, 1:]).max() < 1e-14, key
    # input in shells <= 1: row 0 has no entry in shell 4 (|R| = sqrt5 > 0 + 1 + 1)
    X = np.zeros((3, 100, 21, 21))
    X[:, :, :5, :5] = synth.random_channels(100, 5, seed=3)
    kp = cross_projections(pt, X, ff)
    for key, val in kp.items():
        assert np.abs(val[:, 0, 13:]).max() < 1e-13, key
        assert np.abs(val[:, 0, :13]).max() > 1e-3, key


def test_flowed_state_symmetries():
    """Appendix C: along the flow P, C, D stay symmetric, P = pi_m pi_n P,
    C(-l) = C(l), D(-l) = D(l); then V^P, V^C, V^D are symmetric too.
    (Random states lack these relations, so V is not symmetric for them.)"""
    from oracle.flow import flow_rk4
    pt = synth.Point(t=1.0, tp=-0.2, U=3.0, Lq=8, Lk=16, shells=2, mu=-0.5)
    ff = FormFactors(2)
    X = flow_rk4(pt, 10.0, 0.5, 6, 1e9).X
    assert np.abs(X).max() > 1e-3
    np.testing.assert_allclose(X, np.swapaxes(X, -1, -2), atol=1e-13)
    odd = np.outer(ff.parity, ff.parity) < 0
    assert np.abs(X[0][:, odd]).max() < 1e-14
    qx, qy = q_grid(8)
    for i in range(qx.size):
        if qx[i] == -np.pi or qy[i] == -np.pi:
            continue
        j = int(np.flatnonzero(np.isclose(qx, -qx[i]) & np.isclose(qy, -qy[i]))[0])
        np.testing.assert_allclose(X[1:, j], X[1:, i], atol=1e-13)
    V = project(pt, X, ff)
    np.testing.assert_allclose(V, np.swapaxes(V, -1, -2), atol=1e-12)
