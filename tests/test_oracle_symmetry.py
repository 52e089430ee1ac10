"""Pins of the point-group covariance law (oracle/symmetry.py).

The law X(q) = T X(q') T^T (h q = q' + G) is derived from the grid sum of
eqn. chis.  It is checked here against quantities the oracle computes
without it: the loops' own grid sums (any point, both regulators), and the
full increment of a symmetrised random state (projections and products
included).  A planted mistake (dropping the half shift G/2 of the zone-edge
momenta) must fail the loop pin.
"""
import numpy as np
import pytest

import synth
from oracle import symmetry as S
from oracle.bubbles import bubbles
from oracle.lattice import FormFactors
from oracle.rhs import rhs


class _Point:
    def __init__(self, shells, Lq, Lk, t=1.0, tp=-0.25, mu=-0.9, U=3.0):
        self.shells, self.Lq, self.Lk = shells, Lq, Lk
        self.t, self.tp, self.mu, self.U = t, tp, mu, U


@pytest.mark.parametrize("shells", [0, 1, 2, 3, 4])
def test_transforms_are_signed_permutations_and_a_representation(shells):
    ff = FormFactors(shells)
    seen = []
    for o, h in enumerate(S.C4V_OPS):
        for g in ((0, 0), (1, 0), (0, 1), (1, 1)):
            T = S.ff_transform(ff, h, g)
            # one entry +-1 per row and column: a signed permutation, orthogonal
            assert np.allclose(np.abs(T).sum(axis=1), 1.0) and np.allclose(np.abs(T).sum(axis=0), 1.0)
            assert np.allclose(np.abs(T).max(axis=1), 1.0)
            assert np.allclose(T @ T.T, np.eye(ff.nff), atol=1e-13)
            seen.append(T)
    assert np.allclose(S.ff_transform(ff, S.C4V_OPS[0], (0, 0)), np.eye(ff.nff))
    # the half shift composes with the operation: f_m(h^-1 (k - G/2)) =
    # sum_n T(h, 0)_mn f_n(k - G/2), so T(h, g) = T(h, 0) T(1, g)
    for o, h in enumerate(S.C4V_OPS):
        T0 = S.ff_transform(ff, h, (0, 0))
        for g in ((1, 0), (0, 1), (1, 1)):
            assert np.allclose(S.ff_transform(ff, h, g), T0 @ S.ff_transform(ff, S.C4V_OPS[0], g), atol=1e-13)
    # composition: f_m(h1^-1 h2^-1 k) gives T(h2 h1) = T(h1) T(h2) at G = 0
    for h1 in S.C4V_OPS:
        for h2 in S.C4V_OPS:
            lhs = S.ff_transform(ff, h2 @ h1, (0, 0))
            rhs_ = S.ff_transform(ff, h1, (0, 0)) @ S.ff_transform(ff, h2, (0, 0))
            assert np.allclose(lhs, rhs_, atol=1e-13)


@pytest.mark.parametrize("shells,Lq,Lk,reg", [(1, 6, 12, "T"), (2, 8, 16, "T"), (3, 10, 20, "T"),
                                              (2, 6, 12, "omega"), (4, 6, 12, "T")])
def test_loops_obey_the_law(shells, Lq, Lk, reg):
    ff = FormFactors(shells)
    pt = _Point(shells, Lq, Lk)
    chi = bubbles(pt, 0.1, "dot", ff, regulator=reg)
    scale = np.abs(chi).max()
    assert S.defect(chi, ff, Lq) <= 1e-13 * scale
    # the loop values themselves, not only their derivative
    chi0 = bubbles(pt, 0.1, "value", ff, regulator=reg)
    assert S.defect(chi0, ff, Lq) <= 1e-13 * np.abs(chi0).max()


def test_dropping_the_half_shift_breaks_the_loop_law():
    """Planted mistake: T(h, 0) in place of T(h, G) at the zone-edge momenta."""
    shells, Lq, Lk = 2, 6, 12
    ff = FormFactors(shells)
    chi = bubbles(_Point(shells, Lq, Lk), 0.1, "dot", ff)
    worst = 0.0
    for h in S.C4V_OPS:
        T0 = S.ff_transform(ff, h, (0, 0))
        for q in range(Lq * Lq):
            q2, g = S.image(Lq, h, q)
            worst = max(worst, float(np.abs(chi[:, q] - T0 @ chi[:, q2] @ T0.T).max()))
    assert worst > 1e-3 * np.abs(chi).max()
    assert S.defect(chi, ff, Lq) <= 1e-13 * np.abs(chi).max()


def test_symmetrize_projects_onto_symmetric_states():
    shells, Lq = 2, 8
    ff = FormFactors(shells)
    X = synth.random_channels(Lq * Lq, ff.nff, seed=11)
    assert S.defect(X, ff, Lq) > 0.1
    Xs = S.symmetrize(X, ff, Lq)
    assert S.defect(Xs, ff, Lq) <= 1e-14 * np.abs(Xs).max() * 10
    assert np.abs(S.symmetrize(Xs, ff, Lq) - Xs).max() <= 1e-14 * np.abs(Xs).max() * 10
    # (m, n) symmetry survives the average (T X T^T keeps symmetric matrices symmetric)
    assert np.abs(Xs - np.swapaxes(Xs, -1, -2)).max() <= 1e-15 * np.abs(Xs).max() * 10


@pytest.mark.parametrize("shells,Lq,Lk,reg", [(1, 6, 12, "T"), (3, 10, 20, "T"), (3, 10, 20, "omega"),
                                              (4, 10, 20, "T")])
def test_increment_of_a_symmetric_state_obeys_the_law(shells, Lq, Lk, reg):
    """Projections and products are covariant: a symmetric state has a symmetric increment."""
    ff = FormFactors(shells)
    pt = _Point(shells, Lq, Lk)
    Xs = S.symmetrize(synth.random_channels(Lq * Lq, ff.nff, seed=5), ff, Lq)
    d = rhs(pt, 0.1, Xs, ff, regulator=reg)
    assert S.defect(d, ff, Lq) <= 1e-13 * np.abs(d).max()
    # a random (non-symmetric) state does not give one
    d_r = rhs(pt, 0.1, synth.random_channels(Lq * Lq, ff.nff, seed=5), ff, regulator=reg)
    assert S.defect(d_r, ff, Lq) > 1e-3 * np.abs(d_r).max()
