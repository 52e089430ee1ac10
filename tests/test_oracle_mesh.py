"""Pins of the oracle on non-uniform transfer meshes (Sec. 4: the exchange
propagators on an adaptively dense set of momenta).

Reading: the loops and the products are evaluated at the mesh points; the
projections' Fourier coefficients of the gauged propagators are the mesh
quadrature with the cells' area fractions as weights (1/N_q on the uniform
grid).  Pinned by:
  * a mesh without refined cells = the uniform grid (the DFT path);
  * a mesh refined everywhere by an odd factor f = the uniform grid of
    f Lq points (same points, same weights) evaluated by the uniform path;
  * the six cross projections on a genuinely non-uniform mesh = literal
    double momentum sums of the projection rules applied to the propagator
    the mesh represents (its mesh Fourier series, built independently).
"""
import numpy as np
import pytest

import synth
from brute_force import MeshFourierPropagator, project_brute
from oracle.lattice import FormFactors, q_grid
from oracle.projections import cross_projections
from oracle.rhs import rhs


def _mesh_point(Lq, Lk, shells, mesh, **kw):
    p = synth.Point(t=1.0, tp=kw.get("tp", -0.2), U=kw.get("U", 2.7), Lq=Lq, Lk=Lk, shells=shells,
                    mu=kw.get("mu", -0.4))
    p.mesh = mesh
    return p


def test_unrefined_mesh_is_the_uniform_grid():
    pt = synth.Point(t=1.0, tp=-0.2, U=2.7, Lq=8, Lk=16, shells=2, mu=-0.4)
    mesh = synth.refined_mesh(8, 3, [(0.0, 0.0)], radius=-1)
    qx, qy = q_grid(8)
    assert np.array_equal(mesh.qx, qx) and np.array_equal(mesh.qy, qy)
    pm = _mesh_point(8, 16, 2, mesh)
    X = synth.random_channels(pt.nq, pt.nff, seed=3)
    a, b = rhs(pt, 0.2, X), rhs(pm, 0.2, X)
    assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max()


def test_fully_refined_mesh_is_the_finer_uniform_grid():
    """Every coarse cell refined by 3: the points and weights of the uniform
    grid of 3 Lq points, so every step equals the uniform path there."""
    Lq, f = 6, 3
    mesh = synth.refined_mesh(Lq, f, [(0.0, 0.0)], radius=Lq)
    fine = synth.Point(t=1.0, tp=-0.2, U=2.7, Lq=Lq * f, Lk=20, shells=1, mu=-0.4)
    pm = _mesh_point(Lq, 20, 1, mesh)
    fx, fy = q_grid(Lq * f)
    key = {(round(x, 9), round(y, 9)): i for i, (x, y) in enumerate(zip(fx, fy))}
    perm = np.array([key[(round(x, 9), round(y, 9))] for x, y in zip(mesh.qx, mesh.qy)])
    assert sorted(perm) == list(range(fine.nq)) and np.allclose(mesh.w, 1.0 / fine.nq)
    X = synth.random_channels(fine.nq, fine.nff, seed=4)
    a = rhs(fine, 0.15, X)[:, perm]
    b = rhs(pm, 0.15, X[:, perm])
    assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()


@pytest.mark.parametrize("shells,Lq,wmax,Lf", [(1, 6, 3, 14), (2, 6, 3, 14)])
def test_mesh_cross_projections_equal_double_momentum_sums(shells, Lq, wmax, Lf):
    """On a mesh refined around q = 0 and (pi, pi), each cross projection at
    mesh momenta (refined and coarse ones) equals the literal double integral
    of the projection rule for the propagator the mesh represents (its
    Fourier series includes frequencies beyond those the projections use,
    which the integrals must filter out)."""
    ff = FormFactors(shells)
    mesh = synth.refined_mesh(Lq, 3, [(0.0, 0.0), (np.pi, np.pi)], radius=1)
    pm = _mesh_point(Lq, 8, shells, mesh)
    X = synth.random_channels(mesh.nq, ff.nff, seed=20 + shells)
    kp = cross_projections(pm, X, ff)
    props = {k: MeshFourierPropagator(ff, mesh.qx, mesh.qy, mesh.w, X[i], wmax) for i, k in enumerate("PCD")}
    src = {"SC": props["P"], "C": props["C"], "D": props["D"]}
    pairs = {"P[C]": ("P", "C"), "P[D]": ("P", "D"), "C[P]": ("C", "SC"),
             "C[D]": ("C", "D"), "D[P]": ("D", "SC"), "D[C]": ("D", "C")}
    idx = [0, 1, mesh.nq // 2, mesh.nq - 1]
    for key, (onto, kind) in pairs.items():
        for i in idx:
            b = project_brute(ff, src[kind], onto, kind, mesh.qx[i], mesh.qy[i], Lf)
            assert np.abs(b - kp[key][i]).max() <= 1e-12 * max(1.0, np.abs(b).max()), (key, i)
