"""Pins of the oracle's loop harmonics, surrogate encoding and FP64 MLP.

ghat is pinned against the pinned projected loops (a different route: the
form factors evaluated on the grid), and against its high-temperature
limit; the MLP gradient is pinned by central differences.
"""
import numpy as np
import pytest

import synth
from oracle import bubbles as obub
from oracle import surrogate as osur
from oracle.lattice import FormFactors, q_grid


@pytest.mark.parametrize("shells,Lq,Lk", [(0, 4, 8), (1, 6, 10), (2, 6, 12), (3, 10, 12), (4, 10, 14)])
def test_harmonics_rebuild_the_loops(shells, Lq, Lk):
    pt = synth.Point(t=1.0, tp=-0.27, U=3.0, Lq=Lq, Lk=Lk, shells=shells, mu=-0.4)
    ff = FormFactors(shells)
    S = osur.harmonic_set(ff)
    for T in (3.0, 0.07):
        g = osur.loop_harmonics(pt, T, S)
        chi = osur.chi_from_harmonics(g, ff, S)
        ref = obub.bubbles(pt, T, "dot", ff)
        assert np.abs(chi - ref).max() <= 1e-13 * np.abs(ref).max()


def test_harmonic_counts_and_canonical_pairs():
    for shells, ns in zip(range(5), (1, 13, 25, 41, 69)):
        ff = FormFactors(shells)
        S = osur.harmonic_set(ff)
        assert len(S) == ns
        for s in S:
            Ra, Rb = osur.canonical_pair(ff, s)
            assert (Ra[0] + Rb[0], Ra[1] + Rb[1]) == s
            assert Ra in ff.bonds and Rb in ff.bonds


def test_harmonics_high_temperature_limit():
    """At T >> bandwidth: dL^ph/dT -> +1/(4T^2), dL^pp/dT -> -1/(4T^2),
    constant in p, so ghat(S=0) -> +-1/(4T^2) and ghat(S != 0) -> 0, and the
    targets of S = 0 tend to (-1, +1)."""
    pt = synth.Point(t=1.0, tp=-0.3, U=3.0, Lq=6, Lk=12, shells=1, mu=-0.5)
    ff = FormFactors(1)
    S = osur.harmonic_set(ff)
    j0 = S.index((0, 0))
    T = 1e4
    g = osur.loop_harmonics(pt, T, S)
    np.testing.assert_allclose(g[0, :, j0] * T * T, -0.25, rtol=1e-6)
    np.testing.assert_allclose(g[1, :, j0] * T * T, 0.25, rtol=1e-6)
    others = [j for j in range(len(S)) if j != j0]
    assert np.abs(g[:, :, others]).max() * T * T < 1e-6
    y = osur.targets(T, g[0, :, j0], g[1, :, j0])
    np.testing.assert_allclose(y[:, 0], -1.0, rtol=1e-3)
    np.testing.assert_allclose(y[:, 1], 1.0, rtol=1e-3)
    assert not y[:, 2:].any()


def test_features_layout():
    pt = synth.Point(t=1.0, tp=-0.25, U=3.0, Lq=8, Lk=16, shells=2, mu=-0.9)
    qx, qy = q_grid(8)
    x = osur.features(pt, 0.5, qx, qy, (1, 0), (-1, 1))
    assert x.shape == (64, 9)
    np.testing.assert_allclose(x[:, 0] * np.pi, qx)
    np.testing.assert_allclose(x[:, 2], np.log10(0.5))
    assert (x[:, 3] == -0.9).all() and (x[:, 4] == -0.25).all()
    assert (x[:, 5:] == [0.5, 0.0, -0.5, 0.5]).all()


def test_silu_gradient():
    z = np.linspace(-30, 30, 601)
    h = 1e-6
    num = (osur.silu(z + h) - osur.silu(z - h)) / (2 * h)
    np.testing.assert_allclose(osur.silu_grad(z), num, atol=1e-9)


def test_mlp_gradient_central_differences():
    rng = np.random.default_rng(5)
    widths = [9, 7, 6, 4]
    n = sum(widths[i] * widths[i + 1] + widths[i + 1] for i in range(len(widths) - 1))
    flat = rng.standard_normal(n) * 0.5
    x = rng.standard_normal((5, 9))
    y = rng.standard_normal((5, 4))
    loss, grads = osur.mlp_loss_and_grad(osur.unflatten(flat, widths), x, y)
    g = osur.flatten(grads)
    assert np.isclose(loss, np.mean((osur.mlp_forward(osur.unflatten(flat, widths), x) - y) ** 2))
    h = 1e-6
    num = np.empty(n)
    for i in range(n):
        e = np.zeros(n)
        e[i] = h
        lp, _ = osur.mlp_loss_and_grad(osur.unflatten(flat + e, widths), x, y)
        lm, _ = osur.mlp_loss_and_grad(osur.unflatten(flat - e, widths), x, y)
        num[i] = (lp - lm) / (2 * h)
    np.testing.assert_allclose(g, num, rtol=1e-6, atol=1e-9)


def test_mlp_gradient_catches_planted_mistake():
    """A dropped activation derivative in the backward pass fails the check."""
    rng = np.random.default_rng(6)
    widths = [9, 5, 4]
    n = 9 * 5 + 5 + 5 * 4 + 4
    flat = rng.standard_normal(n)
    x, y = rng.standard_normal((3, 9)), rng.standard_normal((3, 4))
    params = osur.unflatten(flat, widths)
    real = osur.silu_grad
    try:
        osur.silu_grad = lambda z: np.ones_like(z)
        _, bad = osur.mlp_loss_and_grad(params, x, y)
    finally:
        osur.silu_grad = real
    _, good = osur.mlp_loss_and_grad(params, x, y)
    assert np.abs(osur.flatten(bad) - osur.flatten(good)).max() > 1e-3
