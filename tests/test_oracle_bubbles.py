"""Pins of the oracle's loops (eqn. chis, temperature flow)."""
import mpmath as mp
import numpy as np
import pytest
from scipy import integrate, special

import synth
from brute_force import matsubara_loop, matsubara_loop_dot
from oracle.bubbles import bubbles, loop, loop_dot
from oracle.lattice import FormFactors, dispersion, k_grid, q_grid

POINTS = [(0.3, -0.2, 0.5), (1.0, 1.0, 0.2), (0.05, 0.0501, 0.01), (-2.0, 3.0, 1.3),
          (0.0, 0.0, 0.7), (0.4, -0.4, 0.02), (2.5, 2.49, 0.03)]


@pytest.mark.parametrize("ch", ["ph", "pp"])
@pytest.mark.parametrize("e1,e2,T", POINTS)
def test_loop_equals_matsubara_sum(e1, e2, T, ch):
    ref = matsubara_loop(e1, e2, T, ch)
    assert abs(float(mp.im(ref))) < 1e-30
    val = float(loop(e1, e2, T, ch))
    assert abs(val - float(mp.re(ref))) <= 1e-14 * max(1.0, abs(float(mp.re(ref))))


@pytest.mark.parametrize("ch", ["ph", "pp"])
@pytest.mark.parametrize("e1,e2,T", POINTS[:5])
def test_loop_dot_equals_T_derivative_of_matsubara_sum(e1, e2, T, ch):
    ref = float(mp.re(matsubara_loop_dot(e1, e2, T, ch)))
    val = float(loop_dot(e1, e2, T, ch))
    assert abs(val - ref) <= 1e-12 * max(1.0, abs(ref))


def test_loop_far_from_fermi_surface_is_finite():
    """Log-domain evaluation: no overflow at |eps/T| ~ 1e4 (both signs)."""
    e1 = np.array([8.0, 8.0, -8.0, 1e-3, 4.0])
    e2 = np.array([-8.0, 7.9, -7.99, -1e-3, 4.0])
    for ch in ("ph", "pp"):
        for T in (1e-3, 1e-2):
            v, d = loop(e1, e2, T, ch), loop_dot(e1, e2, T, ch)
            assert np.all(np.isfinite(v)) and np.all(np.isfinite(d))
    # opposite-sign pair: L^ph = (n(e1) - n(e2))/(e1 - e2) -> -1/(e1 - e2) at T -> 0
    assert np.isclose(loop(8.0, -8.0, 1e-3, "ph"), -1.0 / 16.0, rtol=1e-14)
    assert np.isclose(loop(8.0, -8.0, 1e-3, "pp"), 0.0, atol=1e-300)
    # both below the Fermi level: L^pp = (1 - 1 - 1)/(e1 + e2) = +1/16
    assert np.isclose(loop(-8.0, -8.0, 1e-3, "pp"), 1.0 / 16.0, rtol=1e-14)


def test_loop_dot_matches_numpy_central_difference():
    rng = np.random.default_rng(3)
    e1, e2 = rng.uniform(-3, 3, 50), rng.uniform(-3, 3, 50)
    T, h = 0.37, 1e-5
    for ch in ("ph", "pp"):
        fd = (loop(e1, e2, T + h, ch) - loop(e1, e2, T - h, ch)) / (2 * h)
        np.testing.assert_allclose(loop_dot(e1, e2, T, ch), fd, rtol=1e-7, atol=1e-9)


@pytest.mark.parametrize("Lk", [16, 24, 32])
@pytest.mark.parametrize("which", ["value", "dot"])
def test_nesting_identity_half_filling(Lk, which):
    """t'=0, mu=0: eps(p + Q) = -eps(p) gives chi^ph_00(Q) = -chi^pp_00(0) for Lk = 0 mod 4 ... and 8."""
    if Lk % 4:
        pytest.skip("needs Lk divisible by 4")
    p = synth.Point(t=1.0, tp=0.0, U=3.0, Lq=8, Lk=Lk, shells=1, mu=0.0)
    qx, qy = q_grid(8)
    iQ = int(np.flatnonzero((qx == -np.pi) & (qy == -np.pi))[0])
    i0 = int(np.flatnonzero((qx == 0) & (qy == 0))[0])
    for T in (0.05, 0.3, 2.0):
        b = bubbles(p, T, which)
        scale = abs(b[0, i0, 0, 0])
        assert abs(b[1, iQ, 0, 0] + b[0, i0, 0, 0]) <= 1e-14 * scale


def test_chi_ph_q0_is_fermi_derivative():
    p = synth.small_point(Lq=6, Lk=20, shells=1)
    T = 0.23
    b = bubbles(p, T, "value")
    qx, qy = q_grid(6)
    i0 = int(np.flatnonzero((qx == 0) & (qy == 0))[0])
    kx, ky = k_grid(20)
    e = dispersion(kx, ky, p.t, p.tp, p.mu)
    ref = np.mean(-1.0 / (4 * T * np.cosh(e / (2 * T)) ** 2))
    assert abs(b[1, i0, 0, 0] - ref) < 1e-14 * abs(ref)


def test_high_temperature_limits():
    p = synth.small_point(Lq=6, Lk=12, shells=1)
    T = 1e4
    b = bubbles(p, T, "value")
    d = bubbles(p, T, "dot")
    np.testing.assert_allclose(b[1, :, 0, 0], -1 / (4 * T), rtol=1e-6)
    np.testing.assert_allclose(b[0, :, 0, 0], 1 / (4 * T), rtol=1e-6)
    np.testing.assert_allclose(d[1, :, 0, 0], 1 / (4 * T * T), rtol=1e-6)
    np.testing.assert_allclose(d[0, :, 0, 0], -1 / (4 * T * T), rtol=1e-6)
    # orthonormal form factors: chi_mn -> +-delta_mn/(4T)
    np.testing.assert_allclose(b[0, 3], np.eye(5) / (4 * T), atol=1e-9 / T)


def test_continuum_dos_closed_form():
    """t'=0, mu=0, q=0: grid sums converge to the DOS integrals with
    rho(e) = K(sqrt(1 - e^2/16))/(2 pi^2) (t = 1)."""
    T = 0.5
    p = synth.Point(t=1.0, tp=0.0, U=3.0, Lq=6, Lk=64, shells=0, mu=0.0)
    qx, qy = q_grid(6)
    i0 = int(np.flatnonzero((qx == 0) & (qy == 0))[0])
    b = bubbles(p, T, "value", q_index=[i0])
    rho = lambda e: special.ellipkm1(e * e / 16.0) / (2 * np.pi ** 2)   # K(m = 1 - e^2/16)
    fpp = lambda e: rho(e) * (np.tanh(e / (2 * T)) / (2 * e) if e != 0 else 1 / (4 * T))
    fph = lambda e: -rho(e) / (4 * T * np.cosh(e / (2 * T)) ** 2)
    # both integrands are even in e; the log singularity of rho sits at the end point 0
    opts = dict(limit=400, epsabs=1e-15, epsrel=1e-13)
    pp = 2 * integrate.quad(fpp, 0, 4, **opts)[0]
    ph = 2 * integrate.quad(fph, 0, 4, **opts)[0]
    assert abs(b[0, 0, 0, 0] - pp) < 1e-10 * abs(pp)
    assert abs(b[1, 0, 0, 0] - ph) < 1e-10 * abs(ph)


@pytest.mark.parametrize("shells", [1, 2, 4])
def test_bubble_symmetric_parity_blocks_and_c4v(shells):
    p = synth.Point(t=1.0, tp=-0.2, U=3.0, Lq=8, Lk=16, shells=shells, mu=-0.4)
    ff = FormFactors(shells)
    d = bubbles(p, 0.15, "dot", ff)
    np.testing.assert_allclose(d, np.swapaxes(d, -1, -2), atol=1e-15 * np.abs(d).max())
    odd = np.outer(ff.parity, ff.parity) < 0
    assert np.abs(d[:, :, odd]).max() < 1e-15 * np.abs(d).max()
    # C4 rotation of the transfer momentum (interior grid points only)
    qx, qy = q_grid(8)
    g = 2 * np.pi * np.arange(16) / 16
    kx, ky = np.meshgrid(g, g, indexing="ij")
    F = ff.values(kx, ky).reshape(ff.nff, -1)
    FS = ff.values(-ky, kx).reshape(ff.nff, -1)
    CS = FS @ F.T / F.shape[1]
    for i in range(qx.size):
        if qx[i] == -np.pi or qy[i] == -np.pi:
            continue
        j = int(np.flatnonzero(np.isclose(qx, -qy[i]) & np.isclose(qy, qx[i]))[0])
        for c in range(2):
            np.testing.assert_allclose(d[c, j], CS @ d[c, i] @ CS.T, atol=1e-14 * np.abs(d).max())


def _fermi_form_dot(e1, e2, T, ch):
    """d/dT of (n_F(e1) - n_F(e2))/(e1 - e2) or (1 - n_F(e1) - n_F(e2))/(e1 + e2).

    600 digits: n_F = 1 - O(e^{-|eps|/T}) must stay distinguishable from 1."""
    mp.mp.dps = 600
    a, b = mp.mpf(e1), mp.mpf(e2)
    nF = lambda e, t: 1 / (mp.exp(e / t) + 1)
    if ch == "ph":
        f = lambda t: (nF(a, t) - nF(b, t)) / (a - b)
    else:
        f = lambda t: (1 - nF(a, t) - nF(b, t)) / (a + b)
    r = float(mp.diff(f, mp.mpf(T)))
    mp.mp.dps = 15
    return r


@pytest.mark.parametrize("ch", ["ph", "pp"])
@pytest.mark.parametrize("e1,e2,T", [(0.05, 0.06, 1e-3), (-0.4, -0.3, 1e-3), (0.2, -0.35, 1e-3),
                                     (3.0, 2.5, 0.01), (-6.0, 5.0, 0.02), (0.12, -0.11, 2e-3)])
def test_loop_dot_relative_accuracy_in_tails(e1, e2, T, ch):
    """Far from the Fermi surface dL/dT is exponentially small; it must keep its
    relative accuracy there (no cancellation between O(|eps|/T) terms)."""
    ref = _fermi_form_dot(e1, e2, T, ch)
    val = float(loop_dot(e1, e2, T, ch))
    assert abs(val - ref) <= 1e-11 * abs(ref), (val, ref)
