"""Pins of the oracle's Omega-cutoff loops and flow (the regulator named in Sec. 3, T = 0).

The closed forms of the oracle are checked against what does not use them:
direct numerical quadrature of the frequency integrals of the regulated
propagators and of their scale derivative, the sum rule that integrates the
scale derivative back to the unregulated zero-temperature loop, limits on the
grid, and flows that reduce to RPA ladders or scalar ODEs.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import synth
from oracle.bubbles import bubbles, loop_omega, loop_omega_dot
from oracle.flow import STATUS_REACHED_TMIN, flow_rk4
from oracle.lattice import FormFactors

# (eps1, eps2, Omega): both signs, near-diagonal pairs, |eps|/Omega from 0 to 1e3
PAIRS = [(0.3, -0.2, 0.5), (1.0, 1.0, 0.2), (0.05, 0.0501, 0.01), (-2.0, 3.0, 1.3),
         (0.0, 0.0, 0.7), (0.4, -0.4, 0.02), (2.5, 2.49, 0.03), (-1.7, -1.7000001, 0.4),
         (3.0, 0.0, 0.003), (-0.8, 0.6, 5.0), (1e-9, -2e-9, 0.1)]


def _regulator(w, Om):
    return w * w / (w * w + Om * Om)


def _gg(w, e1, e2, ch):
    g1 = 1.0 / (1j * w - e1)
    g2 = 1.0 / (1j * w - e2) if ch == "ph" else 1.0 / (-1j * w - e2)
    return g1 * g2


def _quad_even(fn, scale):
    """int_{-inf}^{inf} dw/2pi fn(w) for an integrand whose real part is even."""
    pts = sorted({0.0, scale})
    total = 0.0
    edges = [0.0] + [p for p in pts if p > 0] + [np.inf]
    for lo, hi in zip(edges[:-1], edges[1:]):
        v, _ = integrate.quad(lambda w: fn(w).real, lo, hi, epsabs=0.0, epsrel=1e-13, limit=400)
        total += v
    return 2.0 * total / (2.0 * math.pi)


@pytest.mark.parametrize("ch", ["ph", "pp"])
@pytest.mark.parametrize("e1,e2,Om", PAIRS)
def test_omega_loop_equals_frequency_integral(e1, e2, Om, ch):
    """L^X = int dw/2pi chi(w)^2 G(iw, e1) G(+-iw, e2) with chi = w^2/(w^2+Om^2)."""
    ref = _quad_even(lambda w: _regulator(w, Om) ** 2 * _gg(w, e1, e2, ch), Om)
    val = float(loop_omega(e1, e2, Om, ch))
    assert abs(val - ref) <= 1e-10 * max(abs(ref), 1.0 / (4 * Om) * 1e-6)


@pytest.mark.parametrize("ch", ["ph", "pp"])
@pytest.mark.parametrize("e1,e2,Om", PAIRS)
def test_omega_loop_dot_equals_integral_of_scale_derivative(e1, e2, Om, ch):
    """dL/dOm = int dw/2pi d(chi^2)/dOm G G, d(chi^2)/dOm = -4 Om w^4/(w^2+Om^2)^3."""
    dreg = lambda w: -4.0 * Om * w ** 4 / (w * w + Om * Om) ** 3
    ref = _quad_even(lambda w: dreg(w) * _gg(w, e1, e2, ch), Om)
    val = float(loop_omega_dot(e1, e2, Om, ch))
    assert abs(val - ref) <= 1e-10 * max(abs(ref), 1.0 / (4 * Om * Om) * 1e-6)


def test_omega_loop_dot_matches_central_difference():
    rng = np.random.default_rng(4)
    e1, e2 = rng.uniform(-3, 3, 60), rng.uniform(-3, 3, 60)
    Om, h = 0.37, 1e-5
    for ch in ("ph", "pp"):
        fd = (loop_omega(e1, e2, Om + h, ch) - loop_omega(e1, e2, Om - h, ch)) / (2 * h)
        np.testing.assert_allclose(loop_omega_dot(e1, e2, Om, ch), fd, rtol=1e-7, atol=1e-9)


def _lindhard_T0(e1, e2, ch):
    """Unregulated zero-temperature loops: (n(e1)-n(e2))/(e1-e2), (1-n(e1)-n(e2))/(e1+e2)."""
    n = lambda e: 1.0 if e < 0 else 0.0
    if ch == "ph":
        return (n(e1) - n(e2)) / (e1 - e2)
    return (1.0 - n(e1) - n(e2)) / (e1 + e2)


@pytest.mark.parametrize("ch", ["ph", "pp"])
@pytest.mark.parametrize("e1,e2", [(0.3, -0.2), (-2.0, 3.0), (0.4, -0.4 + 1e-3), (1.0, 2.0),
                                   (-0.5, -1.5), (0.7, 0.1)])
def test_omega_flow_sum_rule(e1, e2, ch):
    """L(Om -> inf) = 0 and L(Om -> 0) = the T = 0 loop, so
    int_0^inf dOm dL/dOm = -L_{T=0}; integrated in s = ln Om."""
    f = lambda s: math.exp(s) * float(loop_omega_dot(e1, e2, math.exp(s), ch))
    v, _ = integrate.quad(f, -40.0, 40.0, epsabs=1e-14, epsrel=1e-12, limit=400,
                          points=[math.log(abs(e1) + 1e-30), math.log(abs(e2) + 1e-30)])
    ref = -_lindhard_T0(e1, e2, ch)
    assert abs(v - ref) <= 1e-9 * max(1.0, abs(ref))


def test_omega_large_scale_limit_on_grid():
    """|eps| << Om: dL^ph/dOm -> 1/(4 Om^2), dL^pp/dOm -> -1/(4 Om^2) pairwise, so
    the projected loops tend to +-delta_mn/(4 Om^2) (orthonormal form factors)."""
    pt = synth.Point(t=1.0, tp=-0.2, U=3.0, Lq=6, Lk=16, shells=2, mu=-0.4)
    Om = 1e6
    d = bubbles(pt, Om, "dot", regulator="omega") * 4 * Om * Om
    eye = np.eye(FormFactors(2).nff)
    np.testing.assert_allclose(d[1], np.broadcast_to(eye, d[1].shape), atol=2e-5)
    np.testing.assert_allclose(d[0], -np.broadcast_to(eye, d[0].shape), atol=2e-5)


@pytest.mark.parametrize("which", ["value", "dot"])
def test_omega_nesting_identity_half_filling(which):
    """t'=0, mu=0: eps(p + Q) = -eps(p) gives chi^ph_00(Q) = -chi^pp_00(0)."""
    pt = synth.Point(t=1.0, tp=0.0, U=3.0, Lq=8, Lk=24, shells=0, mu=0.0)
    Lq = pt.Lq
    for Om in (0.05, 0.7, 4.0):
        b = bubbles(pt, Om, which, regulator="omega")
        iQ = 0                           # q = (-pi, -pi) = (pi, pi)
        i0 = (Lq // 2) * Lq + Lq // 2    # q = 0
        assert abs(b[1, iQ, 0, 0] + b[0, i0, 0, 0]) <= 1e-13 * abs(b[0, i0, 0, 0])


def _rpa_omega(point, Om0, Om, U):
    b0 = bubbles(point, Om0, "value", regulator="omega")
    b1 = bubbles(point, Om, "value", regulator="omega")
    dpp = b1[0, :, 0, 0] - b0[0, :, 0, 0]
    dph = b1[1, :, 0, 0] - b0[1, :, 0, 0]
    return U / (1 + U * dpp), U / (1 + U * dph), U / (1 - U * dph)


def test_decoupled_omega_flow_is_rpa_ladder():
    """Without inter-channel terms the Omega flow integrates the loop derivative
    to RPA ladders built from the Omega-regulated loop values themselves."""
    pt = synth.Point(t=1.0, tp=-0.1, U=2.0, Lq=6, Lk=16, shells=0, mu=-0.2)
    Om0, Om1 = 50.0, 0.2
    r = flow_rk4(pt, Om0, Om1, 200, Xmax=1e9, no_cross=True, regulator="omega")
    assert r.status == STATUS_REACHED_TMIN
    P, C, D = r.X[:, :, 0, 0]
    VP, VC, W = _rpa_omega(pt, Om0, Om1, 2.0)
    np.testing.assert_allclose(2.0 - P, VP, rtol=2e-8)
    np.testing.assert_allclose(2.0 + C, VC, rtol=2e-8)
    np.testing.assert_allclose(2 * (2.0 + D) - (2.0 + C), W, rtol=2e-8)


def test_onsite_coupled_omega_flow_matches_scalar_ode():
    """N_ff = 1 coupled Omega flow = three scalar per-q ODEs coupled by BZ means."""
    pt = synth.Point(t=1.0, tp=-0.15, U=2.0, Lq=6, Lk=12, shells=0, mu=-0.3)
    U, Om0, Om1, n = 2.0, 20.0, 0.5, 40
    r = flow_rk4(pt, Om0, Om1, n, Xmax=1e9, regulator="omega")

    def f(Om, y):
        P, C, D = y
        chi = bubbles(pt, Om, "dot", regulator="omega")
        pp, ph = chi[0, :, 0, 0], chi[1, :, 0, 0]
        VP = U - P + C.mean() + D.mean()
        VC = U - P.mean() + C + D.mean()
        VD = U - P.mean() + C.mean() + D
        return np.stack([VP * pp * VP, -VC * ph * VC, 2 * VD * ph * VD - 2 * VC * ph * VD])

    y = np.zeros((3, 36))
    s, h = math.log(Om0), (math.log(Om1) - math.log(Om0)) / n
    g = lambda sv, yv: math.exp(sv) * f(math.exp(sv), yv)
    for i in range(n):
        k1 = g(s, y)
        k2 = g(s + h / 2, y + h / 2 * k1)
        k3 = g(s + h / 2, y + h / 2 * k2)
        k4 = g(s + h, y + h * k3)
        y = y + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        s += h
    np.testing.assert_allclose(r.X[:, :, 0, 0], y, atol=1e-13)
