"""Pins of the oracle's products and flow (eqns. matmul-P/C/D, Sec. 3-4)."""
import math

import numpy as np
import pytest

import synth
from oracle.bubbles import bubbles
from oracle.flow import (STATUS_DIVERGED, STATUS_NONFINITE, STATUS_REACHED_TMIN, classify,
                         flow_dopri5, flow_rk4)
from oracle.lattice import FormFactors
from oracle.rhs import products, rhs


def test_products_su2_spin_charge_identity_and_symmetry():
    """2 dD - dC = (2V^D - V^C) chi^ph (2V^D - V^C): the charge combination
    obeys a single-ladder equation (SU(2) structure of eqn. matmul-D)."""
    rng = np.random.default_rng(0)
    nq, nff = 7, 9
    sym = lambda a: 0.5 * (a + np.swapaxes(a, -1, -2))
    V = sym(rng.standard_normal((3, nq, nff, nff)))
    chi = sym(rng.standard_normal((2, nq, nff, nff)))
    d = products(V, chi)
    W = 2 * V[2] - V[1]
    np.testing.assert_allclose(2 * d[2] - d[1], W @ chi[1] @ W, atol=1e-12)
    np.testing.assert_allclose(d, np.swapaxes(d, -1, -2), atol=1e-12)
    # 1x1: scalar ladders
    V1 = rng.standard_normal((3, 4, 1, 1))
    c1 = rng.standard_normal((2, 4, 1, 1))
    d1 = products(V1, c1)
    np.testing.assert_allclose(d1[0], V1[0] ** 2 * c1[0])
    np.testing.assert_allclose(d1[1], -V1[1] ** 2 * c1[1])


def _rpa(point, T0, T, U):
    b0, b1 = bubbles(point, T0, "value"), bubbles(point, T, "value")
    dpp = b1[0, :, 0, 0] - b0[0, :, 0, 0]
    dph = b1[1, :, 0, 0] - b0[1, :, 0, 0]
    return U / (1 + U * dpp), U / (1 + U * dph), U / (1 - U * dph)


def test_decoupled_flow_is_rpa_ladder():
    """Without inter-channel terms each channel integrates to a momentum-resolved
    RPA ladder: V^P = U/(1+U dchi^pp), V^C = U/(1+U dchi^ph),
    2V^D - V^C = U/(1 - U dchi^ph), dchi = chi(T) - chi(T0)."""
    pt = synth.Point(t=1.0, tp=-0.1, U=2.0, Lq=6, Lk=16, shells=0, mu=-0.2)
    T0, T1 = 10.0, 0.3
    r = flow_rk4(pt, T0, T1, 200, Xmax=1e9, no_cross=True)
    assert r.status == STATUS_REACHED_TMIN
    P, C, D = r.X[:, :, 0, 0]
    VP, VC, W = _rpa(pt, T0, T1, 2.0)
    np.testing.assert_allclose(2.0 - P, VP, rtol=2e-8)
    np.testing.assert_allclose(2.0 + C, VC, rtol=2e-8)
    np.testing.assert_allclose(2 * (2.0 + D) - (2.0 + C), W, rtol=2e-8)


def test_rk4_fourth_order():
    pt = synth.Point(t=1.0, tp=-0.1, U=2.5, Lq=6, Lk=12, shells=0, mu=-0.2)
    T0, T1 = 10.0, 0.4
    exact = _rpa(pt, T0, T1, 2.5)[1]
    errs = []
    for n in (40, 80):
        r = flow_rk4(pt, T0, T1, n, Xmax=1e9, no_cross=True)
        errs.append(np.abs(2.5 + r.X[1, :, 0, 0] - exact).max())
    assert 14.0 < errs[0] / errs[1] < 18.0


def test_onsite_coupled_flow_matches_scalar_ode():
    """N_ff = 1 coupled flow = three scalar per-q ODEs coupled by BZ means."""
    pt = synth.Point(t=1.0, tp=-0.15, U=2.0, Lq=6, Lk=12, shells=0, mu=-0.3)
    U, T0, T1, n = 2.0, 10.0, 0.5, 40
    r = flow_rk4(pt, T0, T1, n, Xmax=1e9)

    def f(T, y):
        P, C, D = y
        chi = bubbles(pt, T, "dot")
        pp, ph = chi[0, :, 0, 0], chi[1, :, 0, 0]
        VP = U - P + C.mean() + D.mean()
        VC = U - P.mean() + C + D.mean()
        VD = U - P.mean() + C.mean() + D
        return np.stack([VP * pp * VP, -VC * ph * VC, 2 * VD * ph * VD - 2 * VC * ph * VD])

    y = np.zeros((3, 36))
    s, h = math.log(T0), (math.log(T1) - math.log(T0)) / n
    g = lambda sv, yv: math.exp(sv) * f(math.exp(sv), yv)
    for i in range(n):
        k1 = g(s, y)
        k2 = g(s + h / 2, y + h / 2 * k1)
        k3 = g(s + h / 2, y + h / 2 * k2)
        k4 = g(s + h, y + h * k3)
        y = y + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        s += h
    np.testing.assert_allclose(r.X[:, :, 0, 0], y, atol=1e-13)


def test_halffilling_flow_is_sdw_and_integrators_agree():
    """t'=0 at half filling: the magnetic channel (C) diverges at (pi,pi) with
    s-wave symmetry (the SDW regime of Sec. 4); RK4 and adaptive DOPRI5
    critical scales agree to 1%."""
    w = synth.cfg1()
    pt = w.points[0]
    r = flow_rk4(pt, w.T0, w.Tmin, w.nsteps, w.Xmax)
    assert r.status == STATUS_DIVERGED
    assert r.channel == "C" and r.irrep == "A1"
    assert r.q_index == 0           # q = (-pi, -pi) = (pi, pi)
    assert 0.1 < r.Tc < 0.5
    r2 = flow_dopri5(pt, w.T0, w.Tmin, w.Xmax, rtol=1e-7, atol=1e-9)
    assert r2.status == STATUS_DIVERGED and r2.channel == "C"
    assert abs(r2.Tc / r.Tc - 1) < 0.01


def test_nonfinite_state_stops_flow():
    pt = synth.small_point(Lq=6, Lk=8, shells=0)
    X0 = np.zeros((3, 36, 1, 1))
    X0[1, 3, 0, 0] = np.nan
    r = flow_rk4(pt, 10.0, 0.1, 10, 20.0, X0=X0)
    assert r.status == STATUS_NONFINITE and r.n_steps == 1


def test_resume_equals_uninterrupted():
    pt = synth.small_point(Lq=6, Lk=8, shells=1)
    full = flow_rk4(pt, 10.0, 0.5, 8, 1e9)
    h = (math.log(0.5) - math.log(10.0)) / 8
    T_mid = math.exp(math.log(10.0) + 4 * h)
    first = flow_rk4(pt, 10.0, T_mid, 4, 1e9)
    second = flow_rk4(pt, T_mid, 0.5, 4, 1e9, X0=first.X)
    np.testing.assert_allclose(second.X, full.X, rtol=1e-13, atol=1e-15)


def test_classify_picks_argmax_and_irrep():
    ff = FormFactors(1)
    X = np.zeros((3, 4, 5, 5))
    X[0, 2, 2, 2] = -30.0          # d_x2-y2 pairing (form factor 2, irrep B1)
    X[1, 1, 0, 0] = 10.0
    assert classify(X, ff) == ("P", 2, "B1")


def _dopri5_local_errors(hs):
    """Local errors of one Dormand-Prince step of y' = y cos(s) (exact solution
    y = exp(sin s - sin s0)) for each step size: fifth-order solution, the
    fourth-order solution X5 - err, and the embedded estimate itself."""
    import oracle.flow as oflow
    s0 = 0.3
    g = lambda s, y: y * math.cos(s)
    y0 = np.array([1.0])
    out = []
    for h in hs:
        y5, err, _ = oflow.dopri5_step(g, s0, y0, h, g(s0, y0))
        exact = math.exp(math.sin(s0 + h) - math.sin(s0))
        out.append((abs(y5[0] - exact), abs(y5[0] - err[0] - exact), abs(err[0])))
    return np.array(out)


def _orders(errs):
    return np.log2(errs[:-1] / errs[1:])


def test_dopri5_step_orders():
    """The embedded pair has local errors O(h^6) (fifth-order solution) and
    O(h^5) (fourth-order solution), so the error estimate scales as h^5."""
    e = _dopri5_local_errors([0.2, 0.1, 0.05, 0.025])
    o5, o4, oe = (_orders(e[:, i]) for i in range(3))
    assert np.all(o5 > 5.6), o5          # -> 6
    assert np.all(np.abs(o4 - 5.0) < 0.35), o4
    assert np.all(np.abs(oe - 5.0) < 0.35), oe


def test_dopri5_order_pin_catches_a_wrong_weight(monkeypatch):
    """A planted mistake in one fourth-order weight (the oracle's tableau)
    breaks the order of the error estimate."""
    import oracle.flow as oflow
    bad = list(oflow.DP_B4)
    bad[3] = 393 / 641
    monkeypatch.setattr(oflow, "DP_B4", bad)
    e = _dopri5_local_errors([0.2, 0.1, 0.05, 0.025])
    assert not np.all(np.abs(_orders(e[:, 2]) - 5.0) < 0.35)


def test_dopri5_decoupled_flow_is_rpa_ladder():
    """The adaptive flow at tight tolerances reproduces the closed-form RPA
    ladders of the decoupled channels (independently of RK4)."""
    pt = synth.Point(t=1.0, tp=-0.1, U=2.0, Lq=6, Lk=16, shells=0, mu=-0.2)
    T0, T1 = 10.0, 0.3
    r = flow_dopri5(pt, T0, T1, Xmax=1e9, rtol=1e-11, atol=1e-13, no_cross=True)
    assert r.status == STATUS_REACHED_TMIN
    P, C, D = r.X[:, :, 0, 0]
    VP, VC, W = _rpa(pt, T0, T1, 2.0)
    np.testing.assert_allclose(2.0 - P, VP, rtol=1e-8)
    np.testing.assert_allclose(2.0 + C, VC, rtol=1e-8)
    np.testing.assert_allclose(2 * (2.0 + D) - (2.0 + C), W, rtol=1e-8)
    # the error scales with the tolerance
    loose = flow_dopri5(pt, T0, T1, Xmax=1e9, rtol=1e-6, atol=1e-8, no_cross=True)
    e_tight = np.abs(2.0 + C - VC).max()
    e_loose = np.abs(2.0 + loose.X[1, :, 0, 0] - VC).max()
    assert e_loose > 10 * e_tight and e_loose < 1e-4


def test_dopri5_step_budget_and_step_sign():
    """A flow that uses up max_steps reports it (not 'reached Tmin'), and a
    first step pointing away from Tmin is rejected."""
    import oracle.flow as oflow
    pt = synth.small_point(Lq=6, Lk=8, shells=0)
    r = flow_dopri5(pt, 10.0, 0.01, 1e9, max_steps=3)
    assert r.status == oflow.STATUS_MAX_STEPS and r.n_steps <= 3
    with pytest.raises(ValueError):
        flow_dopri5(pt, 10.0, 0.01, 1e9, h0=0.1)
