"""ODE flow of the exchange propagators, critical scale and classification.

TEST INFRASTRUCTURE ONLY (plain FP64 CPU oracle; never used by the GPU path).

Paper Sec. 3 (an explicit ODE solver integrates the increments) and Sec. 4
(start far above the bandwidth, stop when the largest exchange propagator
exceeds a threshold; classify by channel, ordering vector and form-factor
symmetry).  Readings used here:
  * the flow variable is s = ln T, dX/ds = T dX/dT, integrated downwards
    from T0 with X(T0) = 0 (with regulator="omega" the scale T is the Omega
    cutoff at zero temperature, and T_c is the critical Omega);
  * fixed-step RK4 uses uniform steps in s;
  * adaptive stepping is Dormand-Prince 5(4) with its embedded error
    estimate, RMS error norm with atol + rtol max(|y|,|y_new|), step factor
    0.9 err^(-1/5) clipped to [0.2, 5];
  * a DOPRI5 flow that uses up its step budget before diverging or reaching
    Tmin ends with its own status (max steps);
  * divergence: max |X| over channels, momenta and form factors exceeds
    Xmax after an accepted step (a non-finite state also stops the flow);
  * T_c: linear interpolation of ln max|X| in s between the last two
    accepted steps to ln Xmax;
  * classification: the channel and momentum of the largest |X_mn(q)|, and
    the C4v irrep carrying most weight of the leading eigenvector of that
    channel's matrix at that momentum (ties: lowest flat index).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional

import numpy as np

from .lattice import FormFactors, transfer_points
from .rhs import rhs

CHANNELS = ("P", "C", "D")
STATUS_DIVERGED, STATUS_REACHED_TMIN, STATUS_NONFINITE, STATUS_MAX_STEPS = 1, 2, 3, 4


@dataclasses.dataclass
class FlowResult:
    status: int
    Tc: Optional[float]
    channel: Optional[str]
    q_index: Optional[int]
    irrep: Optional[str]
    max_abs_X: float
    n_rhs: int
    n_steps: int
    s_history: List[float]
    max_history: List[float]
    X: np.ndarray


def classify(X: np.ndarray, ff: FormFactors):
    """(channel, q_index, irrep) of the leading instability of state X."""
    a = np.abs(X)
    flat = int(np.argmax(a))
    ch, q, _, _ = np.unravel_index(flat, a.shape)
    M = X[ch, q]
    w, v = np.linalg.eigh(0.5 * (M + M.T))
    lead = v[:, int(np.argmax(np.abs(w)))]
    weights = {}
    for m, ir in enumerate(ff.irrep):
        weights[ir] = weights.get(ir, 0.0) + lead[m] ** 2
    irrep = max(weights, key=lambda k: weights[k])
    return CHANNELS[ch], int(q), irrep


def _max_abs(X):
    return float(np.max(np.abs(X)))


def _finish(status, s_hist, m_hist, Xmax, X, ff, n_rhs, n_steps):
    Tc = None
    ch = qi = ir = None
    if status == STATUS_DIVERGED:
        s0, s1 = s_hist[-2], s_hist[-1]
        m0, m1 = m_hist[-2], m_hist[-1]
        if m0 <= 0.0:
            sc = s1
        else:
            sc = s0 + (math.log(Xmax) - math.log(m0)) * (s1 - s0) / (math.log(m1) - math.log(m0))
        Tc = math.exp(sc)
        ch, qi, ir = classify(X, ff)
    return FlowResult(status, Tc, ch, qi, ir, m_hist[-1], n_rhs, n_steps,
                      list(s_hist), list(m_hist), X)


def flow_rk4(point, T0: float, Tmin: float, nsteps: int, Xmax: float,
             X0: Optional[np.ndarray] = None, no_cross: bool = False,
             rhs_fn: Optional[Callable] = None, regulator: str = "T") -> FlowResult:
    """Classical RK4 with nsteps uniform steps in s = ln T from T0 to Tmin."""
    ff = FormFactors(point.shells)
    f = rhs_fn or (lambda T, X: rhs(point, T, X, ff, no_cross=no_cross, regulator=regulator))
    X = np.zeros((3, transfer_points(point)[0].size, ff.nff, ff.nff)) if X0 is None else X0.copy()
    s, h = math.log(T0), (math.log(Tmin) - math.log(T0)) / nsteps

    def g(sv, Xv):
        T = math.exp(sv)
        return T * f(T, Xv)

    s_hist, m_hist, n_rhs = [s], [_max_abs(X)], 0
    for step in range(nsteps):
        k1 = g(s, X)
        k2 = g(s + 0.5 * h, X + 0.5 * h * k1)
        k3 = g(s + 0.5 * h, X + 0.5 * h * k2)
        k4 = g(s + h, X + h * k3)
        n_rhs += 4
        X = X + (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
        s = math.log(T0) + (step + 1) * h
        m = _max_abs(X)
        s_hist.append(s)
        m_hist.append(m)
        if not np.isfinite(m):
            return _finish(STATUS_NONFINITE, s_hist, m_hist, Xmax, X, ff, n_rhs, step + 1)
        if m > Xmax:
            return _finish(STATUS_DIVERGED, s_hist, m_hist, Xmax, X, ff, n_rhs, step + 1)
    return _finish(STATUS_REACHED_TMIN, s_hist, m_hist, Xmax, X, ff, n_rhs, nsteps)


# Dormand-Prince 5(4) tableau (Dormand & Prince 1980; Hairer, Norsett and
# Wanner, Solving ODE I, Table 5.2).
DP_C = [0.0, 1 / 5, 3 / 10, 4 / 5, 8 / 9, 1.0, 1.0]
DP_A = [
    [],
    [1 / 5],
    [3 / 40, 9 / 40],
    [44 / 45, -56 / 15, 32 / 9],
    [19372 / 6561, -25360 / 2187, 64448 / 6561, -212 / 729],
    [9017 / 3168, -355 / 33, 46732 / 5247, 49 / 176, -5103 / 18656],
    [35 / 384, 0.0, 500 / 1113, 125 / 192, -2187 / 6784, 11 / 84],
]
DP_B5 = [35 / 384, 0.0, 500 / 1113, 125 / 192, -2187 / 6784, 11 / 84, 0.0]
DP_B4 = [5179 / 57600, 0.0, 7571 / 16695, 393 / 640, -92097 / 339200, 187 / 2100, 1 / 40]


def dopri5_step(g: Callable, s: float, X: np.ndarray, h: float, k0: np.ndarray):
    """One Dormand-Prince 5(4) step of dX/ds = g(s, X) from (s, X) with slope
    k0 = g(s, X): returns (X5, err_vec, k) with X5 the fifth-order solution,
    err_vec = X5 - X4 the embedded error estimate (X4 the fourth-order
    solution) and k the seven stage slopes (k[6] = g(s + h, X5), first same as
    last)."""
    k = [None] * 7
    k[0] = k0
    for i in range(1, 7):
        Xi = X.copy()
        for j, a in enumerate(DP_A[i]):
            if a != 0.0:
                Xi = Xi + h * a * k[j]
        k[i] = g(s + DP_C[i] * h, Xi)
    X5 = X.copy()
    for j in range(7):
        if DP_B5[j] != 0.0:
            X5 = X5 + h * DP_B5[j] * k[j]
    err_vec = sum(h * (DP_B5[j] - DP_B4[j]) * k[j] for j in range(7))
    return X5, err_vec, k


def flow_dopri5(point, T0: float, Tmin: float, Xmax: float, rtol: float = 1e-7,
                atol: float = 1e-9, h0: Optional[float] = None, max_steps: int = 100000,
                X0: Optional[np.ndarray] = None, no_cross: bool = False,
                rhs_fn: Optional[Callable] = None, regulator: str = "T") -> FlowResult:
    """Adaptive Dormand-Prince 5(4) in s = ln T (FSAL), from T0 down to Tmin.

    A first step h0 must point from T0 towards Tmin (h0 < 0); max_steps bounds
    the attempted steps, and a flow that uses them up before reaching Tmin or
    diverging ends with STATUS_MAX_STEPS."""
    ff = FormFactors(point.shells)
    f = rhs_fn or (lambda T, X: rhs(point, T, X, ff, no_cross=no_cross, regulator=regulator))
    X = np.zeros((3, transfer_points(point)[0].size, ff.nff, ff.nff)) if X0 is None else X0.copy()
    s, s_end = math.log(T0), math.log(Tmin)
    if h0 is not None and not h0 * (s_end - s) > 0.0:
        raise ValueError("h0 must point from T0 towards Tmin")
    h = h0 if h0 is not None else (s_end - s) / 200.0

    def g(sv, Xv):
        T = math.exp(sv)
        return T * f(T, Xv)

    s_hist, m_hist = [s], [_max_abs(X)]
    k0 = g(s, X)
    n_rhs, n_acc = 1, 0
    for _ in range(max_steps):
        if s + h < s_end:
            h = s_end - s
        X5, err_vec, k = dopri5_step(g, s, X, h, k0)
        n_rhs += 6
        sc = atol + rtol * np.maximum(np.abs(X), np.abs(X5))
        err = float(np.sqrt(np.mean((err_vec / sc) ** 2)))
        if not np.isfinite(err):
            s_hist.append(s + h)
            m_hist.append(float("nan"))
            return _finish(STATUS_NONFINITE, s_hist, m_hist, Xmax, X5, ff, n_rhs, n_acc)
        if err <= 1.0:
            s = s + h
            X = X5
            k0 = k[6]
            n_acc += 1
            m = _max_abs(X)
            s_hist.append(s)
            m_hist.append(m)
            if m > Xmax:
                return _finish(STATUS_DIVERGED, s_hist, m_hist, Xmax, X, ff, n_rhs, n_acc)
            if s <= s_end + 1e-15:
                return _finish(STATUS_REACHED_TMIN, s_hist, m_hist, Xmax, X, ff, n_rhs, n_acc)
        fac = 5.0 if err == 0.0 else min(5.0, max(0.2, 0.9 * err ** (-0.2)))
        h = h * fac
    return _finish(STATUS_MAX_STEPS, s_hist, m_hist, Xmax, X, ff, n_rhs, n_acc)
