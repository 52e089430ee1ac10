"""Form-factor projected fermionic loops chi^pp, chi^ph and their scale derivatives.

TEST INFRASTRUCTURE ONLY (plain FP64 CPU oracle; never used by the GPU path).

Paper: eqn. chis (Sec. 2.4) defines
    chi^pp_mn(l) = int dp G(l/2 + p) G(l/2 - p) f_m(p) f_n(p),
    chi^ph_mn(l) = int dp G(p + l/2) G(p - l/2) f_m(p) f_n(p),
with int dp = T sum_{Matsubara n} (1/N_k) sum_p at zero bosonic frequency
(frequency dependence dropped, Sec. 2.3).  The regulator here is the
temperature: G(i w, eps) = 1/(i w - eps) unrescaled, and the "dot" of the
flow (Fig. diags-fleq: a scale derivative is implicit on closed loops) is
d/dT of the loop.

Per (q, p), with eps1 = eps(p + q/2), eps2 = eps(p - q/2) (the pp pair
eps(q/2 + p), eps(q/2 - p) is the same pair because eps is even),
a = eps1/T, b = eps2/T, the Matsubara sums are the textbook closed forms
    L^ph = T sum_n G(i w_n, eps1) G(i w_n, eps2)
         = (n_F(eps1) - n_F(eps2))/(eps1 - eps2)
         = -(1/4T) sinhc((a-b)/2) sech(a/2) sech(b/2),
    L^pp = T sum_n G(i w_n, eps1) G(-i w_n, eps2)
         = (1 - n_F(eps1) - n_F(eps2))/(eps1 + eps2)
         = +(1/4T) sinhc((a+b)/2) sech(a/2) sech(b/2),
and differentiating at fixed energies,
    dL/dT = (L/T) [ (a/2) tanh(a/2) + (b/2) tanh(b/2) - x coth x ],
with x = (a-b)/2 (ph) or (a+b)/2 (pp) and x coth x = 1 at x = 0.
L is evaluated in the log domain so that no intermediate overflows; the
bracket is split into its exact linear part and small one-signed tails, so
that exponentially small derivatives keep their relative accuracy.

Omega-cutoff regulator (regulator="omega"; Sec. 3 names the Omega cutoff of
Husemann and Salmhofer, with the self-energy neglected, as the regulator of
its runs): at T = 0
    G(i w, eps) = chi(w) / (i w - eps),   chi(w) = w^2 / (w^2 + Om^2),
the Matsubara sum becomes int dw/2pi and the dot of the flow is d/dOm (the
scale argument of these functions is then Om).  Writing
1/((iw-a)(iw-b)) = [1/(iw-a) - 1/(iw-b)]/(a-b) and keeping the part of
1/(iw-a) that is even in w, -a/(w^2+a^2),
    L^ph = -(I(eps1) - I(eps2))/(eps1 - eps2),
    L^pp = +(I(eps1) + I(eps2))/(eps1 + eps2),
    I(a) = int dw/2pi chi(w)^2 a/(w^2+a^2) = a (Om + 2|a|) / (4 (Om + |a|)^2)
(partial fractions in w^2), and the flow derivative replaces I by
dI/dOm = -a (Om + 3|a|) / (4 (Om + |a|)^3).
"""
from __future__ import annotations

import numpy as np

from .lattice import FormFactors, dispersion, k_grid, transfer_points

LN2 = np.log(2.0)


def _ln_sinhc_tail(x):
    """log(sinh(x)/x) - |x|: the part left after the linear term |x|."""
    x = np.abs(np.asarray(x, dtype=float))
    out = np.empty_like(x)
    small = x < 1e-3
    xs = x[small]
    out[small] = np.log1p(xs * xs / 6.0 + xs ** 4 / 120.0) - xs
    xl = x[~small]
    out[~small] = np.log1p(-np.exp(-2.0 * xl)) - np.log(2.0 * xl)
    return out


def _ln_cosh_tail(y):
    """log(cosh(y)) - |y| = log1p(exp(-2|y|)) - log 2."""
    return np.log1p(np.exp(-2.0 * np.abs(y))) - LN2


def _x_and_linear_part(a, b, channel):
    """x of the channel and the exact value of |x| - |a|/2 - |b|/2.

    ph: x = (a - b)/2, pp: x = (a + b)/2.  |x| equals |a|/2 + |b|/2 or
    | |a|/2 - |b|/2 | depending on the signs, so the linear part is exactly
    0 or -2 min(|a|, |b|)/2.
    """
    if channel == "ph":
        x, cancel = 0.5 * (a - b), (a * b >= 0)
    elif channel == "pp":
        x, cancel = 0.5 * (a + b), (a * b < 0)
    else:
        raise ValueError(channel)
    lin = np.where(cancel, -np.minimum(np.abs(a), np.abs(b)), 0.0)
    return x, lin


def loop(eps1, eps2, T, channel: str):
    """L^X(eps1, eps2; T) for X in {'ph', 'pp'}."""
    a = np.asarray(eps1, dtype=float) / T
    b = np.asarray(eps2, dtype=float) / T
    x, lin = _x_and_linear_part(a, b, channel)
    sign = -1.0 if channel == "ph" else 1.0
    # log of sinhc(x) sech(a/2) sech(b/2) with the linear parts taken exactly
    ln = lin + _ln_sinhc_tail(x) - _ln_cosh_tail(0.5 * a) - _ln_cosh_tail(0.5 * b)
    return sign * np.exp(ln) / (4.0 * T)


def loop_dot(eps1, eps2, T, channel: str):
    """dL^X/dT at fixed energies: (L/T) [(a/2) tanh(a/2) + (b/2) tanh(b/2) - x coth x].

    With A = |a|/2, B = |b|/2, X = |x| (each term is even), y tanh y =
    y - 2y/(e^{2y}+1) and x coth x = x + 2x/(e^{2x}-1), so the bracket is
    (A + B - X) - 2A/(e^{2A}+1) - 2B/(e^{2B}+1) - 2X/expm1(2X), whose
    linear part is exact (see _x_and_linear_part) and whose remaining terms
    share one sign: exponentially small derivatives keep relative accuracy.
    """
    a = np.asarray(eps1, dtype=float) / T
    b = np.asarray(eps2, dtype=float) / T
    x, lin = _x_and_linear_part(a, b, channel)
    A, B, X = 0.5 * np.abs(a), 0.5 * np.abs(b), np.abs(x)
    with np.errstate(over="ignore"):
        tail_a = 2.0 * A / (np.exp(2.0 * A) + 1.0)
        tail_b = 2.0 * B / (np.exp(2.0 * B) + 1.0)
    small = X < 1e-8
    Xs = np.where(small, 1.0, X)
    with np.errstate(over="ignore"):
        tail_x = np.where(small, 1.0 - X, 2.0 * Xs / np.expm1(2.0 * Xs))
    bracket = -lin - tail_a - tail_b - tail_x
    return loop(eps1, eps2, T, channel) * bracket / T


# ------------------------------------------------------------ Omega cutoff
def omega_I(a, Om, dot: bool = False):
    """I(a) = int dw/2pi chi(w)^2 a/(w^2+a^2), or dI/dOm (dot=True); odd in a."""
    a = np.asarray(a, dtype=float)
    u = Om + np.abs(a)
    if dot:
        return -a * (Om + 3.0 * np.abs(a)) / (4.0 * u ** 3)
    return a * (Om + 2.0 * np.abs(a)) / (4.0 * u * u)


def _omega_divided_difference(a, b, Om, dot: bool):
    """(I(a) - I(b)) / (a - b) (or of dI/dOm) without cancellation.

    I(a) = sgn(a) G(|a|) with G rational in u = Om + |a|:
        G      = 1/2 - 3 Om/(4u) + Om^2/(4u^2),
        dG/dOm = -3/(4u) + 5 Om/(4u^2) - Om^2/(2u^3),
    so for a, b of one sign (u, v = Om + |a|, Om + |b|) the difference
    quotient is the exact rational expression below; for opposite signs
    I(a) and I(b) have opposite signs and the plain quotient does not cancel.
    """
    a = np.asarray(a, dtype=float)
    b = np.asarray(b, dtype=float)
    u, v = Om + np.abs(a), Om + np.abs(b)
    if dot:
        same = 3.0 / (4.0 * u * v) - 5.0 * Om * (u + v) / (4.0 * u * u * v * v) \
            + Om * Om * (u * u + u * v + v * v) / (2.0 * u ** 3 * v ** 3)
    else:
        same = 3.0 * Om / (4.0 * u * v) - Om * Om * (u + v) / (4.0 * u * u * v * v)
    one_sign = a * b >= 0
    d = np.where(one_sign, 1.0, a - b)
    opposite = (omega_I(a, Om, dot) - omega_I(b, Om, dot)) / d
    return np.where(one_sign, same, opposite)


def loop_omega(eps1, eps2, Om, channel: str, dot: bool = False):
    """L^X at T = 0 with the Omega cutoff (dot=True: dL^X/dOm at fixed energies)."""
    if channel == "ph":
        return -_omega_divided_difference(eps1, eps2, Om, dot)
    if channel == "pp":
        return _omega_divided_difference(eps1, -np.asarray(eps2, dtype=float), Om, dot)
    raise ValueError(channel)


def loop_omega_dot(eps1, eps2, Om, channel: str):
    return loop_omega(eps1, eps2, Om, channel, dot=True)


REGULATORS = ("T", "omega")


def bubbles(point, T: float, which: str = "dot", ff: FormFactors | None = None,
            q_index=None, regulator: str = "T"):
    """chi (which='value') or its scale derivative (which='dot') on the transfer grid.

    Returns an array [2][nq_sel][nff][nff] ordered (pp, ph).  The loop
    integral is the literal pairwise grid average
        chi_mn(q) = (1/N_k) sum_p L(eps(p+q/2), eps(p-q/2)) f_m(p) f_n(p)
    (discretised eqn. chis: p on the unshifted fine grid, energies taken at
    p +- q/2, form factors at p).  regulator="T": the scale T is the
    temperature (d/dT); regulator="omega": T = 0 and the scale is the
    Omega cutoff (d/dOm).
    """
    if regulator not in REGULATORS:
        raise ValueError(regulator)
    ff = ff or FormFactors(point.shells)
    qx, qy, _ = transfer_points(point)
    if q_index is not None:
        qx, qy = qx[q_index], qy[q_index]
    px, py = k_grid(point.Lk)
    F = ff.values(px, py)                         # [nff, Nk]
    Nk = px.size
    if regulator == "omega":
        fn = loop_omega_dot if which == "dot" else loop_omega
    else:
        fn = loop_dot if which == "dot" else loop
    out = np.empty((2, qx.size, ff.nff, ff.nff))
    for i in range(qx.size):
        e1 = dispersion(px + 0.5 * qx[i], py + 0.5 * qy[i], point.t, point.tp, point.mu)
        e2 = dispersion(px - 0.5 * qx[i], py - 0.5 * qy[i], point.t, point.tp, point.mu)
        for c, ch in enumerate(("pp", "ph")):
            w = fn(e1, e2, T, ch)
            out[c, i] = (F * w) @ F.T / Nk
    return out
