"""Brute-force evaluations used to pin the oracle (tiny sizes only).

These follow the paper's definitions literally and share none of the
oracle's shortcuts:
  * Matsubara sums of G(i w_n, eps) = 1/(i w_n - eps) at 40 digits (mpmath);
  * projections as double momentum sums of the projection rules
    (eqns. proj-P/C/D) applied to the channel decomposition eqn. simple-deco,
    with exchange propagators given as explicit functions of momentum.
"""
from __future__ import annotations

import itertools

import mpmath as mp
import numpy as np


# ----------------------------------------------------------------- loops
def matsubara_loop(eps1, eps2, T, channel, nmax=4000):
    """T sum_n G(i w_n, eps1) G(+-i w_n, eps2), plus the analytic tail.

    Summed symmetrically over |n| < nmax; the remainder is integrated with
    Euler-Maclaurin (mpmath.nsum with the default extrapolation).
    """
    mp.mp.dps = 40
    e1, e2, T = mp.mpf(eps1), mp.mpf(eps2), mp.mpf(T)

    def term(n):
        w = (2 * n + 1) * mp.pi * T
        g1 = 1 / (1j * w - e1)
        g2 = 1 / (1j * w - e2) if channel == "ph" else 1 / (-1j * w - e2)
        return g1 * g2

    s = mp.nsum(term, [-mp.inf, mp.inf])
    return T * s


def matsubara_loop_dot(eps1, eps2, T, channel, h=None):
    """d/dT of the Matsubara sum by a 4-point central difference at 40 digits."""
    mp.mp.dps = 40
    T = mp.mpf(T)
    h = h if h is not None else T * mp.mpf("1e-8")
    f = lambda x: matsubara_loop(eps1, eps2, x, channel)
    return (-f(T + 2 * h) + 8 * f(T + h) - 8 * f(T - h) + f(T - 2 * h)) / (12 * h)


# ----------------------------------------------------------- propagators
class TrigPropagator:
    """An exchange propagator X_mn(l) defined at every momentum l.

    X_{R1R2}(l) = exp(i l.(R1+R2)/2) sum_{|W|<=wmax} Y_{R1R2}(W) exp(-i l.W),
    X_mn(l) = sum_{R1R2} conj(c_{m,R1}) conj(c_{n,R2}) X_{R1R2}(l).
    The coefficients are random with Y_{R1R2}(W)* = Y_{-R1,-R2}(-W), which
    makes X_mn(l) real.  The half-bond phase makes the channel function
    periodic in every fermion momentum (checked in the tests).
    """

    def __init__(self, ff, wmax, seed, symmetric=True):
        rng = np.random.default_rng(seed)
        self.ff = ff
        self.Ws = list(itertools.product(range(-wmax, wmax + 1), repeat=2))
        nb = ff.nff
        Y = rng.standard_normal((len(self.Ws), nb, nb)) + 1j * rng.standard_normal((len(self.Ws), nb, nb))
        neg_b = [ff.bonds.index((-b[0], -b[1])) for b in ff.bonds]
        neg_w = [self.Ws.index((-w[0], -w[1])) for w in self.Ws]
        Yh = 0.5 * (Y + np.conj(Y[neg_w][:, neg_b][:, :, neg_b]))
        if symmetric:
            Yh = 0.5 * (Yh + np.swapaxes(Yh, 1, 2))
        self.Y = Yh / len(self.Ws)
        self.B = np.array(ff.bonds, dtype=float)

    def __call__(self, lx, ly):
        """X_mn at momenta (lx, ly) (arrays of equal shape): [..., nff, nff] real."""
        lx = np.asarray(lx, dtype=float)
        ly = np.asarray(ly, dtype=float)
        W = np.array(self.Ws, dtype=float)
        eW = np.exp(-1j * (lx[..., None] * W[:, 0] + ly[..., None] * W[:, 1]))   # [..., nW]
        nb = self.Y.shape[1]
        XB = (eW @ self.Y.reshape(len(self.Ws), nb * nb)).reshape(eW.shape[:-1] + (nb, nb))
        gx = 0.5 * (self.B[:, None, 0] + self.B[None, :, 0])
        gy = 0.5 * (self.B[:, None, 1] + self.B[None, :, 1])
        XB = XB * np.exp(1j * (lx[..., None, None] * gx + ly[..., None, None] * gy))
        cc = np.conj(self.ff.c)
        Xmn = cc @ XB @ cc.T
        assert np.abs(Xmn.imag).max() < 1e-12 * max(1.0, np.abs(Xmn).max())
        return Xmn.real


def channel_function(ff, prop, kind, k1, k2, k3):
    """Phi^kind evaluated at (k1, k2, k3) via eqn. simple-deco and app-Phi*.

    k* are tuples (kx_array, ky_array).  kind in {'SC', 'C', 'D'}.
    """
    k4 = (k1[0] + k2[0] - k3[0], k1[1] + k2[1] - k3[1])
    if kind == "SC":
        l = (k1[0] + k2[0], k1[1] + k2[1])
        a = (0.5 * (k1[0] - k2[0]), 0.5 * (k1[1] - k2[1]))
        b = (0.5 * (k4[0] - k3[0]), 0.5 * (k4[1] - k3[1]))
    elif kind == "C":
        l = (k1[0] - k3[0], k1[1] - k3[1])
        a = (0.5 * (k1[0] + k3[0]), 0.5 * (k1[1] + k3[1]))
        b = (0.5 * (k2[0] + k4[0]), 0.5 * (k2[1] + k4[1]))
    elif kind == "D":
        l = (k3[0] - k2[0], k3[1] - k2[1])
        a = (0.5 * (k1[0] + k4[0]), 0.5 * (k1[1] + k4[1]))
        b = (0.5 * (k2[0] + k3[0]), 0.5 * (k2[1] + k3[1]))
    else:
        raise ValueError(kind)
    fa = ff.values(*a)           # [nff, ...]
    fb = ff.values(*b)
    X = prop(*l)                 # [..., nff, nff]
    return np.einsum("m...,...mn,n...->...", fa, X, fb)


def project_brute(ff, prop, onto, kind, lx, ly, Lf):
    """onto-projection (P, C or D rule) of Phi^kind at transfer momentum l.

    Double grid sum over k, k' on an Lf x Lf grid (exact for trig
    polynomials of degree < Lf).  Returns [nff, nff].
    """
    g = 2 * np.pi * np.arange(Lf) / Lf
    kx, ky, kpx, kpy = np.meshgrid(g, g, g, g, indexing="ij")
    kx, ky, kpx, kpy = (a.ravel() for a in (kx, ky, kpx, kpy))
    hx, hy = 0.5 * lx, 0.5 * ly
    if onto == "P":
        k1, k2, k3 = (hx + kx, hy + ky), (hx - kx, hy - ky), (hx - kpx, hy - kpy)
    elif onto == "C":
        k1, k2, k3 = (kx + hx, ky + hy), (kpx - hx, kpy - hy), (kx - hx, ky - hy)
    elif onto == "D":
        k1, k2, k3 = (kx + hx, ky + hy), (kpx - hx, kpy - hy), (kpx + hx, kpy + hy)
    else:
        raise ValueError(onto)
    F = channel_function(ff, prop, kind, k1, k2, k3)
    fm = ff.values(kx, ky)
    fn = ff.values(kpx, kpy)
    return (fm * F) @ fn.T / F.size


class MeshFourierPropagator(TrigPropagator):
    """The exchange propagator that a non-uniform transfer mesh represents:
    its values X_mn(u) at the mesh points give the Fourier coefficients of
    the gauged bond-space propagator by the mesh quadrature
        Y_{R1R2}(W) = sum_u w_u X_{R1R2}(u) exp(i u.(W - (R1+R2)/2)),
        X_{R1R2}(u) = sum_{m'n'} c_{m'R1} c_{n'R2} X_{m'n'}(u),
    for every |W_x|, |W_y| <= wmax, and the propagator at any momentum l is
    the series exp(i l.(R1+R2)/2) sum_W Y(W) exp(-i l.W) (the TrigPropagator
    form).  Written with explicit loops over bonds, independently of the
    oracle's transform."""

    def __init__(self, ff, qx, qy, w, Xm, wmax):
        self.ff = ff
        self.Ws = list(itertools.product(range(-wmax, wmax + 1), repeat=2))
        nb = ff.nff
        self.B = np.array(ff.bonds, dtype=float)
        Y = np.zeros((len(self.Ws), nb, nb), dtype=complex)
        for b1 in range(nb):
            for b2 in range(nb):
                xb = np.zeros(qx.size, dtype=complex)
                for m in range(nb):
                    for n in range(nb):
                        coef = ff.c[m, b1] * ff.c[n, b2]
                        if coef != 0:
                            xb += coef * Xm[:, m, n]
                gx = 0.5 * (self.B[b1, 0] + self.B[b2, 0])
                gy = 0.5 * (self.B[b1, 1] + self.B[b2, 1])
                for i, (wx, wy) in enumerate(self.Ws):
                    Y[i, b1, b2] = np.sum(w * xb * np.exp(1j * (qx * (wx - gx) + qy * (wy - gy))))
        self.Y = Y
