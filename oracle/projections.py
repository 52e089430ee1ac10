"""Inter-channel projections V^P, V^C, V^D (step i of the TUfRG increment).

TEST INFRASTRUCTURE ONLY (plain FP64 CPU oracle; never used by the GPU path).

Paper: eqns. proj_VP, proj_VC, proj_VD (Sec. 2.4) with the projection
rules eqns. proj-P, proj-C, proj-D (Sec. 2.3), the channel decomposition
eqn. simple-deco, the exchange parametrisations eqns. app-PhiP/C/D, and the
position-space form eqn. proj_pos.

Derivation used here (written out so it can be checked by eye).
Put the exchange propagator in bond space,
    X_{R1R2}(u) = sum_{m'n'} c_{m'R1} c_{n'R2} X_{m'n'}(u),
so that Phi^X_{u,k,k'} = sum_{R1R2} exp(-i k.R1) exp(-i k'.R2) X_{R1R2}(u).
Periodicity of V in each fermion momentum makes X quasi-periodic,
X_{R1R2}(u + G) = exp(i G.(R1+R2)/2) X_{R1R2}(u), so the gauged function
exp(-i u.(R1+R2)/2) X_{R1R2}(u) is periodic and has Fourier coefficients
    Yhat_{R1R2}(W) = (1/N_q) sum_u X_{R1R2}(u) exp(i u.(W - (R1+R2)/2)),  W in Z^2
(the "Fourier series" of the exchange propagator used with the stored
projection tensors in the appendix on symmetries; on the uniform grid this
is the DFT, i.e. trigonometric interpolation of the propagator; on a
non-uniform transfer mesh, Sec. 4, the sum over u carries the quadrature
weights of the mesh cells instead of 1/N_q).
Substituting into the projection rules and doing the k, k' integrals with
int dk f_m(k) exp(i k.R) = c_{m,R} gives two kernels:
    K1[X]_mn(l) = sum_{R1,R2,W} exp(-i l.(R1+R2)/2) c_{m,R2-W} c_{n,R1-W} Yhat_{R1R2}(W)
    K2[X]_mn(l) = sum_{R1,R2,W} exp(-i l.(R1-R2)/2) c_{m,-W} c_{n,W-R1-R2} Yhat_{R1R2}(W)
and the six cross projections
    P[Phi^C] = K1[C]            P[Phi^D]  = K1[D] diag(pi)
    C[Phi^SC] = K1[P]           C[Phi^D]  = K2[D]
    D[Phi^SC] = K2[P] diag(pi)  D[Phi^C]  = K2[C]
(pi_n = parity of f_n; c_{n,-R} = pi_n c_{n,R}).  The K1 form is eqn.
proj_pos with its R3 running over the half-shifted lattice Z^2 - (R1+R2)/2.
The bare onsite interaction projects to U delta_m0 delta_n0 in every channel
because only f_0 = 1 has a non-zero BZ mean.  All results are real at zero
bosonic frequency (appendix on symmetries); the imaginary part is rounding
and is dropped after a check.
"""
from __future__ import annotations

import itertools

import numpy as np

from .lattice import FormFactors, transfer_points


def bond_space(X: np.ndarray, ff: FormFactors) -> np.ndarray:
    """X[nq, m', n'] -> X_{R1R2}[nq, b1, b2] = sum c_{m'b1} c_{n'b2} X_{m'n'}."""
    return np.einsum("ma,qmn,nb->qab", ff.c, X.astype(complex), ff.c, optimize=True)


def w_range(ff: FormFactors):
    """Integer vectors W that can pair two bonds of the set: |W_x|, |W_y| <= 2 rmax."""
    r = 2 * ff.rmax
    return list(itertools.product(range(-r, r + 1), repeat=2))


def gauged_fourier(X: np.ndarray, ff: FormFactors, point) -> dict:
    """Yhat_{R1R2}(W) for every W of w_range: {W: array [b1, b2] complex}.

    Yhat_{R1R2}(W) = sum_u w_u X_{R1R2}(u) exp(i u.(W - (R1+R2)/2)), the
    quadrature of the Fourier integral over the zone with the weights w_u of
    the transfer momenta: 1/N_q on the uniform grid (the DFT), the cell area
    fractions on a non-uniform mesh.
    """
    if point.Lq <= 4 * ff.rmax:
        raise ValueError("transfer grid too coarse: need Lq > 4 * largest bond component")
    qx, qy, w = transfer_points(point)
    XB = bond_space(X, ff)
    B = np.array(ff.bonds, dtype=float)
    gx = 0.5 * (B[:, None, 0] + B[None, :, 0])
    gy = 0.5 * (B[:, None, 1] + B[None, :, 1])
    G = XB * np.exp(-1j * (qx[:, None, None] * gx[None] + qy[:, None, None] * gy[None]))
    Ws = w_range(ff)
    ph = np.exp(1j * (np.outer([v[0] for v in Ws], qx) + np.outer([v[1] for v in Ws], qy)))
    if getattr(point, "mesh", None) is None:
        Yall = ph @ G.reshape(qx.size, -1) / qx.size
    else:
        Yall = ph @ (w[:, None] * G.reshape(qx.size, -1))
    Yall = Yall.reshape(len(Ws), ff.nff, ff.nff)
    return {W: Yall[i] for i, W in enumerate(Ws)}


def _coef_vector(ff: FormFactors, R) -> np.ndarray:
    """[c_{m,R} for every m]; zero vector when R is not a bond."""
    return ff.coefficient_column(R)


def kernel_K1(X: np.ndarray, ff: FormFactors, point, l_index=None) -> np.ndarray:
    """K1[X]_mn(l) at the transfer momenta (or at the momenta l_index): [nl, nff, nff] complex.

    K1[X]_mn(l) = sum_{R1,R2} exp(-i l.(R1+R2)/2) sum_W c_{m,R2-W} c_{n,R1-W} Yhat_{R1R2}(W).
    """
    Y = gauged_fourier(X, ff, point)
    qx, qy, _ = transfer_points(point)
    if l_index is not None:
        qx, qy = qx[l_index], qy[l_index]
    out = np.zeros((qx.size, ff.nff, ff.nff), dtype=complex)
    for b1, R1 in enumerate(ff.bonds):
        for b2, R2 in enumerate(ff.bonds):
            M = np.zeros((ff.nff, ff.nff), dtype=complex)
            for W, Yw in Y.items():
                cm = _coef_vector(ff, (R2[0] - W[0], R2[1] - W[1]))
                cn = _coef_vector(ff, (R1[0] - W[0], R1[1] - W[1]))
                if np.any(cm) and np.any(cn):
                    M += Yw[b1, b2] * np.outer(cm, cn)
            if np.any(M):
                ph = np.exp(-0.5j * (qx * (R1[0] + R2[0]) + qy * (R1[1] + R2[1])))
                out += ph[:, None, None] * M[None]
    return out


def kernel_K2(X: np.ndarray, ff: FormFactors, point, l_index=None) -> np.ndarray:
    """K2[X]_mn(l) at the transfer momenta (or at the momenta l_index): [nl, nff, nff] complex.

    K2[X]_mn(l) = sum_{R1,R2} exp(-i l.(R1-R2)/2) sum_W c_{m,-W} c_{n,W-R1-R2} Yhat_{R1R2}(W).
    """
    Y = gauged_fourier(X, ff, point)
    qx, qy, _ = transfer_points(point)
    if l_index is not None:
        qx, qy = qx[l_index], qy[l_index]
    out = np.zeros((qx.size, ff.nff, ff.nff), dtype=complex)
    for b1, R1 in enumerate(ff.bonds):
        for b2, R2 in enumerate(ff.bonds):
            M = np.zeros((ff.nff, ff.nff), dtype=complex)
            for W, Yw in Y.items():
                cm = _coef_vector(ff, (-W[0], -W[1]))
                cn = _coef_vector(ff, (W[0] - R1[0] - R2[0], W[1] - R1[1] - R2[1]))
                if np.any(cm) and np.any(cn):
                    M += Yw[b1, b2] * np.outer(cm, cn)
            if np.any(M):
                ph = np.exp(-0.5j * (qx * (R1[0] - R2[0]) + qy * (R1[1] - R2[1])))
                out += ph[:, None, None] * M[None]
    return out


def _real(Z: np.ndarray, what: str) -> np.ndarray:
    scale = max(1.0, float(np.abs(Z).max()))
    im = float(np.abs(Z.imag).max()) if Z.size else 0.0
    if im > 1e-11 * scale:
        raise AssertionError(f"{what}: imaginary residue {im:.3e} (scale {scale:.3e})")
    return Z.real.copy()


def cross_projections(point, X: np.ndarray, ff: FormFactors | None = None, l_index=None) -> dict:
    """The six cross projections of eqns. proj_VP/VC/VD for state X[3][nq][nff][nff].

    Keys: 'P[C]', 'P[D]', 'C[P]', 'C[D]', 'D[P]', 'D[C]' meaning e.g.
    P[C] = Phat[Phi^C].
    """
    ff = ff or FormFactors(point.shells)
    P, C, D = X
    pi = ff.parity
    K1C, K1D, K1P = (kernel_K1(Z, ff, point, l_index) for Z in (C, D, P))
    K2D, K2C, K2P = (kernel_K2(Z, ff, point, l_index) for Z in (D, C, P))
    return {
        "P[C]": _real(K1C, "P[C]"),
        "P[D]": _real(K1D * pi[None, None, :], "P[D]"),
        "C[P]": _real(K1P, "C[P]"),
        "C[D]": _real(K2D, "C[D]"),
        "D[P]": _real(K2P * pi[None, None, :], "D[P]"),
        "D[C]": _real(K2C, "D[C]"),
    }


def project(point, X: np.ndarray, ff: FormFactors | None = None,
            no_cross: bool = False, l_index=None) -> np.ndarray:
    """V[3][nq][nff][nff] = (V^P, V^C, V^D) per eqns. proj_VP, proj_VC, proj_VD.

    l_index selects the momenta l at which V is returned (all by default).
    no_cross drops every inter-channel term (decoupled channels); it is a
    test seam for closed forms, not part of the method.
    """
    ff = ff or FormFactors(point.shells)
    P, C, D = X
    if l_index is not None:
        P, C, D = P[l_index], C[l_index], D[l_index]
    nq, nff = P.shape[0], ff.nff
    bare = np.zeros((nq, nff, nff))
    bare[:, 0, 0] = point.U
    if no_cross:
        return np.stack([bare - P, bare + C, bare + D])
    k = cross_projections(point, X, ff, l_index)
    VP = bare - P + k["P[C]"] + k["P[D]"]
    VC = bare - k["C[P]"] + C + k["C[D]"]
    VD = bare - k["D[P]"] + k["D[C]"] + D
    return np.stack([VP, VC, VD])
