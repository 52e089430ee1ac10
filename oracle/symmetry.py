"""Point-group (C4v) covariance of the exchange propagators on the transfer grid.

TEST INFRASTRUCTURE ONLY (plain FP64 CPU oracle; never used by the GPU path).

The lattice symmetries of Sec. 3 (the 8 operations of C4v, under which the
dispersion and the unshifted fine grid are invariant) act on a state X(q)
given in the form-factor basis.  With the form factors taken at the loop
momentum p and the energies at p +- q/2 (discretised eqn. chis), the
substitution p = h^-1 (p'' - G/2) in the grid sum gives, for an operation h
with h q = q' + G (q' on the transfer grid, G a reciprocal-lattice vector in
{0, 2 pi}^2, which arises when h q lands on the zone edge +pi):

    X(q) = T X(q') T^T,    f_m(h^-1 (k - G/2)) = sum_n T_mn f_n(k).

The loops obey this for any point (they are invariant lattice sums); a state
that obeys it (a symmetric state, e.g. every state of a flow started at zero)
gives increments that obey it, because the projections and the products are
covariant as well.  The tests pin both statements: the loops against their
own grid sums, the increment of a symmetrised random state for its defect.
"""
from __future__ import annotations

import numpy as np

from .lattice import FormFactors

# The eight operations of C4v as integer matrices acting on (qx, qy).
C4V_OPS = [
    np.array([[1, 0], [0, 1]]), np.array([[-1, 0], [0, 1]]),
    np.array([[1, 0], [0, -1]]), np.array([[-1, 0], [0, -1]]),
    np.array([[0, 1], [1, 0]]), np.array([[0, -1], [1, 0]]),
    np.array([[0, 1], [-1, 0]]), np.array([[0, -1], [-1, 0]]),
]


def ff_transform(ff: FormFactors, h: np.ndarray, g) -> np.ndarray:
    """T[m, n] with f_m(h^-1 (k - G/2)) = sum_n T[m, n] f_n(k), G/2 = pi (g[0], g[1]).

    The form factors are orthonormal under the BZ average and their span is
    closed under the operation (each shell's bonds map onto the shell, the
    half shift multiplies plane waves by signs), so T is the overlap on a
    grid fine enough to integrate the products exactly (components <= 4 < 8).
    """
    L = 16
    k1 = 2 * np.pi * np.arange(L) / L
    kx, ky = np.meshgrid(k1, k1, indexing="ij")
    kx, ky = kx.ravel(), ky.ravel()
    hinv = h.T                                        # h is orthogonal
    ux, uy = kx - np.pi * g[0], ky - np.pi * g[1]
    ax = hinv[0, 0] * ux + hinv[0, 1] * uy
    ay = hinv[1, 0] * ux + hinv[1, 1] * uy
    A = ff.values(ax, ay)                             # f_m(h^-1 (k - G/2))
    B = ff.values(kx, ky)
    T = A @ B.T / kx.size
    if np.abs(A - T @ B).max() > 1e-12:
        raise ValueError("form-factor span not closed under the operation")
    # the overlaps are integers (each form factor maps to +- another): take
    # them exactly, so that T X T^T only moves and negates entries
    Ti = np.round(T)
    if np.abs(T - Ti).max() < 1e-12:
        T = Ti
    return T


def image(Lq: int, h: np.ndarray, q: int):
    """(q', g) with h q = q' + 2 pi g on the grid q_i = 2 pi (i - Lq/2)/Lq."""
    half = Lq // 2
    a, b = q // Lq - half, q % Lq - half
    a2 = h[0, 0] * a + h[0, 1] * b
    b2 = h[1, 0] * a + h[1, 1] * b
    gx = 1 if a2 >= half else 0
    gy = 1 if b2 >= half else 0
    a2 -= gx * Lq
    b2 -= gy * Lq
    return (a2 + half) * Lq + (b2 + half), (gx, gy)


def law(ff: FormFactors, Lq: int):
    """For every operation o and momentum q: (q', T) of X(q) = T X(q') T^T."""
    cache = {}
    out = []
    for o, h in enumerate(C4V_OPS):
        row = []
        for q in range(Lq * Lq):
            q2, g = image(Lq, h, q)
            if (o, g) not in cache:
                cache[(o, g)] = ff_transform(ff, h, g)
            row.append((q2, cache[(o, g)]))
        out.append(row)
    return out


def defect(X: np.ndarray, ff: FormFactors, Lq: int) -> float:
    """max |X(q) - T X(q') T^T| over operations, momenta and the leading axes of X[..., nq, nff, nff]."""
    worst = 0.0
    for row in law(ff, Lq):
        for q, (q2, T) in enumerate(row):
            d = X[..., q, :, :] - T @ X[..., q2, :, :] @ T.T
            worst = max(worst, float(np.abs(d).max()))
    return worst


def symmetrize(X: np.ndarray, ff: FormFactors, Lq: int) -> np.ndarray:
    """The group average (1/8) sum_h T X(q') T^T of a state X[..., nq, nff, nff]."""
    out = np.zeros_like(X)
    for row in law(ff, Lq):
        for q, (q2, T) in enumerate(row):
            out[..., q, :, :] += T @ X[..., q2, :, :] @ T.T
    return out / len(C4V_OPS)
