"""Lattice objects of the TUfRG oracle: grids, bond form factors, dispersion.

TEST INFRASTRUCTURE ONLY.  The oracle is a plain, slow FP64 CPU
implementation used by the tests and by the benchmark's CPU-baseline leg.
The GPU library never imports, links or calls anything in this package.

Conventions (paper Sec. 2.3, Sec. 3 and the appendix on smooth form factors):
  * form factors f_m(k) are real functions on the Brillouin zone (BZ),
    orthonormal under the BZ average, each tied to one bond length; the
    truncation keeps every bond up to the n-th nearest neighbour;
  * real-space coefficients are defined by f_m(k) = sum_R c_{m,R} exp(-i k.R)
    (appendix on smooth form factors); they are real for even and purely
    imaginary for odd form factors;
  * transfer momenta live on q_i = 2 pi (i - L/2)/L per axis, i.e. the zone
    [-pi, pi)^2; the fine loop grid is p_j = 2 pi j / L_k (unshifted);
  * every BZ integral is the plain grid average (1/N) sum.
"""
from __future__ import annotations

import numpy as np

SQ2 = np.sqrt(2.0)

# Bond shells by length: 0, 1, sqrt2, 2, sqrt5 (1st..4th nearest neighbours).
SHELL_BONDS = [
    [(0, 0)],
    [(1, 0), (-1, 0), (0, 1), (0, -1)],
    [(1, 1), (-1, -1), (1, -1), (-1, 1)],
    [(2, 0), (-2, 0), (0, 2), (0, -2)],
    [(2, 1), (-2, -1), (2, -1), (-2, 1), (1, 2), (-1, -2), (1, -2), (-1, 2)],
]


def _c(x):
    return np.cos(x)


def _s(x):
    return np.sin(x)


# Form factors per shell, ordered A1, B1, B2, A2, E (C4v irreps, Sec. 3
# footnote on the form-factor basis).  Each entry: (name, irrep, parity, f).
FORM_FACTORS = [
    [("s", "A1", +1, lambda kx, ky: np.ones(np.broadcast(kx, ky).shape))],
    [("s*", "A1", +1, lambda kx, ky: _c(kx) + _c(ky)),
     ("d_x2-y2", "B1", +1, lambda kx, ky: _c(kx) - _c(ky)),
     ("p_x", "E", -1, lambda kx, ky: SQ2 * _s(kx)),
     ("p_y", "E", -1, lambda kx, ky: SQ2 * _s(ky))],
    [("s_xy", "A1", +1, lambda kx, ky: 2 * _c(kx) * _c(ky)),
     ("d_xy", "B2", +1, lambda kx, ky: 2 * _s(kx) * _s(ky)),
     ("p_x'", "E", -1, lambda kx, ky: 2 * _s(kx) * _c(ky)),
     ("p_y'", "E", -1, lambda kx, ky: 2 * _c(kx) * _s(ky))],
    [("s**", "A1", +1, lambda kx, ky: _c(2 * kx) + _c(2 * ky)),
     ("d_x2-y2'", "B1", +1, lambda kx, ky: _c(2 * kx) - _c(2 * ky)),
     ("p_x''", "E", -1, lambda kx, ky: SQ2 * _s(2 * kx)),
     ("p_y''", "E", -1, lambda kx, ky: SQ2 * _s(2 * ky))],
    [("s5", "A1", +1, lambda kx, ky: SQ2 * (_c(2 * kx) * _c(ky) + _c(kx) * _c(2 * ky))),
     ("d5", "B1", +1, lambda kx, ky: SQ2 * (_c(2 * kx) * _c(ky) - _c(kx) * _c(2 * ky))),
     ("dxy5", "B2", +1, lambda kx, ky: SQ2 * (_s(2 * kx) * _s(ky) + _s(kx) * _s(2 * ky))),
     ("g", "A2", +1, lambda kx, ky: SQ2 * (_s(2 * kx) * _s(ky) - _s(kx) * _s(2 * ky))),
     ("p5a", "E", -1, lambda kx, ky: 2 * _s(2 * kx) * _c(ky)),
     ("p5b", "E", -1, lambda kx, ky: 2 * _c(kx) * _s(2 * ky)),
     ("p5c", "E", -1, lambda kx, ky: 2 * _s(kx) * _c(2 * ky)),
     ("p5d", "E", -1, lambda kx, ky: 2 * _c(2 * kx) * _s(ky))],
]

NFF_OF_SHELLS = {0: 1, 1: 5, 2: 9, 3: 13, 4: 21}


class FormFactors:
    """Truncated bond form-factor basis up to shell `shells` (0..4)."""

    def __init__(self, shells: int):
        if shells not in NFF_OF_SHELLS:
            raise ValueError("shells must be 0..4")
        self.shells = shells
        self.entries = [e for s in range(shells + 1) for e in FORM_FACTORS[s]]
        self.shell_of = np.array([s for s in range(shells + 1) for _ in FORM_FACTORS[s]])
        self.bonds = [b for s in range(shells + 1) for b in SHELL_BONDS[s]]
        self.nff = len(self.entries)
        assert self.nff == len(self.bonds) == NFF_OF_SHELLS[shells]
        self.parity = np.array([e[2] for e in self.entries], dtype=float)
        self.irrep = [e[1] for e in self.entries]
        self.names = [e[0] for e in self.entries]
        self.bond_index = {b: i for i, b in enumerate(self.bonds)}
        self.rmax = max(max(abs(b[0]), abs(b[1])) for b in self.bonds)
        self.c = self._real_space_coefficients()

    def values(self, kx, ky) -> np.ndarray:
        """f_m(k) for all m: array [nff, *shape]."""
        return np.stack([np.asarray(e[3](kx, ky), dtype=float) for e in self.entries])

    def _real_space_coefficients(self) -> np.ndarray:
        """c[m, b] with f_m(k) = sum_b c[m, b] exp(-i k . R_b).

        Obtained by inverting the Fourier series on an 8x8 grid,
        c_{m,R} = <f_m(k) exp(+i k.R)>_BZ, which is exact for these trig
        polynomials (largest bond component 2 < 8/2).
        """
        L = 8
        k = 2 * np.pi * np.arange(L) / L
        kx, ky = np.meshgrid(k, k, indexing="ij")
        f = self.values(kx, ky)
        c = np.zeros((self.nff, self.nff), dtype=complex)
        for b, (rx, ry) in enumerate(self.bonds):
            ph = np.exp(1j * (kx * rx + ky * ry))
            c[:, b] = (f * ph).reshape(self.nff, -1).mean(axis=1)
        c[np.abs(c) < 1e-14] = 0.0
        return c

    def coefficient(self, m: int, R) -> complex:
        """c_{m,R}; zero when R is not a bond of the truncated set."""
        b = self.bond_index.get((int(R[0]), int(R[1])))
        return 0.0 if b is None else self.c[m, b]

    def coefficient_column(self, R) -> np.ndarray:
        """[c_{m,R} for every m]; the zero vector when R is not a bond."""
        b = self.bond_index.get((int(R[0]), int(R[1])))
        if b is None:
            return np.zeros(self.nff, dtype=complex)
        return self.c[:, b]


def q_grid(Lq: int):
    """Transfer grid q_i = 2 pi (i - Lq/2)/Lq per axis; flat index ix*Lq + iy."""
    q1 = 2 * np.pi * (np.arange(Lq) - Lq // 2) / Lq
    qx, qy = np.meshgrid(q1, q1, indexing="ij")
    return qx.ravel(), qy.ravel()


def transfer_points(point):
    """Transfer momenta of a point and their quadrature weights: (qx, qy, w).

    The uniform grid q_grid(point.Lq) with weights 1/N_q, or the point's
    non-uniform mesh (point.mesh: arrays qx, qy in [-pi, pi) and weights w,
    the fractions of the zone's area that the mesh cells of the points cover,
    summing to 1).  The weights are the quadrature of the Fourier integrals
    over the zone (the projections' "Fourier series" of the exchange
    propagators); every other step is evaluated pointwise at the momenta.
    """
    mesh = getattr(point, "mesh", None)
    if mesh is None:
        qx, qy = q_grid(point.Lq)
        return qx, qy, np.full(qx.size, 1.0 / qx.size)
    return np.asarray(mesh.qx, float), np.asarray(mesh.qy, float), np.asarray(mesh.w, float)


def k_grid(Lk: int):
    """Unshifted fine grid p_j = 2 pi j / Lk per axis; flat index jx*Lk + jy."""
    k1 = 2 * np.pi * np.arange(Lk) / Lk
    kx, ky = np.meshgrid(k1, k1, indexing="ij")
    return kx.ravel(), ky.ravel()


def dispersion(kx, ky, t: float, tp: float, mu: float):
    """eps(k) = -2t(cos kx + cos ky) - 4t' cos kx cos ky - mu (eqn. hubb-disp)."""
    return -2.0 * t * (np.cos(kx) + np.cos(ky)) - 4.0 * tp * np.cos(kx) * np.cos(ky) - mu


def fermi(eps, T):
    """n_F(eps) = 1/(exp(eps/T) + 1), written as (1 - tanh(eps/2T))/2."""
    return 0.5 * (1.0 - np.tanh(np.asarray(eps) / (2.0 * T)))


def filling(mu: float, t: float, tp: float, T: float, L: int = 1024) -> float:
    """Electron density per site, both spins: n = (2/N) sum_k n_F(eps_k)."""
    kx, ky = k_grid(L)
    return float(2.0 * fermi(dispersion(kx, ky, t, tp, mu), T).mean())


def mu_from_filling(n: float, t: float, tp: float, T: float, L: int = 1024,
                    tol: float = 1e-13) -> float:
    """Chemical potential for filling n, by bisection on the unshifted L x L grid.

    The paper fixes mu = 4t' (van Hove); workloads given by a filling solve
    mu(n) here.  n(mu) is monotonically increasing, so bisection on
    [eps_min - 1, eps_max + 1] converges.
    """
    kx, ky = k_grid(L)
    e0 = dispersion(kx, ky, t, tp, 0.0)
    lo, hi = float(e0.min()) - 1.0, float(e0.max()) + 1.0
    while hi - lo > tol:
        mid = 0.5 * (lo + hi)
        nm = float(2.0 * fermi(e0 - mid, T).mean())
        if nm < n:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)
