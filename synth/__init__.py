"""Seeded synthetic inputs for the TUfRG flow right-hand side.

This module is shared by the CPU oracle and by the GPU library's tests and
benchmark.  It holds workload *definitions* and seeded random draws only:
no part of the method's arithmetic (no dispersion, no loops, no
projections) lives here.  Quantities that need the method's arithmetic,
such as the chemical potential belonging to a filling, are solved by each
side on its own.

Workloads follow the t-t' Hubbard model of Sec. 4 (dispersion eqn.
hubb-disp, onsite U) with a temperature flow on uniform L_q x L_q transfer
grids and uniform L_k x L_k fine grids.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

BASE_SEED = 160406296

# number of form factors for a truncation at shell s (bond lengths 0, 1,
# sqrt2, 2, sqrt5: nearest-neighbour order of Sec. 3)
NFF_OF_SHELLS = {0: 1, 1: 5, 2: 9, 3: 13, 4: 21}
SHELLS_OF_NFF = {v: k for k, v in NFF_OF_SHELLS.items()}


@dataclasses.dataclass
class Mesh:
    """A non-uniform transfer-momentum mesh: points (qx, qy) in [-pi, pi)^2 and
    the fractions w of the zone's area covered by their cells (sum 1)."""
    qx: np.ndarray
    qy: np.ndarray
    w: np.ndarray

    @property
    def nq(self) -> int:
        return int(self.qx.size)


def refined_mesh(Lq: int, factor: int, centers, radius: int) -> Mesh:
    """The uniform Lq x Lq transfer grid with the cells near the given centers
    refined: a coarse cell (side 2 pi / Lq around q_i = 2 pi (i - Lq/2)/Lq per
    axis) within `radius` cells of a center (Chebyshev distance on the
    periodic grid) is replaced by factor x factor sub-cells (factor odd) whose
    centers are its points, each of weight 1/(Lq^2 factor^2); the other cells
    keep their point with weight 1/Lq^2.  Points are wrapped into [-pi, pi).
    Order: coarse cells in flat order ix * Lq + iy, the sub-points of a
    refined cell in their own flat order.  This is a geometry description
    only (the method's arithmetic lives in the oracle and in the library)."""
    if factor < 1 or factor % 2 == 0:
        raise ValueError("factor must be odd")
    h = 2 * np.pi / Lq
    cen = [(int(round(c[0] / h)) % Lq, int(round(c[1] / h)) % Lq) for c in centers]
    qx, qy, w = [], [], []
    for ix in range(Lq):
        for iy in range(Lq):
            x0, y0 = h * (ix - Lq // 2), h * (iy - Lq // 2)
            a, b = (ix - Lq // 2) % Lq, (iy - Lq // 2) % Lq
            near = any(min(abs(a - cx), Lq - abs(a - cx)) <= radius and
                       min(abs(b - cy), Lq - abs(b - cy)) <= radius for cx, cy in cen)
            f = factor if near else 1
            for sa in range(f):
                for sb in range(f):
                    dx, dy = h * (sa - (f - 1) // 2) / f, h * (sb - (f - 1) // 2) / f
                    qx.append((x0 + dx + np.pi) % (2 * np.pi) - np.pi)
                    qy.append((y0 + dy + np.pi) % (2 * np.pi) - np.pi)
                    w.append(1.0 / (Lq * Lq * f * f))
    return Mesh(np.array(qx), np.array(qy), np.array(w))


@dataclasses.dataclass
class Point:
    """One model/discretisation point.

    mu is None when the point is defined by a filling n; each side then
    solves mu(n) itself at temperature mu_T on a mu_L x mu_L grid.  mesh, when
    set, replaces the uniform Lq x Lq transfer grid (Lq then names the coarse
    grid the mesh refines).
    """
    t: float
    tp: float
    U: float
    Lq: int
    Lk: int
    shells: int
    mu: Optional[float] = None
    filling: Optional[float] = None
    mu_T: float = 1e-3
    mu_L: int = 1024
    mesh: Optional[Mesh] = None

    @property
    def nff(self) -> int:
        return NFF_OF_SHELLS[self.shells]

    @property
    def nq(self) -> int:
        return self.mesh.nq if self.mesh is not None else self.Lq * self.Lq


@dataclasses.dataclass
class Workload:
    name: str
    points: List[Point]
    T0: float
    Tmin: float
    Xmax: float
    scheme: str          # "rk4" or "dopri5"
    nsteps: int = 200    # rk4: number of uniform steps in ln T
    rtol: float = 1e-7
    atol: float = 1e-9
    precision: str = "fp64"
    regulator: str = "T"   # "T": temperature flow; "omega": Omega cutoff at T = 0


def cfg1() -> Workload:
    """Half-filled square lattice, N_ff = 5, 8x8 transfer grid, 32x32 fine grid."""
    p = Point(t=1.0, tp=0.0, U=3.0, Lq=8, Lk=32, shells=1, mu=0.0)
    return Workload("hubbard_halffill_nff5_q8_k32_rk4", [p], T0=10.0, Tmin=0.01,
                    Xmax=20.0, scheme="rk4", nsteps=200)


def cfg2() -> Workload:
    """t' = -0.25 at filling 0.85, N_ff = 13, 24x24 transfer grid, 96x96 fine grid."""
    p = Point(t=1.0, tp=-0.25, U=3.0, Lq=24, Lk=96, shells=3, filling=0.85,
              mu_T=1e-3)
    return Workload("hubbard_tp-0.25_n0.85_nff13_q24_k96_dopri5", [p], T0=10.0,
                    Tmin=1e-3, Xmax=20.0, scheme="dopri5")


def cfg2_omega() -> Workload:
    """cfg2's point flowed with the Omega cutoff at zero temperature: Omega from
    800 (two orders of magnitude above the bandwidth 8t) down to 1e-3, stopping
    at max|X| > 80 (one order of magnitude above the bandwidth)."""
    w = cfg2()
    return Workload("hubbard_tp-0.25_n0.85_nff13_q24_k96_omega_dopri5", w.points, T0=800.0,
                    Tmin=1e-3, Xmax=80.0, scheme="dopri5", regulator="omega")


def cfg3() -> Workload:
    """t' = -0.3, seeded mu in [-1.2, 0], N_ff = 21, 48x48 transfer grid, 128x128 fine grid."""
    rng = np.random.default_rng(BASE_SEED + 3)
    mu = float(rng.uniform(-1.2, 0.0))
    p = Point(t=1.0, tp=-0.3, U=3.0, Lq=48, Lk=128, shells=4, mu=mu)
    return Workload("hubbard_tp-0.3_nff21_q48_k128_mixed", [p], T0=10.0, Tmin=0.01,
                    Xmax=20.0, scheme="rk4", nsteps=200, precision="mixed")


def cfg4(npoints: int = 64) -> Workload:
    """Seeded sweep of uneven points for one batched launch."""
    rng = np.random.default_rng(BASE_SEED + 4)
    pts = []
    for _ in range(npoints):
        tp = float(rng.uniform(-0.35, 0.0))
        n = float(rng.uniform(0.7, 1.0))
        U = float(rng.uniform(2.0, 4.0))
        Lq = int(rng.choice(np.arange(16, 41, 2)))
        shells = int(rng.choice([1, 2, 3, 4]))
        pts.append(Point(t=1.0, tp=tp, U=U, Lq=Lq, Lk=4 * Lq, shells=shells,
                         filling=n, mu_T=0.01))
    return Workload("hubbard_sweep64_batched", pts, T0=10.0, Tmin=0.01, Xmax=20.0,
                    scheme="rk4", nsteps=200)


def cfg5() -> Workload:
    """cfg3 physics at N_ff = 21 on a 64x64 transfer grid with a 160x160 fine grid."""
    w3 = cfg3()
    p3 = w3.points[0]
    p = Point(t=p3.t, tp=p3.tp, U=p3.U, Lq=64, Lk=160, shells=4, mu=p3.mu)
    return Workload("hubbard_tp-0.3_nff21_q64_k160_surrogate", [p], T0=10.0, Tmin=0.01,
                    Xmax=20.0, scheme="rk4", nsteps=200)


def surrogate_training_points(npoints: int = 64) -> List[Point]:
    """Seeded (t', mu) draws over the cfg2-cfg3 parameter ranges on the cfg5
    grids (N_ff = 21, 64x64 transfer, 160x160 fine), for surrogate labels."""
    rng = np.random.default_rng(BASE_SEED + 5)
    pts = []
    for _ in range(npoints):
        tp = float(rng.uniform(-0.35, -0.2))
        mu = float(rng.uniform(-1.2, 0.0))
        pts.append(Point(t=1.0, tp=tp, U=3.0, Lq=64, Lk=160, shells=4, mu=mu))
    return pts


def surrogate_training_temperatures(npoints: int, rounds: int, seed: int = BASE_SEED + 55,
                                    lo: float = 0.01, hi: float = 10.0) -> np.ndarray:
    """[rounds][npoints] log-uniform temperatures of the flow range."""
    rng = np.random.default_rng(seed)
    return np.exp(rng.uniform(np.log(lo), np.log(hi), (rounds, npoints)))


def small_point(Lq=6, Lk=12, shells=1, t=1.0, tp=-0.2, mu=-0.3, U=2.5) -> Point:
    return Point(t=t, tp=tp, U=U, Lq=Lq, Lk=Lk, shells=shells, mu=mu)


def random_channels(nq: int, nff: int, seed: int, scale: float = 1.0,
                    symmetric: bool = True) -> np.ndarray:
    """Random exchange-propagator state X[3][nq][nff][nff] (P, C, D), FP64.

    Matrices are symmetric in (m, n) when `symmetric` (the symmetry of the
    exchange propagators stated in the appendix on symmetries); no other
    structure is imposed.
    """
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((3, nq, nff, nff)) * scale
    if symmetric:
        X = 0.5 * (X + np.swapaxes(X, -1, -2))
    return np.ascontiguousarray(X)


def random_temperatures(n: int, seed: int, lo: float = 1e-3, hi: float = 10.0) -> np.ndarray:
    """Log-uniform temperatures in [lo, hi]."""
    rng = np.random.default_rng(seed)
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size=n))


def sample_indices(n: int, k: int, seed: int) -> np.ndarray:
    """k distinct sorted indices out of range(n)."""
    rng = np.random.default_rng(seed)
    k = min(k, n)
    return np.sort(rng.choice(n, size=k, replace=False))
