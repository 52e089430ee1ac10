"""Pins of the oracle's lattice objects: form factors, bonds, dispersion, mu(n)."""
import json
import os

import numpy as np
import pytest

from oracle.lattice import (FormFactors, SHELL_BONDS, dispersion, filling, k_grid,
                            mu_from_filling, q_grid)

HERE = os.path.dirname(__file__)

# The eight C4v operations acting on (kx, ky).
C4V = {
    "E": lambda x, y: (x, y),
    "C4": lambda x, y: (-y, x),
    "C2": lambda x, y: (-x, -y),
    "C4^3": lambda x, y: (y, -x),
    "sx": lambda x, y: (-x, y),
    "sy": lambda x, y: (x, -y),
    "sd": lambda x, y: (y, x),
    "sd'": lambda x, y: (-y, -x),
}

# Characters of the 1D irreps on the operations above (textbook C4v table).
CHAR = {
    "A1": dict(E=1, C4=1, C2=1, **{"C4^3": 1}, sx=1, sy=1, sd=1, **{"sd'": 1}),
    "A2": dict(E=1, C4=1, C2=1, **{"C4^3": 1}, sx=-1, sy=-1, sd=-1, **{"sd'": -1}),
    "B1": dict(E=1, C4=-1, C2=1, **{"C4^3": -1}, sx=1, sy=1, sd=-1, **{"sd'": -1}),
    "B2": dict(E=1, C4=-1, C2=1, **{"C4^3": -1}, sx=-1, sy=-1, sd=1, **{"sd'": 1}),
}


def _grid(L=16):
    g = 2 * np.pi * np.arange(L) / L
    return np.meshgrid(g, g, indexing="ij")


def test_counting_pin_fifth_neighbour():
    """8.9e6 = (992 + 2*6632) * N_ff^2 fixes N_ff = 25 at 5th-neighbour truncation."""
    pin = json.load(open(os.path.join(HERE, "golden", "paper_counting_pin.json")))
    # bonds within the 5th nearest neighbour: all R with |R|^2 among the 6 smallest norms
    norms = sorted({x * x + y * y for x in range(-4, 5) for y in range(-4, 5)})[: pin["truncation_nn"] + 1]
    n25 = sum(1 for x in range(-4, 5) for y in range(-4, 5) if x * x + y * y in norms)
    dim = (pin["nq_P"] + 2 * pin["nq_CD"]) * n25 ** 2
    assert n25 == 25
    assert f"{dim:.1e}" == f"{pin['printed_dimension']:.1e}"
    # our shells 0..4 are the first five bond lengths, the counts 1,5,9,13,21
    counts = np.cumsum([len(s) for s in SHELL_BONDS])
    assert list(counts) == [1, 5, 9, 13, 21]
    assert [len(s) for s in SHELL_BONDS] == [sum(1 for x in range(-4, 5) for y in range(-4, 5)
                                                if x * x + y * y == nrm) for nrm in norms[:5]]


@pytest.mark.parametrize("shells", [0, 1, 2, 3, 4])
def test_form_factor_orthonormal_parity_real_space(shells):
    ff = FormFactors(shells)
    kx, ky = _grid()
    F = ff.values(kx, ky).reshape(ff.nff, -1)
    np.testing.assert_allclose(F @ F.T / F.shape[1], np.eye(ff.nff), atol=1e-14)
    Fm = ff.values(-kx, -ky).reshape(ff.nff, -1)
    np.testing.assert_allclose(Fm, ff.parity[:, None] * F, atol=1e-14)
    # f_m(k) = sum_R c_mR exp(-i k.R) reproduces the functions exactly
    rec = np.zeros_like(F, dtype=complex)
    for b, (rx, ry) in enumerate(ff.bonds):
        rec += ff.c[:, b][:, None] * np.exp(-1j * (kx * rx + ky * ry)).ravel()[None]
    np.testing.assert_allclose(rec.real, F, atol=1e-14)
    assert np.abs(rec.imag).max() < 1e-14
    # each form factor lives on one bond length (fixed-bond-length basis)
    for m in range(ff.nff):
        lens = {ff.bonds[b][0] ** 2 + ff.bonds[b][1] ** 2 for b in range(ff.nff) if abs(ff.c[m, b]) > 0}
        assert len(lens) == 1
    # real coefficients for even, imaginary for odd form factors; unitary
    for m in range(ff.nff):
        part = ff.c[m].imag if ff.parity[m] > 0 else ff.c[m].real
        assert np.abs(part).max() < 1e-15
    np.testing.assert_allclose(ff.c @ ff.c.conj().T, np.eye(ff.nff), atol=1e-14)


@pytest.mark.parametrize("shells", [1, 2, 3, 4])
def test_form_factor_irreps(shells):
    """f_m(S k) = sum C^S_{m,m~} f_m~(k) with C^S orthogonal; 1D irreps carry their characters."""
    ff = FormFactors(shells)
    kx, ky = _grid()
    F = ff.values(kx, ky).reshape(ff.nff, -1)
    for name, S in C4V.items():
        sx, sy = S(kx, ky)
        FS = ff.values(sx, sy).reshape(ff.nff, -1)
        CS = FS @ F.T / F.shape[1]
        np.testing.assert_allclose(CS @ F, FS, atol=1e-13)
        np.testing.assert_allclose(CS @ CS.T, np.eye(ff.nff), atol=1e-13)
        for m, ir in enumerate(ff.irrep):
            if ir in CHAR:
                assert abs(CS[m, m] - CHAR[ir][name]) < 1e-13, (m, ir, name)
            # never mixes irreps or shells
            for n in range(ff.nff):
                if ff.irrep[n] != ir or ff.shell_of[n] != ff.shell_of[m]:
                    assert abs(CS[m, n]) < 1e-13


def test_grids():
    qx, qy = q_grid(4)
    assert np.allclose(sorted(set(np.round(qx, 12))), np.round([-np.pi, -np.pi / 2, 0, np.pi / 2], 12))
    assert qx[1 * 4 + 2] == -np.pi / 2 and qy[1 * 4 + 2] == 0.0
    kx, ky = k_grid(4)
    assert kx[0] == 0.0 and np.isclose(ky[3], 1.5 * np.pi)


def test_dispersion_van_hove_and_symmetry():
    t, tp = 1.0, -0.3
    # van Hove filling mu = 4t' puts the saddle point (pi, 0) at the Fermi level (Sec. 4)
    assert abs(dispersion(np.pi, 0.0, t, tp, 4 * tp)) < 1e-15
    kx, ky = _grid(12)
    e = dispersion(kx, ky, t, tp, 0.2)
    np.testing.assert_allclose(e, dispersion(-ky, kx, t, tp, 0.2), atol=1e-14)
    # bandwidth 8t at t' = 0
    e0 = dispersion(kx, ky, 1.0, 0.0, 0.0)
    assert np.isclose(e0.max() - e0.min(), 8.0)


def test_mu_from_filling():
    # particle-hole symmetry at t' = 0: half filling at mu = 0
    assert abs(mu_from_filling(1.0, 1.0, 0.0, 0.01, L=64)) < 1e-12
    mu = mu_from_filling(0.85, 1.0, -0.25, 1e-3, L=256)
    assert abs(filling(mu, 1.0, -0.25, 1e-3, L=256) - 0.85) < 1e-10
    assert -2.0 < mu < 0.0
