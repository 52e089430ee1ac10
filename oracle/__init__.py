"""Plain FP64 CPU oracle of the TUfRG flow right-hand side.

TEST INFRASTRUCTURE ONLY.  Only the tests, the package smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code
with the GPU library (the two never import each other); only the seeded
input generators in `synth` serve both.

Modules:
  lattice      grids, bond form factors (C4v irreps), dispersion, mu(n)
  bubbles      loops chi^pp, chi^ph and d/dT (eqn. chis, temperature flow)
  projections  V^P, V^C, V^D (eqns. proj_VP/VC/VD via eqn. proj_pos)
  rhs          products (eqns. matmul-P/C/D) and the full increment
  flow         RK4 / Dormand-Prince flow in ln T, critical scale, classification
  symmetry     C4v covariance law of the exchange propagators, symmetrisation
  surrogate    loop harmonics ghat(q, S), surrogate features/targets, FP64 MLP

Parity status: every function is pinned by tests under tests/ against
closed forms, brute force or invariants, except the coupled flow at
N_ff >= 5, which is pinned only through its parts (tests/test_oracle_rhs.py).
"""
from . import bubbles, flow, lattice, projections, rhs, surrogate, symmetry  # noqa: F401
