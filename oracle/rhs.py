"""Flow right-hand side: steps i.-iii. of the TUfRG increment.

TEST INFRASTRUCTURE ONLY (plain FP64 CPU oracle; never used by the GPU path).

Paper Sec. 2.4: i.) projections (eqns. proj_VP/VC/VD), ii.) loops
(eqn. chis), iii.) matrix products per transfer momentum
    dP/dT =  V^P chi'^pp V^P                              (eqn. matmul-P)
    dC/dT = -V^C chi'^ph V^C                              (eqn. matmul-C)
    dD/dT = 2 V^D chi'^ph V^D - V^C chi'^ph V^D - V^D chi'^ph V^C   (eqn. matmul-D)
with chi' = d chi / dT (temperature flow), or d chi / dOm with the Omega
cutoff (regulator="omega"; the scale argument is then Om).
"""
from __future__ import annotations

import numpy as np

from .bubbles import bubbles
from .lattice import FormFactors
from .projections import project


def products(V: np.ndarray, dchi: np.ndarray) -> np.ndarray:
    """dX/dT[3][nq][nff][nff] from V[3][...] and dchi[2][...] = (pp, ph)."""
    VP, VC, VD = V
    xpp, xph = dchi
    dP = VP @ xpp @ VP
    dC = -(VC @ xph @ VC)
    dD = 2.0 * (VD @ xph @ VD) - VC @ xph @ VD - VD @ xph @ VC
    return np.stack([dP, dC, dD])


def rhs(point, T: float, X: np.ndarray, ff: FormFactors | None = None,
        no_cross: bool = False, return_parts: bool = False, q_index=None,
        regulator: str = "T"):
    """dX/dT at scale T for state X = (P, C, D), at the momenta q_index (all by default)."""
    ff = ff or FormFactors(point.shells)
    V = project(point, X, ff, no_cross=no_cross, l_index=q_index)
    dchi = bubbles(point, T, "dot", ff, q_index=q_index, regulator=regulator)
    dX = products(V, dchi)
    if return_parts:
        return dX, V, dchi
    return dX
