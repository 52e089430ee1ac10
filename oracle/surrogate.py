"""Loop harmonics, surrogate features and targets, and an FP64 MLP.

TEST INFRASTRUCTURE ONLY (plain FP64 CPU oracle; never used by the GPU path).

Loop harmonics.  Writing f_m(p) = sum_b c_mb exp(-i p.R_b), the projected
loop of eqn. chis becomes
    chi'_mn(q) = sum_{a,b} c_ma c_nb ghat(q, R_a + R_b),
    ghat_X(q, S) = (1/N_k) sum_p dL^X/dT(eps(p+q/2), eps(p-q/2)) cos(p.S),
real and even in S because the pair (p + q/2, p - q/2) maps to its swap
under p -> -p.  So one value per (q, S) with S in the set bonds + bonds
carries the whole loop; a surrogate predicts these values.

Surrogate encoding (a reading: the paper has no surrogate).  A query is one
(q, S) at one temperature and model point; S is represented by its
canonical bond pair, the first pair (a, b) in the order of the form-factor
bond list with R_a + R_b = S.  Nine features
    (qx/pi, qy/pi, log10 T, mu/t, t'/t, R_a/2, R_b/2)
and four targets
    (T (1 + 4T) ghat_pp, (1 + 4T^2) ghat_ph, 0, 0)
(the last two are the imaginary parts, identically zero).  The scale
factors follow the asymptotics of the loop derivatives (1/(4T^2) at high T;
pp ~ 1/T and ph ~ 1 at low T) so that targets stay of order one.

MLP.  Layers z_l = a_{l-1} W_l^T + b_l with a_l = silu(z_l) = z_l
sigmoid(z_l) on hidden layers and a linear output; loss = mean over all
outputs of (a_L - y)^2.  Gradients by plain backpropagation.
"""
from __future__ import annotations

import numpy as np

from .bubbles import loop_dot
from .lattice import FormFactors, dispersion, k_grid, q_grid


def harmonic_set(ff: FormFactors):
    """The distinct S in bonds + bonds, as a sorted list of (Sx, Sy)."""
    return sorted({(a[0] + b[0], a[1] + b[1]) for a in ff.bonds for b in ff.bonds})


def canonical_pair(ff: FormFactors, S):
    """First (a, b) in bond-list order with R_a + R_b = S."""
    for a, Ra in enumerate(ff.bonds):
        for b, Rb in enumerate(ff.bonds):
            if Ra[0] + Rb[0] == S[0] and Ra[1] + Rb[1] == S[1]:
                return Ra, Rb
    raise ValueError(f"{S} is not a sum of two bonds")


def loop_harmonics(point, T: float, S_list, q_index=None) -> np.ndarray:
    """ghat_X(q, S) for X = (pp, ph): array [2][nq_sel][len(S_list)]."""
    qx, qy = q_grid(point.Lq)
    if q_index is not None:
        qx, qy = qx[q_index], qy[q_index]
    px, py = k_grid(point.Lk)
    S = np.asarray(S_list, dtype=float).reshape(-1, 2)
    cosS = np.cos(np.outer(px, S[:, 0]) + np.outer(py, S[:, 1]))      # [Nk][nS]
    out = np.empty((2, qx.size, S.shape[0]))
    for i in range(qx.size):
        e1 = dispersion(px + 0.5 * qx[i], py + 0.5 * qy[i], point.t, point.tp, point.mu)
        e2 = dispersion(px - 0.5 * qx[i], py - 0.5 * qy[i], point.t, point.tp, point.mu)
        for c, ch in enumerate(("pp", "ph")):
            out[c, i] = loop_dot(e1, e2, T, ch) @ cosS / px.size
    return out


def chi_from_harmonics(ghat: np.ndarray, ff: FormFactors, S_list) -> np.ndarray:
    """chi'_mn(q) = sum_{a,b} c_ma c_nb ghat(q, R_a + R_b): [2][nq][nff][nff]."""
    index = {tuple(s): j for j, s in enumerate(S_list)}
    E = np.zeros((ff.nff, ff.nff, len(S_list)), dtype=complex)
    for a, Ra in enumerate(ff.bonds):
        for b, Rb in enumerate(ff.bonds):
            j = index[(Ra[0] + Rb[0], Ra[1] + Rb[1])]
            E[:, :, j] += np.outer(ff.c[:, a], ff.c[:, b])
    chi = np.einsum("mnj,cqj->cqmn", E, ghat)
    assert np.abs(chi.imag).max() <= 1e-12 * max(np.abs(chi.real).max(), 1e-300)
    return chi.real


def features(point, T: float, qx, qy, Ra, Rb) -> np.ndarray:
    """The nine inputs of each query (arrays broadcast over queries)."""
    qx, qy = np.broadcast_arrays(np.asarray(qx, float), np.asarray(qy, float))
    n = qx.size
    Ra = np.broadcast_to(np.asarray(Ra, float), (n, 2))
    Rb = np.broadcast_to(np.asarray(Rb, float), (n, 2))
    col = lambda v: np.full(n, v)
    return np.stack([qx.ravel() / np.pi, qy.ravel() / np.pi, col(np.log10(T)),
                     col(point.mu / point.t), col(point.tp / point.t),
                     Ra[:, 0] / 2, Ra[:, 1] / 2, Rb[:, 0] / 2, Rb[:, 1] / 2], axis=1)


def target_scales(T: float):
    """Factors (pp, ph) that map ghat to the surrogate targets."""
    return T * (1.0 + 4.0 * T), 1.0 + 4.0 * T * T


def targets(T: float, ghat_pp, ghat_ph) -> np.ndarray:
    spp, sph = target_scales(T)
    gpp = np.asarray(ghat_pp, float).ravel()
    return np.stack([spp * gpp, sph * np.asarray(ghat_ph, float).ravel(),
                     np.zeros_like(gpp), np.zeros_like(gpp)], axis=1)


# ------------------------------------------------------------------- MLP
def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def unflatten(flat: np.ndarray, widths):
    """Flat parameter vector (per layer: W[out][in] row-major, then b[out])
    -> list of (W, b)."""
    params, o = [], 0
    for i in range(len(widths) - 1):
        n_in, n_out = widths[i], widths[i + 1]
        W = flat[o:o + n_out * n_in].reshape(n_out, n_in)
        o += n_out * n_in
        b = flat[o:o + n_out]
        o += n_out
        params.append((np.asarray(W, float), np.asarray(b, float)))
    assert o == flat.size
    return params


def flatten(grads) -> np.ndarray:
    return np.concatenate([np.concatenate([gW.ravel(), gb.ravel()]) for gW, gb in grads])


def mlp_forward(params, x: np.ndarray) -> np.ndarray:
    a = np.asarray(x, float)
    for i, (W, b) in enumerate(params):
        z = a @ W.T + b
        a = silu(z) if i + 1 < len(params) else z
    return a


def mlp_loss_and_grad(params, x: np.ndarray, y: np.ndarray):
    """Mean-squared loss and its gradient [(dW, db)] by backpropagation."""
    acts, zs = [np.asarray(x, float)], []
    for i, (W, b) in enumerate(params):
        z = acts[-1] @ W.T + b
        zs.append(z)
        acts.append(silu(z) if i + 1 < len(params) else z)
    r = acts[-1] - y
    loss = float(np.mean(r * r))
    delta = 2.0 * r / r.size                           # dloss / d a_L = dloss / d z_L
    grads = [None] * len(params)
    for i in range(len(params) - 1, -1, -1):
        W, _ = params[i]
        grads[i] = (delta.T @ acts[i], delta.sum(axis=0))
        if i > 0:
            delta = (delta @ W) * silu_grad(zs[i - 1])
    return loss, grads
