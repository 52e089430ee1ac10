"""Training driver of the loop surrogate: sequences library calls only.

Labels come from the exact FP64 loop kernel (tufrg_surrogate_dataset) over a
batched context of many model points, one round of temperatures per call;
the networks are trained by the library's MLP kernels (tufrg_mlp_train).
"""
from __future__ import annotations

import time

from .binding import MLP, Context

WIDTHS = (9, 256, 256, 256, 256, 4)


def make_training_set(points, temperatures, samples_per_round: int, seed: int):
    """(x [n][9], y [n][4]) float32 CUDA tensors, n = rounds * samples_per_round."""
    import torch
    ctx = Context(points)
    rounds = len(temperatures)
    n = rounds * samples_per_round
    x = torch.empty((n, 9), dtype=torch.float32, device="cuda")
    y = torch.empty((n, 4), dtype=torch.float32, device="cuda")
    for r, Ts in enumerate(temperatures):
        sl = slice(r * samples_per_round, (r + 1) * samples_per_round)
        ctx.surrogate_dataset([float(T) for T in Ts], samples_per_round, seed=seed + r, x=x[sl], y=y[sl])
    ctx.sync()
    ctx.close()
    return x, y


def train_ensemble(x, y, steps: int, batch: int = 4096, lr: float = 2e-3, seeds=(1, 2),
                   max_rows: int = 65536):
    """Two (or more) networks trained from different initialisations and
    minibatch draws; returns [(net, loss history, seconds)]."""
    import torch
    out = []
    for s in seeds:
        net = MLP(WIDTHS, max_rows=max(max_rows, batch), seed=s)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hist = net.train(x, y, steps, batch, lr, seed=1000 + s)
        out.append((net, hist, time.perf_counter() - t0))
    return out


def validation_error(net, x, y):
    """Relative RMS error of the two real targets (all, and per decade of T),
    the largest absolute error, and the largest predicted imaginary part."""
    out = net.forward(x)
    err = out[:, :2] - y[:, :2]
    res = {"rel_rms": float(err.pow(2).mean().sqrt() / y[:, :2].pow(2).mean().sqrt()),
           "max_abs": float(err.abs().max()), "imag_max": float(out[:, 2:].abs().max())}
    decades = {}
    for lo in (-2, -1, 0):
        m = (x[:, 2] >= lo) & (x[:, 2] < lo + 1)
        if int(m.sum()) > 0:
            e, t = err[m], y[m, :2]
            decades[f"T_1e{lo}"] = float(e.pow(2).mean().sqrt() / t.pow(2).mean().sqrt())
    res["rel_rms_by_decade"] = decades
    return res
