"""The per-kernel timing entry point (tufrg_kernel_times).

Each projection kernel and the products run alone, back to back, on the data
one right-hand side leaves in the workspace.  Checked here: the products'
output after the repeated launches equals tufrg_rhs bit for bit (every stage
writes its outputs, none accumulates); the per-stage flop counts add up to
tufrg_flop_count's projections and products (with symmetric states the
inverse transform and the products count one momentum per point-group
orbit); the durations are positive; the unsupported options are refused.
"""
import numpy as np
import pytest

import synth
from oracle.lattice import FormFactors
from oracle.symmetry import symmetrize

pytestmark = pytest.mark.gpu
STAGES = ("forward_transform", "bond_basis", "gather", "inverse_transform", "products")


@pytest.fixture(scope="module")
def tf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1604_06296_amd as tf
    tf.load_library()
    return tf


def _state(ctx, pts, seed, symmetric=False):
    import torch
    X = torch.zeros((3, ctx.S), dtype=torch.float64, device="cuda")
    for i, pt in enumerate(pts):
        ff = FormFactors(pt.shells)
        x = synth.random_channels(pt.nq, ff.nff, seed=seed + i, scale=1.0)
        if symmetric:
            x = symmetrize(x, ff, pt.Lq)
        ctx.view(X, i).copy_(torch.from_numpy(np.ascontiguousarray(x)))
    return X


def _orbits(L):
    """Number of C4v orbits of the L x L transfer grid (brute force)."""
    seen, n = set(), 0
    for a in range(L):
        for b in range(L):
            if (a, b) in seen:
                continue
            n += 1
            for sx in (1, -1):
                for sy in (1, -1):
                    for u, v in ((a, b), (b, a)):
                        seen.add(((sx * u) % L, (sy * v) % L))
    return n


def _check(ctx, T, X, reps=3, rows_fraction=None):
    import torch
    ref = ctx.rhs(T, X)
    out = ctx.empty(3)
    kt = ctx.kernel_times(T, X, out, reps=reps)
    assert tuple(kt) == STAGES
    for k, (us, fl) in kt.items():
        assert np.isfinite(us) and us > 0.0, (k, us)
        assert fl > 0.0, (k, fl)
    assert torch.equal(out, ref), "products after the timed launches differ from tufrg_rhs"
    fc = ctx.flop_count()
    proj = sum(kt[k][1] for k in STAGES[:4])
    if rows_fraction is None:
        assert proj == fc["projections"]
        assert kt["products"][1] == fc["products"]
        assert kt["inverse_transform"][1] == kt["forward_transform"][1]
    else:
        assert kt["inverse_transform"][1] == pytest.approx(kt["forward_transform"][1] * rows_fraction, rel=1e-15)
        assert kt["products"][1] == pytest.approx(fc["products"] * rows_fraction, rel=1e-15)
    return kt


def test_kernel_times_bench_point(tf):
    w = synth.cfg2()
    pt = w.points[0]
    pt.mu = tf.mu_from_filling(pt.t, pt.tp, pt.filling, pt.mu_T, pt.mu_L)
    ctx = tf.Context([pt])
    _check(ctx, 0.05, _state(ctx, [pt], 3), reps=5)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_kernel_times_batch_of_uneven_points(tf, precision):
    pts = [synth.small_point(Lq=6, Lk=12, shells=1), synth.small_point(Lq=10, Lk=24, shells=3, tp=-0.3, mu=-0.5),
           synth.small_point(Lq=8, Lk=20, shells=2, tp=0.0, mu=0.0)]
    ctx = tf.Context(pts, precision=precision)
    _check(ctx, [0.2, 0.1, 0.3], _state(ctx, pts, 7))


def test_kernel_times_symmetric_state(tf):
    pt = synth.small_point(Lq=12, Lk=24, shells=2)
    ctx = tf.Context([pt], symmetric_state=True)
    _check(ctx, 0.15, _state(ctx, [pt], 11, symmetric=True), rows_fraction=_orbits(12) / 144)


def test_kernel_times_refuses_unsupported(tf):
    pt = synth.small_point()
    ctx = tf.Context([pt], no_cross=True)
    X = _state(ctx, [pt], 5)
    with pytest.raises(tf.TufrgError):
        ctx.kernel_times(0.2, X, ctx.empty(3))
    ctx2 = tf.Context([pt])
    with pytest.raises(tf.TufrgError):
        ctx2.kernel_times(0.2, X, X)
