"""The allocation-free right-hand side (tufrg_rhs_noalloc) against tufrg_rhs.

Two calls in a row through the C ABI, the second on a smaller context (the
static scratch keeps the first call's contents), each compared with the
same context's tufrg_rhs; a context whose workspace exceeds the scratch is
rejected."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _ctx_and_state(tf, pt, seed, **kw):
    import torch
    ctx = tf.Context([pt], **kw)
    X = torch.from_numpy(synth.random_channels(pt.nq, pt.nff, seed=seed).reshape(3, -1)).cuda().contiguous()
    return ctx, X


def test_noalloc_rhs_equals_rhs_on_two_calls():
    import torch

    import paper_1604_06296_amd as tf
    big = synth.Point(t=1.0, tp=-0.25, U=3.0, Lq=24, Lk=96, shells=3, mu=-0.9)
    small = synth.Point(t=1.0, tp=-0.1, U=2.5, Lq=10, Lk=20, shells=1, mu=-0.3)
    runs = []
    for pt, seed, T in ((big, 3, 0.05), (small, 4, 0.2)):
        print(f"[noalloc] Lq={pt.Lq} Lk={pt.Lk} shells={pt.shells} T={T}", flush=True)
        ctx, X = _ctx_and_state(tf, pt, seed)
        a = ctx.empty(3).fill_(np.nan)
        ctx.rhs_noalloc(T, X, a)
        runs.append((ctx, X, T, a))
    for ctx, X, T, a in runs:
        ref = ctx.rhs(T, X)
        torch.cuda.synchronize()
        assert torch.isfinite(a).all()
        assert torch.equal(a, ref)          # same kernels, same summation order
    # the smaller context again after the larger one, and a fused/two-stream
    # and a mixed-precision context
    for kw in (dict(fuse=False), dict(precision="mixed")):
        print(f"[noalloc] {kw}", flush=True)
        ctx, X = _ctx_and_state(tf, big, 5, **kw)
        a = ctx.empty(3)
        ctx.rhs_noalloc(0.1, X, a)
        ref = ctx.rhs(0.1, X)
        torch.cuda.synchronize()
        assert torch.equal(a, ref)


def test_noalloc_rejects_workspace_beyond_scratch():
    import paper_1604_06296_amd as tf
    from paper_1604_06296_amd.binding import TufrgError
    pt = synth.Point(t=1.0, tp=-0.3, U=3.0, Lq=48, Lk=32, shells=4, mu=-0.5)
    ctx, X = _ctx_and_state(tf, pt, 6)
    with pytest.raises(TufrgError, match="static scratch"):
        ctx.rhs_noalloc(0.1, X, ctx.empty(3))
