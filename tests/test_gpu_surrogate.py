"""GPU parity of the loop surrogate: loop harmonics, training data, the MLP
(forward and gradient against the FP64 NumPy backprop of the oracle), training,
and the exact-fallback mechanics of the surrogate loops.

Tolerances: loop harmonics FP64 1e-10 normwise per channel; features and
targets to FP32 rounding; MLP forward (BF16 hi/lo split products, FP32
accumulation) 2e-4 of the largest output; MLP gradient (plain BF16 products)
3e-2 of each layer's largest gradient entry, loss 1e-4 relative.
"""
import numpy as np
import pytest

import synth
from oracle import bubbles as obub
from oracle import rhs as orhs
from oracle import surrogate as osur
from oracle.lattice import FormFactors, q_grid

pytestmark = pytest.mark.gpu
WIDTHS = [9, 256, 256, 256, 256, 4]


@pytest.fixture(scope="module")
def tf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1604_06296_amd as tf
    tf.load_library()
    return tf


def _torch():
    import torch
    return torch


def _pt(shells, Lq, Lk, tp=-0.27, mu=-0.61, U=3.0):
    return synth.Point(t=1.0, tp=tp, U=U, Lq=Lq, Lk=Lk, shells=shells, mu=mu)


def _orbits(Lq):
    """Number of C4v orbits of the Lq x Lq transfer grid modulo the reciprocal
    lattice (the surrogate works on one representative per orbit)."""
    seen, n = set(), 0
    for a in range(Lq):
        for b in range(Lq):
            if (a, b) in seen:
                continue
            n += 1
            for x, y in ((a, b), (b, a)):
                for sx in (1, -1):
                    for sy in (1, -1):
                        seen.add(((sx * x) % Lq, (sy * y) % Lq))
    return n


@pytest.mark.parametrize("shells,Lq,Lk", [(0, 6, 12), (1, 6, 14), (2, 8, 16), (3, 10, 20), (4, 10, 22)])
def test_loop_harmonics_vs_oracle(tf, shells, Lq, Lk):
    pt = _pt(shells, Lq, Lk)
    print(f"[harmonics] shells={shells} Lq={Lq} Lk={Lk}", flush=True)
    ctx = tf.Context([pt])
    n, tab, off = ctx.harmonics(0)
    assert n == (1, 7, 13, 21, 35)[shells] and off == 0
    S = [tuple(r[:2]) for r in tab]
    ff = FormFactors(shells)
    for r in tab:            # canonical pairs: the oracle's definition
        Ra, Rb = osur.canonical_pair(ff, tuple(r[:2]))
        assert (tuple(r[2:4]), tuple(r[4:6])) == (Ra, Rb)
    for T in (5.0, 0.2, 0.011):
        got = ctx.loop_harmonics(T).cpu().numpy().reshape(pt.nq, 2, n).transpose(1, 0, 2)
        ref = osur.loop_harmonics(pt, T, S)
        for c in range(2):
            assert np.abs(got[c] - ref[c]).max() <= 1e-10 * np.abs(ref[c]).max()
        # and they rebuild the exact loops (ghat is even in S: extend the half set)
        neg = [j for j, s in enumerate(S) if s != (0, 0)]
        S_full = S + [(-S[j][0], -S[j][1]) for j in neg]
        chi = osur.chi_from_harmonics(np.concatenate([got, got[:, :, neg]], axis=2), ff, S_full)
        assert np.abs(chi - obub.bubbles(pt, T, "dot", ff)).max() <= 1e-10 * np.abs(chi).max()


def test_dataset_vs_oracle(tf):
    pts = [_pt(4, 10, 20, tp=-0.3, mu=-1.0), _pt(2, 8, 16, tp=-0.22, mu=-0.4)]
    ctx = tf.Context(pts)
    Ts = [0.07, 1.3]
    x, y, idx = ctx.surrogate_dataset(Ts, 3000, seed=17, with_index=True)
    x, y, idx = x.cpu().numpy(), y.cpu().numpy(), idx.cpu().numpy()
    assert set(idx[:, 0]) == {0, 1}
    for p, pt in enumerate(pts):
        n, tab, _ = ctx.harmonics(p)
        S = [tuple(r[:2]) for r in tab]
        g = osur.loop_harmonics(pt, Ts[p], S)
        qx, qy = q_grid(pt.Lq)
        rows = np.where(idx[:, 0] == p)[0]
        q, j = idx[rows, 1], idx[rows, 2]
        ref_x = np.stack([osur.features(pt, Ts[p], qx[qi], qy[qi], tuple(tab[ji, 2:4]), tuple(tab[ji, 4:6]))[0]
                          for qi, ji in zip(q, j)])
        np.testing.assert_allclose(x[rows], ref_x.astype(np.float32), rtol=1e-6, atol=1e-6)
        ref_y = osur.targets(Ts[p], g[0, q, j], g[1, q, j])
        scale = np.abs(ref_y[:, :2]).max()
        assert np.abs(y[rows] - ref_y).max() <= 1e-6 * scale


def _random_params(seed, widths, scale=1.0):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(len(widths) - 1):
        lim = scale * np.sqrt(6.0 / (widths[i] + widths[i + 1]))
        out.append(rng.uniform(-lim, lim, widths[i] * widths[i + 1]))
        out.append(rng.uniform(-0.1, 0.1, widths[i + 1]))
    return np.concatenate(out)


def test_mlp_forward_and_gradient_vs_fp64(tf):
    torch = _torch()
    flat = _random_params(3, WIDTHS)
    net = tf.MLP(WIDTHS, max_rows=256, seed=1)
    assert net.nparams == flat.size == 9 * 256 + 256 + 3 * (256 * 256 + 256) + 256 * 4 + 4
    net.set_params(torch.from_numpy(flat.astype(np.float32)).cuda())
    flat32 = net.params().cpu().numpy().astype(np.float64)
    params = osur.unflatten(flat32, WIDTHS)
    rng = np.random.default_rng(4)
    x = rng.uniform(-1, 1, (64, 9)).astype(np.float32)
    y = rng.standard_normal((64, 4)).astype(np.float32)
    xd, yd = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    out = net.forward(xd).cpu().numpy()
    ref = osur.mlp_forward(params, x.astype(np.float64))
    assert np.abs(out - ref).max() <= 2e-4 * np.abs(ref).max()
    g, loss = net.gradient(xd, yd)
    ref_loss, ref_grads = osur.mlp_loss_and_grad(params, x.astype(np.float64), y.astype(np.float64))
    assert abs(loss / ref_loss - 1) < 1e-4
    g = g.cpu().numpy()
    o = 0
    for i, (gW, gb) in enumerate(ref_grads):
        for name, ref_part in (("W", gW.ravel()), ("b", gb)):
            got = g[o:o + ref_part.size]
            o += ref_part.size
            err = np.abs(got - ref_part).max()
            assert err <= 3e-2 * np.abs(ref_part).max(), f"layer {i} {name}: err {err:.3e}"
    # forward in chunks of max_rows equals one pass
    xb = torch.from_numpy(rng.uniform(-1, 1, (700, 9)).astype(np.float32)).cuda()
    yb = net.forward(xb)
    assert torch.equal(yb[:256], net.forward(xb[:256].contiguous()))


def test_mlp_training_fits_a_smooth_map(tf):
    torch = _torch()
    rng = np.random.default_rng(8)
    x = rng.uniform(-1, 1, (16384, 9)).astype(np.float32)
    y = np.stack([np.sin(2 * x[:, 0]) * x[:, 1], np.cos(x[:, 2] + x[:, 3]), x[:, 4] ** 2 - x[:, 5],
                  0 * x[:, 0]], axis=1).astype(np.float32)
    net = tf.MLP(WIDTHS, max_rows=1024, seed=2)
    hist = net.train(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda(), steps=600, batch=512,
                     lr=2e-3, seed=5)
    print(f"[mlp] loss {hist[0]:.3e} -> {hist[-20:].mean():.3e}", flush=True)
    assert np.isfinite(hist).all()
    assert hist[-20:].mean() < 2e-2 * hist[:5].mean()


def test_surrogate_disagreeing_nets_fall_back_everywhere(tf):
    """Two independent untrained networks disagree at every momentum, so every
    loop is exact: the surrogate right-hand side equals the exact one."""
    torch = _torch()
    pt = _pt(3, 10, 20, tp=-0.3, mu=-0.9)
    ff = FormFactors(3)
    exact = tf.Context([pt])
    ctx = tf.Context([pt])
    a, b = tf.MLP(WIDTHS, max_rows=4096, seed=11), tf.MLP(WIDTHS, max_rows=4096, seed=12)
    ctx.attach_surrogate(a, b, tol=1e-3, check_stride=8)
    X = torch.from_numpy(synth.random_channels(pt.nq, ff.nff, seed=3).reshape(3, -1)).cuda()
    for T in (2.0, 0.05):
        ref = exact.rhs(T, X).cpu().numpy()
        got = ctx.rhs(T, X).cpu().numpy()
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
        rb = exact.bubbles(T).cpu().numpy()
        gb = ctx.bubbles(T).cpu().numpy()
        assert np.abs(gb - rb).max() <= 1e-12 * np.abs(rb).max()
    st = ctx.surrogate_stats()
    assert st["exact_q"] == st["queried_q"] == 4 * _orbits(pt.Lq)
    ctx.detach_surrogate()
    assert torch.equal(ctx.bubbles(0.3), exact.bubbles(0.3))


def test_surrogate_rotating_check_flags_bad_predictions(tf):
    """One untrained network twice: no disagreement, so only the rotating
    check finds the (wrong) predictions; after one full rotation every
    momentum is flagged and the loops are exact again."""
    torch = _torch()
    pt = _pt(1, 8, 16)
    exact = tf.Context([pt])
    ctx = tf.Context([pt])
    a = tf.MLP(WIDTHS, max_rows=4096, seed=21)
    stride = 4
    ctx.attach_surrogate(a, a, tol=1e-3, check_stride=stride)
    T = 0.4
    for _ in range(stride):
        ctx.bubbles(T)
    st = ctx.surrogate_stats()
    assert st["failed_checks"] == _orbits(pt.Lq)   # every representative checked once, all failed
    ref = exact.bubbles(T).cpu().numpy()
    got = ctx.bubbles(T).cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    st2 = ctx.surrogate_stats()
    assert st2["exact_q"] - st["exact_q"] == _orbits(pt.Lq)


def test_surrogate_flow_graph_equals_exact(tf):
    """The surrogate pipeline inside a captured RK4 step: with disagreeing
    networks every loop falls back, so the flow equals the exact flow."""
    pt = _pt(1, 8, 16, tp=0.0, mu=0.0, U=3.0)
    opts = tf.FlowOptions(T0=10.0, Tmin=0.05, Xmax=20.0, scheme="rk4", nsteps=40, use_graph=True)
    exact = tf.Context([pt])
    Xe = exact.empty(3).zero_()
    re = exact.flow(Xe, opts)[0]
    ctx = tf.Context([pt])
    a, b = tf.MLP(WIDTHS, max_rows=4096, seed=31), tf.MLP(WIDTHS, max_rows=4096, seed=32)
    ctx.attach_surrogate(a, b)
    Xs = ctx.empty(3).zero_()
    rs = ctx.flow(Xs, opts)[0]
    print("exact", re, "surrogate", rs, flush=True)
    assert rs.status == re.status and rs.n_steps == re.n_steps
    if re.status == "diverged":
        assert abs(rs.Tc / re.Tc - 1) < 1e-9
    ref = Xe.cpu().numpy()
    assert np.abs(Xs.cpu().numpy() - ref).max() <= 1e-9 * np.abs(ref).max()


def _high_T_nets(tf, pt, nets=2, steps=3000):
    """Networks trained briefly on the point's own exact loop harmonics at
    2 <= T <= 8 (smooth loops), with their validation error there."""
    import torch
    from paper_1604_06296_amd import surrogate as sur
    temps = np.exp(np.random.default_rng(7).uniform(np.log(2.0), np.log(8.0), (5, 16)))
    x, y = sur.make_training_set([pt] * 16, temps[:4], 16384, seed=40)
    xv, yv = sur.make_training_set([pt] * 16, temps[4:], 8192, seed=90)
    out = sur.train_ensemble(x, y, steps=steps, batch=1024, lr=2e-3, seeds=tuple(range(1, nets + 1)),
                             max_rows=4096)
    errs = [sur.validation_error(n, xv, yv)["rel_rms"] for n, _, _ in out]
    torch.cuda.synchronize()
    return [n for n, _, _ in out], max(errs)


@pytest.mark.parametrize("nets", [2, 1])
def test_surrogate_accepted_predictions_match_oracle(tf, nets):
    """Where predictions are accepted (networks trained at high T, a tolerance
    that admits them), the loops and the right-hand side stay within the
    acceptance tolerance of the oracle's: chi' within 8 tol max|chi'| (each
    entry sums a few harmonics, each off by at most ~tol of the largest),
    and the stats show that predictions were used."""
    torch = _torch()
    from oracle import bubbles as obub
    pt = _pt(1, 8, 16, tp=-0.25, mu=-0.7)
    ff = FormFactors(1)
    models, err = _high_T_nets(tf, pt, nets=nets)
    tol = max(4.0 * err, 1e-3)
    print(f"[surrogate] {nets} net(s): validation rel. error {err:.2e}, tol {tol:.2e}", flush=True)
    assert tol < 0.2
    ctx = tf.Context([pt])
    ctx.attach_surrogate(models[0], models[1] if nets == 2 else None, tol=tol, check_stride=8)
    X = synth.random_channels(pt.nq, ff.nff, seed=8, scale=0.3)
    Xd = torch.from_numpy(X.reshape(3, -1)).cuda()
    for T in (4.0, 3.0, 5.0):
        got = ctx.view(ctx.bubbles(T)).cpu().numpy()
        ref = obub.bubbles(pt, T, "dot", ff)
        assert np.abs(got - ref).max() <= 8 * tol * np.abs(ref).max(), T
        gr = ctx.view(ctx.rhs(T, Xd)).cpu().numpy()
        rr = orhs.rhs(pt, T, X, ff)
        assert np.abs(gr - rr).max() <= 30 * tol * np.abs(rr).max(), T
    st = ctx.surrogate_stats()
    print(f"[surrogate] stats {st}", flush=True)
    assert st["exact_q"] < st["queried_q"]          # predictions were accepted


def test_single_network_wrong_everywhere_is_flagged_within_one_rotation(tf):
    """One untrained network (no ensemble): only the rotating check guards it.
    Within check_stride calls every representative is checked, fails and is
    flagged, after which the loops are exact again."""
    torch = _torch()
    pt = _pt(1, 8, 16)
    exact = tf.Context([pt])
    ctx = tf.Context([pt])
    a = tf.MLP(WIDTHS, max_rows=4096, seed=23)
    stride = 4
    ctx.attach_surrogate(a, None, tol=1e-3, check_stride=stride)
    T = 0.4
    for _ in range(stride):
        ctx.bubbles(T)
    st = ctx.surrogate_stats()
    assert st["failed_checks"] == _orbits(pt.Lq)
    ref = exact.bubbles(T).cpu().numpy()
    got = ctx.bubbles(T).cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
