"""The learned warm start on the GPU, against the FP64 reference (oracle/mlp.py).

* forward, loss and gradient of phi_theta: the oracle rounds every product
  operand to bfloat16 at the same points as the GPU (weights and activations),
  so the comparison measures FP32 accumulation only: gradients within 1e-3 of
  each parameter block's norm, as fixed for this check;
* Adam: one step, elementwise;
* a few training steps through kkm_mlp_train against the oracle's steps;
* feature-space Lloyd, teacher-forced per step (labels equal away from ties);
* every layer of the forward pass fed the GPU's own input of that layer, at the
  FP32 accumulation bar on every row;
* kkm_mlp_train_fresh (the benchmark's trainer) step by step against the
  oracle's loss, gradient and Adam, at d = 128 and d = 1024;
* kkm_warm_start against the composition of its parts, bit for bit;
* the gain: trained on kernel values the Gram kernel computes, the warm start
  reaches a lower objective than the plain random start, and its refined
  labels agree (ARI >= 0.99) with the oracle run converged from the same warm
  labels.
"""
import sys

import numpy as np
import pytest

import datagen
import oracle
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu

D, H1, H2, OUT = 128, 512, 512, 256


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def kkm():
    import torch  # noqa: F401
    import paper_2501_05587_amd as kkm
    kkm.lib()
    return kkm


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def params(seed, d=D):
    th = datagen.mlp_init_params(d, H1, H2, OUT, seed=seed).astype(np.float64)
    th += np.random.default_rng(seed + 1).normal(0, 0.02, th.shape)  # non-zero biases
    return th.astype(np.float32)


def batch(seed, B, d=D):
    w = datagen.WORKLOADS["gmm200k"]
    rng = np.random.default_rng(seed)
    X = rng.normal(0, 1, (B, d)).astype(np.float32)
    K = oracle.kernel_matrix(X, oracle.GAUSS, 1.0 / d)
    return X, K


# (n, d): the last two take the wide-tile product (M * N >= 2^20) in all three
# layers (n = 4100, a ragged tail of 4 rows) or the first two (d = 103: a
# ragged k-slab, rows not 16-byte aligned)
@pytest.mark.parametrize("n,d", [(1, D), (63, D), (300, D), (4100, D), (2500, 103)])
def test_mlp_forward_parity(kkm, n, d):
    import torch
    th = params(0, d)
    X = np.random.default_rng(n).normal(0, 1, (n, d)).astype(np.float32)
    say("mlp forward", n, d)
    F = kkm.kkm_mlp_forward(to_dev(th), to_dev(X))
    torch.cuda.synchronize()
    ref, _ = omlp.forward(th.astype(np.float64), X, d, H1, H2, OUT, bf16_operands=True)
    # Both sides round every product operand to bfloat16, but an activation
    # next to a rounding midpoint may round to the other neighbour after FP32
    # (GPU) or FP64 (reference) accumulation; that moves the rest of its row by
    # about one operand spacing times the weights it meets.  So: every row
    # within one bfloat16 spacing of the output scale (a wrong slab, tail,
    # bias or layer misses that by far), and the typical row within FP32
    # accumulation error.
    err = np.abs(F.cpu().numpy() - ref).max(axis=1)
    scale = np.abs(ref).max()
    assert err.max() <= 2.0 ** -7 * scale, err.max()
    assert np.median(err) <= 2e-4 * scale + 1e-6, np.median(err)


def layer_check(a, W, b, got, gelu, what):
    """One layer fed the GPU's own input: z = bf16(a) bf16(W)^T + b in FP64
    against the GPU's FP32 accumulation, within twice the FP32 bound of a sum
    of K + 1 terms in any order, (K + 1) 2^-24 (sum |a w| + |b|); GELU adds at
    most its slope (< 1.13) times that and a few roundings of its own."""
    u = 2.0 ** -24
    A, Wb = omlp.bf16(a), omlp.bf16(W)
    z = A @ Wb.T + b
    bz = 2.0 * (A.shape[1] + 1) * u * (np.abs(A) @ np.abs(Wb).T + np.abs(b))
    ref = omlp.gelu(z) if gelu else z
    bound = 1.13 * bz + 8.0 * u * (np.abs(ref) + np.abs(z)) if gelu else bz
    r = np.abs(got.astype(np.float64) - ref) / bound
    assert r.max() <= 1.0, "%s: %.3g of the bound at %s" % (what, r.max(),
                                                           np.unravel_index(r.argmax(), r.shape))
    return r.max()


# every layer on every row at the FP32 accumulation bar: each layer takes the
# GPU's own output of the layer before (rounded to bfloat16 as its product
# does), so no activation sits differently on either side of a rounding
# midpoint; (4100, 128) and (2500, 103) take the wide-tile product, d = 1024
# is the benchmark's input layer
@pytest.mark.parametrize("n,d", [(1, D), (63, D), (300, D), (4100, D), (2500, 103), (700, 1024)])
def test_mlp_forward_layer_by_layer(kkm, n, d):
    import torch
    th = params(0, d)
    X = np.random.default_rng(n + 5).normal(0, 1, (n, d)).astype(np.float32)
    say("mlp layers", n, d)
    pd, Xd = to_dev(th), to_dev(X)
    H1g, H2g, Fg = kkm.kkm_mlp_forward_layers(pd, Xd)
    F = kkm.kkm_mlp_forward(pd, Xd)
    torch.cuda.synchronize()
    assert torch.equal(F, Fg)  # the same products as the plain forward pass
    W1, b1, W2, b2, W3, b3 = omlp.unpack(th.astype(np.float64), d, H1, H2, OUT)
    h1, h2 = H1g.cpu().numpy(), H2g.cpu().numpy()
    r1 = layer_check(X, W1, b1, h1, True, "layer 1")
    r2 = layer_check(h1, W2, b2, h2, True, "layer 2")
    r3 = layer_check(h2, W3, b3, Fg.cpu().numpy(), False, "layer 3")
    say("  worst of the bound: %.3g %.3g %.3g" % (r1, r2, r3))


@pytest.mark.parametrize("B", [64, 100])
def test_mlp_loss_grad_parity(kkm, B):
    import torch
    th = params(1)
    X, K = batch(2 + B, B)
    say("mlp grad", B)
    g, loss = kkm.kkm_mlp_loss_grad(to_dev(th), to_dev(X), to_dev(K.astype(np.float32)))
    torch.cuda.synchronize()
    L_ref, g_ref = omlp.loss_and_grad(th.astype(np.float64), X, K.astype(np.float32).astype(np.float64),
                                      D, H1, H2, OUT, bf16_operands=True)
    assert float(loss.item()) == pytest.approx(L_ref, rel=1e-4)
    gg = g.cpu().numpy().astype(np.float64)
    off = 0
    for shape in omlp.param_shapes(D, H1, H2, OUT):
        size = int(np.prod(shape))
        a, b = gg[off:off + size], g_ref[off:off + size]
        assert np.linalg.norm(a - b) <= 1e-3 * np.linalg.norm(b) + 1e-12, (shape, np.linalg.norm(a - b),
                                                                           np.linalg.norm(b))
        off += size
    # and the exact (unrounded) gradient is within bfloat16's reach of it
    _, g_exact = omlp.loss_and_grad(th.astype(np.float64), X, K, D, H1, H2, OUT)
    assert np.linalg.norm(gg - g_exact) <= 5e-2 * np.linalg.norm(g_exact)


def test_mlp_adam_parity(kkm):
    import torch
    rng = np.random.default_rng(7)
    p = rng.normal(0, 1, 5000).astype(np.float32)
    m = rng.normal(0, 0.1, 5000).astype(np.float32)
    v = np.abs(rng.normal(0, 0.1, 5000)).astype(np.float32)
    g = rng.normal(0, 1, 5000).astype(np.float32)
    pd, md, vd = to_dev(p), to_dev(m), to_dev(v)
    kkm.kkm_mlp_adam(pd, md, vd, to_dev(g), 3, lr=1e-2)
    torch.cuda.synchronize()
    pr, mr, vr = omlp.adam_step(p.astype(np.float64), m.astype(np.float64), v.astype(np.float64),
                                g.astype(np.float64), 3, lr=1e-2)
    np.testing.assert_allclose(pd.cpu().numpy(), pr, rtol=0, atol=1e-6)
    np.testing.assert_allclose(md.cpu().numpy(), mr, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(vd.cpu().numpy(), vr, rtol=1e-6, atol=1e-8)


def test_mlp_train_steps_match_oracle(kkm):
    import torch
    m_train, B, steps = 300, 64, 3
    rng = np.random.default_rng(11)
    Xt = rng.normal(0, 1, (m_train, D)).astype(np.float32)
    Kt = oracle.kernel_matrix(Xt, oracle.GAUSS, 1.0 / D).astype(np.float32)
    idx = np.stack([rng.choice(m_train, B, replace=False) for _ in range(steps)]).astype(np.int32)
    th = params(3)
    pd = to_dev(th)
    md = torch.zeros_like(pd)
    vd = torch.zeros_like(pd)
    say("mlp train steps")
    losses = kkm.kkm_mlp_train(pd, md, vd, to_dev(Xt), to_dev(Kt), to_dev(idx), lr=1e-3)
    torch.cuda.synchronize()
    t = th.astype(np.float64)
    mo = np.zeros_like(t)
    vo = np.zeros_like(t)
    for s in range(steps):
        ib = idx[s]
        L, g = omlp.loss_and_grad(t, Xt[ib], Kt[np.ix_(ib, ib)].astype(np.float64), D, H1, H2, OUT,
                                  bf16_operands=True)
        assert float(losses[s].item()) == pytest.approx(L, rel=2e-3)
        t, mo, vo = omlp.adam_step(t, mo, vo, g, s + 1, lr=1e-3)
    # each coordinate moved by about lr per step; the two runs stay within a small part of that
    moved = np.abs(t - th)
    diff = np.abs(pd.cpu().numpy() - t)
    assert np.median(diff) <= 0.05 * np.median(moved)
    assert diff.max() <= 2.5 * 1e-3  # at most a couple of steps' worth anywhere (sign flips of tiny grads)


@pytest.mark.parametrize("d", [D, 1024])
def test_mlp_train_fresh_steps_match_oracle(kkm, d):
    """The trainer the benchmark uses, teacher-forced step by step: each step
    starts from the oracle's parameters and Adam moments (rounded to FP32), takes
    its kernel values from the Gram kernel (FP32) on a fresh batch, then loss,
    gradient and Adam; the oracle takes the kernel values from the definition
    (FP64) on the same rows.  The step's gradient is read back from the first
    Adam moment, m' = beta1 m + (1 - beta1) g, and held per parameter block to
    1e-3 of the block's norm, or to three times the change of the oracle's own
    gradient under an FP32-rounding perturbation of the parameters where that
    is larger; the new parameters and moments must be Adam applied to that
    gradient (FP32 rounding only).  A free-running
    comparison over several steps is not a property of the arithmetic: Adam's
    first steps move a parameter by about lr times the sign of its gradient,
    so a gradient within rounding of zero may move either way."""
    import torch
    B, steps, lr, b1 = 64, 3, 1e-3, 0.9
    rng = np.random.default_rng(13 + d)
    Xt = rng.normal(0, 1, (B * steps, d)).astype(np.float32)
    t = params(4, d).astype(np.float64)
    mo = np.zeros_like(t)
    vo = np.zeros_like(t)
    say("mlp train fresh", d)
    for s_ in range(steps):
        t, mo, vo = (a.astype(np.float32).astype(np.float64) for a in (t, mo, vo))
        pd, md, vd = to_dev(t.astype(np.float32)), to_dev(mo.astype(np.float32)), to_dev(vo.astype(np.float32))
        XB = Xt[s_ * B:(s_ + 1) * B]
        loss = kkm.kkm_mlp_train_fresh(pd, md, vd, to_dev(XB), B, kkm.GAUSS, 1.0 / d, t0=s_, lr=lr)
        torch.cuda.synchronize()
        KB = oracle.kernel_matrix(XB, oracle.GAUSS, 1.0 / d)
        L, g = omlp.loss_and_grad(t, XB, KB, d, H1, H2, OUT, bf16_operands=True)
        assert float(loss[0].item()) == pytest.approx(L, rel=1e-4), s_
        # how far the oracle's own gradient moves when its parameters move by
        # FP32 rounding (2^-24 relative): activations next to a bfloat16
        # rounding midpoint then round to the other neighbour, and the
        # first layer's gradient, a sum with heavy cancellation over the batch,
        # carries that at about 1e-3 of its norm
        tp = t * (1 + np.random.default_rng(s_).normal(0, 2.0 ** -24, t.shape))
        _, gp = omlp.loss_and_grad(tp, XB, KB, d, H1, H2, OUT, bf16_operands=True)
        m_gpu = md.cpu().numpy().astype(np.float64)
        g_gpu = (m_gpu - np.float64(np.float32(b1)) * mo) / np.float64(np.float32(1 - b1))
        off = 0
        for shape in omlp.param_shapes(d, H1, H2, OUT):
            size = int(np.prod(shape))
            a, b, c = g_gpu[off:off + size], g[off:off + size], gp[off:off + size]
            nb = np.linalg.norm(b)
            bar = max(1e-3, 3.0 * np.linalg.norm(c - b) / nb)
            say("  step %d %s: |dg|/|g| %.3g, bar %.3g" % (s_, shape, np.linalg.norm(a - b) / nb, bar))
            assert np.linalg.norm(a - b) <= bar * nb + 1e-12, (s_, shape)
            off += size
        pr, mr, vr = omlp.adam_step(t, mo, vo, g_gpu, s_ + 1, lr=lr)
        np.testing.assert_allclose(pd.cpu().numpy(), pr, rtol=0, atol=1e-6)
        np.testing.assert_allclose(vd.cpu().numpy(), vr, rtol=1e-5, atol=1e-12)
        t, mo, vo = omlp.adam_step(t, mo, vo, g, s_ + 1, lr=lr)


def test_mlp_train_fresh_rejects_bad_kernel(kkm):
    import torch
    pd = to_dev(params(4))
    md, vd = torch.zeros_like(pd), torch.zeros_like(pd)
    X = to_dev(np.zeros((128, D), np.float32))
    for kern, gamma, deg in ((kkm.GAUSS, 0.0, 1), (kkm.GAUSS, float("nan"), 1), (kkm.POLY, 1.0, 0)):
        with pytest.raises(kkm.KKMError) as e:
            kkm.kkm_mlp_train_fresh(pd, md, vd, X, 64, kern, gamma, degree=deg)
        assert e.value.status == -1


def test_warm_start_matches_composition(kkm):
    """kkm_warm_start equals the composition of its parts, bit for bit, for any
    number of streams: the forward pass, each restart's k-means++ seeding and
    Lloyd run, and the lowest feature-space objective (lowest restart on ties)."""
    import torch
    rng = np.random.default_rng(31)
    n, d, k, R = 6000, 64, 24, 5
    mu = rng.normal(0, 2, (k, d))
    X = (mu[rng.integers(0, k, n)] + rng.normal(0, 1, (n, d))).astype(np.float32)
    th = params(6, d)
    pd, Xd = to_dev(th), to_dev(X)
    u = np.stack([datagen.uniforms(k, 700 + r) for r in range(R)])
    F = kkm.kkm_mlp_forward(pd, Xd)
    runs = []
    for r in range(R):
        _, seeded = kkm.kkm_feature_kmeanspp(F, k, u[r])
        lab, it, _, obj = kkm.kkm_feature_lloyd(F, k, seeded, max_iter=40, return_objective=True)
        runs.append((obj, r, lab, it))
    best = min(runs, key=lambda x: (x[0], x[1]))
    for streams in (1, 3, 8):
        say("warm start, streams", streams)
        res = kkm.kkm_warm_start(pd, Xd, k, u, max_iter=40, streams=streams)
        torch.cuda.synchronize()
        assert torch.equal(res["labels"], best[2]), streams
        assert res["best"] == best[1] and res["objective"] == best[0]
        assert res["cheap_iters"] == sum(x[3] for x in runs)
    with pytest.raises(kkm.KKMError) as e:
        kkm.kkm_warm_start(pd, Xd, k, np.full((2, k), 1.0))
    assert e.value.status == -1


# the last two take the wide-tile product for the centroid-point dot products
# (k >= 64 and k * n >= 2^20); f = 70 leaves rows without 16-byte alignment
@pytest.mark.parametrize("n,f,k", [(3000, 256, 17), (700, 40, 5), (65, 3, 64), (20000, 256, 100),
                                   (6000, 70, 300)])
def test_feature_lloyd_teacher_forced(kkm, n, f, k):
    import torch
    rng = np.random.default_rng(n + f)
    mu = rng.normal(0, 2, (k, f))
    F = (mu[rng.integers(0, k, n)] + rng.normal(0, 1, (n, f))).astype(np.float32)
    cur = rng.integers(0, k, n).astype(np.int32)
    Fd = to_dev(F)
    for t in range(6):
        ref, Dr, ch = omlp.lloyd_step(F, k, cur)
        say("feature lloyd", n, f, k, "step", t)
        lab, it, tr = kkm.kkm_feature_lloyd(Fd, k, to_dev(cur), max_iter=1)
        torch.cuda.synchronize()
        lab = lab.cpu().numpy()
        srt = np.sort(np.where(np.isfinite(Dr), Dr, np.inf), axis=1)
        gap = srt[:, 1] - srt[:, 0] if k > 1 else np.full(n, np.inf)
        scale = (F.astype(np.float64) ** 2).sum(axis=1) + np.nanmax(np.where(np.isfinite(Dr), Dr, 0), axis=1)
        near = gap < 1e-5 * scale
        assert it == 1 and tr[0] == int((lab != cur).sum())
        assert not ((lab != ref) & ~near).any()
        if ch == 0:
            break
        cur = ref


def test_feature_lloyd_converges_and_rejects_bad_labels(kkm):
    import torch
    rng = np.random.default_rng(5)
    F = rng.normal(0, 1, (500, 8)).astype(np.float32)
    l0 = rng.integers(0, 6, 500).astype(np.int32)
    lab, it, tr = kkm.kkm_feature_lloyd(to_dev(F), 6, to_dev(l0), max_iter=200)
    torch.cuda.synchronize()
    ref, it_ref = omlp.lloyd(F, 6, l0, 200)
    assert tr[-1] == 0
    assert oracle.adjusted_rand_index(lab.cpu().numpy(), ref) >= 0.99
    bad = l0.copy()
    bad[3] = 9
    with pytest.raises(kkm.KKMError):
        kkm.kkm_feature_lloyd(to_dev(F), 6, to_dev(bad), max_iter=3)


# (70000, 16, 12): more than 256 row groups, so each thread of the seed
# selection sums two group totals before the block scan
@pytest.mark.parametrize("n,f,k", [(2000, 256, 16), (333, 7, 9), (40, 3, 40), (8000, 66, 200),
                                   (70000, 16, 12)])
def test_feature_kmeanspp_parity(kkm, n, f, k):
    import torch
    rng = np.random.default_rng(n + k)
    mu = rng.normal(0, 3, (k, f))
    F = (mu[rng.integers(0, k, n)] + rng.normal(0, 1, (n, f))).astype(np.float32)
    u = rng.random(k)
    say("kmeans++", n, f, k)
    seeds, lab = kkm.kkm_feature_kmeanspp(to_dev(F), k, u)
    torch.cuda.synchronize()
    s_ref, lab_ref, margins = omlp.kmeanspp(F, k, u)
    s_gpu = seeds.cpu().numpy()
    diff = np.nonzero(s_gpu != s_ref)[0]
    if diff.size:
        # FP32 distances on the GPU may only move a draw that landed next to a boundary
        assert margins[diff[0]] < 1e-5, (diff[0], margins[diff[0]])
    else:
        D = ((F.astype(np.float64)[:, None] - F.astype(np.float64)[s_ref][None]) ** 2).sum(-1)
        srt = np.sort(D, axis=1)
        near = (srt[:, 1] - srt[:, 0]) < 1e-5 * srt[:, 1] if k > 1 else np.zeros(n, bool)
        assert not ((lab.cpu().numpy() != lab_ref) & ~near).any()


def test_learned_warm_start_gain(kkm):
    """The learned warm start on the first 20000 points of its benchmark
    workload (the 32-component mixture in R^128, Gaussian 1/128; the same
    draws the benchmark uses): phi trained on 2442 batches of 64 fresh points
    (10^7 kernel values, each batch's computed by the Gram kernel), eight
    k-means++ seedings with Lloyd in phi-space (kkm_warm_start), the lowest
    feature-space objective kept, exact refinement; against the plain random
    start at the same precision (FP32).  The gain asserted is the better local
    optimum of the same objective; the exact iterations saved at equal
    precision are recorded (on this workload they are about zero: the warm
    labels sit in a different basin, which takes as many steps to settle)."""
    import torch
    w = datagen.WORKLOADS["learned100k"]
    rows = 20000
    d, k, gamma = w.d, w.k, w.gamma
    B, steps = 64, 2442
    Xtr, _ = datagen.gmm(B * steps, d, k, 0.5, w.train_seed, means=w.means())
    Xte, truth = w.points(rows=rows)
    l0 = w.labels0(rows=rows)
    pd = to_dev(datagen.mlp_init_params(d, H1, H2, OUT, seed=w.init_seed))
    md, vd = torch.zeros_like(pd), torch.zeros_like(pd)
    say("learned: training")
    losses = kkm.kkm_mlp_train_fresh(pd, md, vd, to_dev(Xtr), B, kkm.GAUSS, gamma, lr=1e-3).cpu().numpy()
    say("learned: loss %.4g -> %.4g" % (losses[:10].mean(), losses[-10:].mean()))
    assert losses[-10:].mean() < 0.5 * losses[:10].mean()
    Xd = to_dev(Xte)
    u = np.stack([datagen.uniforms(k, w.label_seed + 30003 + r) for r in range(8)])
    ws = kkm.kkm_warm_start(pd, Xd, k, u, max_iter=60, streams=4)
    warm = ws["labels"]
    plain = kkm.kkm_fit_ex(Xd, k, to_dev(l0), kkm.GAUSS, gamma, max_iter=300)
    learned = kkm.kkm_fit_ex(Xd, k, warm, kkm.GAUSS, gamma, max_iter=300)
    torch.cuda.synchronize()
    K_or = oracle.kernel_matrix(Xte, oracle.GAUSS, gamma)
    ref = oracle.fit(K_or, k, warm.cpu().numpy(), 300)
    ari_oracle = oracle.adjusted_rand_index(learned["labels"].cpu().numpy(), ref["labels"])
    say("learned: cheap %d, exact %d vs plain %d (saved at equal precision: %d); J %.6g vs plain "
        "%.6g; ARI vs oracle-from-warm %.4f; ARI vs truth %.4f vs plain %.4f" % (
            ws["cheap_iters"], learned["iters"], plain["iters"], plain["iters"] - learned["iters"],
            learned["objective"], plain["objective"], ari_oracle,
            oracle.adjusted_rand_index(learned["labels"].cpu().numpy(), truth),
            oracle.adjusted_rand_index(plain["labels"].cpu().numpy(), truth)))
    assert ari_oracle >= 0.99
    assert learned["objective"] < plain["objective"] * (1 - 1e-3)


def test_concurrent_streams_match_sequential(kkm):
    """The library holds no shared mutable state between calls: k-means++
    seedings and feature-space Lloyd runs issued from four host threads on
    four streams give exactly the labels of the same calls made one after
    another."""
    import threading

    import torch
    rng = np.random.default_rng(21)
    n, f, k = 6000, 64, 24
    mu = rng.normal(0, 2, (k, f))
    F = to_dev((mu[rng.integers(0, k, n)] + rng.normal(0, 1, (n, f))).astype(np.float32))
    us = [datagen.uniforms(k, 900 + r) for r in range(8)]

    def run(r):
        _, seeded = kkm.kkm_feature_kmeanspp(F, k, us[r])
        lab, it, _, obj = kkm.kkm_feature_lloyd(F, k, seeded, max_iter=50, return_objective=True)
        return lab, it, obj

    seq = [run(r) for r in range(8)]
    torch.cuda.synchronize()
    out = [None] * 8
    main = torch.cuda.current_stream()
    streams = [torch.cuda.Stream() for _ in range(4)]

    def worker(t):
        with torch.cuda.stream(streams[t]):
            streams[t].wait_stream(main)
            for r in range(t, 8, 4):
                out[r] = run(r)

    threads = [threading.Thread(target=worker, args=(t,)) for t in range(4)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    torch.cuda.synchronize()
    for r in range(8):
        assert torch.equal(seq[r][0], out[r][0]), r
        assert seq[r][1] == out[r][1] and seq[r][2] == out[r][2], r
