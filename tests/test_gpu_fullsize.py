"""Parity at the benchmark's full sizes, in the launch configuration the
benchmark times (default chunking, FP32 K for the plain path), on outputs the
oracle can compute one by one:

* Gram: sampled entries (random pairs, the ragged last rows, the diagonal)
  against kappa(x_i, x_j) in FP64, and exact symmetry;
* one step: E = K V^T at sampled rows (recovered from the distances and the
  centroid norms) against the oracle's cluster row sums taken from the points;
  on every row, properties that hold at any size: the centroid norms are the
  cluster means of E, each label is the argmin of its row of D, the sizes and
  the changed count follow from the labels, J is the sum of the own-cluster
  distances;
* the precision form (BF16 product and K) and the feature map's forward pass
  at n = 200000 on sampled rows;
* batched: sampled problems of the 512-problem workload against their own
  single runs (bit for bit), and the tuned chunking against the default one.
"""
import sys

import numpy as np
import pytest

import datagen
import oracle

from parity import D_TOL, gram_bound_pairs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def kkm():
    import torch  # noqa: F401
    import paper_2501_05587_amd as kkm
    kkm.lib()
    return kkm


def workload_step_check(kkm, w, rows_sampled=48, pairs=3000):
    import torch
    dev = torch.device("cuda:0")
    say("full size:", w.name, "n=%d d=%d k=%d" % (w.n, w.d, w.k))
    X, _ = w.points()
    l0 = w.labels0()
    Xd = torch.from_numpy(X).to(dev)
    say("  gram")
    K, diag = kkm.kkm_gram(Xd, w.kernel, w.gamma, w.coef0, w.degree)
    torch.cuda.synchronize()
    rng = np.random.default_rng(w.data_seed + 900)
    n = w.n
    I = np.concatenate([rng.integers(0, n, pairs), np.arange(n - 40, n), rng.integers(0, n, 40)])
    J = np.concatenate([rng.integers(0, n, pairs), rng.integers(0, n, 40), np.arange(n - 40, n)])
    It, Jt = torch.from_numpy(I).to(dev), torch.from_numpy(J).to(dev)
    kij = K[It, Jt].double().cpu().numpy()
    kji = K[Jt, It].double().cpu().numpy()
    np.testing.assert_array_equal(kij, kji)
    k_or = np.array([oracle.kappa(X[i], X[j], w.kernel, w.gamma, w.coef0, w.degree)
                     for i, j in zip(I, J)])
    bound = gram_bound_pairs(X, I, J, w.kernel, w.gamma, w.coef0, w.degree, k_or)
    ratio = np.abs(kij - k_or) / bound
    assert ratio.max() <= 1.0, "K error %.3g of the bound at pair %d" % (ratio.max(), ratio.argmax())
    dgl = diag.cpu().numpy().astype(np.float64)
    d_or = np.array([oracle.kappa(X[i], X[i], w.kernel, w.gamma, w.coef0, w.degree)
                     for i in range(n - 20, n)])
    np.testing.assert_allclose(dgl[n - 20:], d_or, rtol=1e-5)

    say("  one step")
    lab, cnt, ch, J_in, D, C = kkm.kkm_iterate(K, diag, torch.from_numpy(l0).to(dev), w.k,
                                               D_out=True, ctilde_out=True)
    torch.cuda.synchronize()
    del K
    torch.cuda.empty_cache()
    D = D.cpu().numpy().astype(np.float64)
    C = C.cpu().numpy().astype(np.float64)
    lab = lab.cpu().numpy()
    counts_in = np.bincount(l0, minlength=w.k).astype(np.float64)
    live = counts_in > 0
    E = 0.5 * (dgl[:, None] + C[None, :] - D)   # E_ic recovered from the step's own terms
    # properties on every row
    assert np.array_equal(lab, np.argmin(D, axis=1).astype(np.int32))
    assert np.array_equal(cnt.cpu().numpy(), np.bincount(lab, minlength=w.k))
    assert int(ch.item()) == int((lab != l0).sum())
    j_rows = D[np.arange(n), l0]
    assert abs(float(J_in.item()) - j_rows.sum()) <= 1e-9 * np.abs(j_rows).sum()
    scale = np.abs(dgl).max() + 2 * np.abs(E[:, live]).max() + np.abs(C[live]).max()
    cmean = np.array([E[l0 == c, c].mean() if live[c] else 0.0 for c in range(w.k)])
    assert (np.abs(cmean - C)[live] / scale).max() <= D_TOL
    # E at sampled rows against the oracle's sums from the points
    R = np.unique(np.concatenate([rng.integers(0, n, rows_sampled), np.arange(n - 8, n)]))
    say("  oracle rows:", len(R))
    S_or = oracle.cluster_row_sums(X, l0, w.k, R, w.kernel, w.gamma, w.coef0, w.degree)
    E_or = np.where(live[None, :], S_or / np.maximum(counts_in, 1)[None, :], 0.0)
    sig = np.abs(dgl[R]) + (2 * np.abs(E_or[:, live]) + np.abs(C[live])[None, :]).max(axis=1)
    err = (np.abs(E[R][:, live] - E_or[:, live]) / sig[:, None]).max()
    assert err <= D_TOL, "E error %.3g sigma" % err


def test_gmm200k_full_size(kkm):
    workload_step_check(kkm, datagen.WORKLOADS["gmm200k"])


def test_mnist_like_full_size(kkm):
    workload_step_check(kkm, datagen.WORKLOADS["mnist_like"])


def test_gmm200k_bf16_full_size(kkm):
    """The precision form at full size (BF16 product, K stored as bfloat16): the
    oracle is fed the bfloat16-rounded points the product multiplies; K may
    differ from it by the FP32 accumulation bound plus bfloat16's unit
    roundoff of the stored value, and E by the mean of those."""
    import torch
    from quantref import bf16_round
    w = datagen.WORKLOADS["gmm200k"]
    dev = torch.device("cuda:0")
    say("full size bf16:", w.name)
    X, _ = w.points()
    Xq = bf16_round(X).astype(np.float32)
    l0 = w.labels0()
    K, diag = kkm.kkm_gram(torch.from_numpy(X).to(dev), w.kernel, w.gamma, gram_prec=kkm.BF16,
                           k_store=kkm.BF16)
    torch.cuda.synchronize()
    rng = np.random.default_rng(909)
    n = w.n
    I = np.concatenate([rng.integers(0, n, 2000), np.arange(n - 30, n)])
    J = np.concatenate([rng.integers(0, n, 2000), rng.integers(0, n, 30)])
    It, Jt = torch.from_numpy(I).to(dev), torch.from_numpy(J).to(dev)
    kij = K[It, Jt].float().double().cpu().numpy()
    assert np.array_equal(kij, K[Jt, It].float().double().cpu().numpy())
    k_or = np.array([oracle.kappa(Xq[i], Xq[j], w.kernel, w.gamma) for i, j in zip(I, J)])
    bound = gram_bound_pairs(Xq, I, J, w.kernel, w.gamma, 0.0, 1, k_or) + 2.0 ** -8 * np.abs(k_or)
    assert (np.abs(kij - k_or) / bound).max() <= 1.0
    say("  one step")
    lab, cnt, ch, J_in, D, C = kkm.kkm_iterate(K, diag, torch.from_numpy(l0).to(dev), w.k,
                                               D_out=True, ctilde_out=True)
    torch.cuda.synchronize()
    del K
    torch.cuda.empty_cache()
    D = D.cpu().numpy().astype(np.float64)
    C = C.cpu().numpy().astype(np.float64)
    dgl = diag.cpu().numpy().astype(np.float64)
    lab = lab.cpu().numpy()
    assert np.array_equal(lab, np.argmin(D, axis=1).astype(np.int32))
    counts = np.bincount(l0, minlength=w.k).astype(np.float64)
    E = 0.5 * (dgl[:, None] + C[None, :] - D)
    R = np.unique(np.concatenate([rng.integers(0, n, 40), np.arange(n - 8, n)]))
    S_or = oracle.cluster_row_sums(Xq, l0, w.k, R, w.kernel, w.gamma)
    E_or = S_or / counts[None, :]
    # per row: the mean over each cluster of the per-entry bounds, bounded by
    # their maximum (rows' kernel values are <= 1 under the Gaussian)
    sig = np.abs(dgl[R]) + (2 * np.abs(E_or) + np.abs(C)[None, :]).max(axis=1)
    tol = 2.0 ** -8 * np.abs(E_or) + D_TOL * sig[:, None]
    assert (np.abs(E[R] - E_or) <= tol).all(), (np.abs(E[R] - E_or) / tol).max()


def test_feature_map_forward_full_size(kkm):
    """phi_theta on all 200000 points of the mixture (the warm start's forward
    pass), sampled rows against the FP64 reference with the same bfloat16
    operand rounding."""
    import torch
    from oracle import mlp as omlp
    w = datagen.WORKLOADS["gmm200k"]
    X, _ = w.points()
    th = datagen.mlp_init_params(w.d, 512, 512, 256, seed=910)
    say("full size forward: n=%d d=%d" % X.shape)
    F = kkm.kkm_mlp_forward(torch.from_numpy(th).cuda(), torch.from_numpy(X).cuda())
    torch.cuda.synchronize()
    R = np.unique(np.concatenate([np.random.default_rng(911).integers(0, w.n, 64),
                                  np.arange(w.n - 8, w.n)]))
    Fs = F[torch.from_numpy(R).cuda()].cpu().numpy().astype(np.float64)
    ref, _ = omlp.forward(th.astype(np.float64), X[R], w.d, 512, 512, 256, bf16_operands=True)
    # Both sides multiply bfloat16-rounded operands, accumulating in FP32 (GPU)
    # or FP64 (reference).  An activation that lies next to a bfloat16 rounding
    # midpoint can round to the other neighbour on one side, so the outputs may
    # differ by a few operand spacings; the bar is one bfloat16 spacing (2^-7)
    # of the output scale.  A wrong layer, bias or activation misses it by
    # orders of magnitude.
    err = np.abs(Fs - ref).max()
    say("  forward error: %.3g (%.3g of one bfloat16 spacing of max|F|)" % (
        err, err / (2.0 ** -7 * np.abs(ref).max())))
    assert err <= 2.0 ** -7 * np.abs(ref).max(), err


def test_batched_512_full_size(kkm):
    import torch
    from paper_2501_05587_amd import autotune
    dev = torch.device("cuda:0")
    specs = datagen.batched_instances(512)
    probs, labs = [], []
    for s in specs:
        X, _ = datagen.gmm(s["n"], s["d"], s["k"], s["sigma"], s["seed"])
        probs.append(dict(X=torch.from_numpy(X).to(dev), k=s["k"], kernel=kkm.GAUSS,
                          gamma=s["gamma"]))
        labs.append(datagen.uniform_labels(s["n"], s["k"], s["label_seed"]))
    l0 = torch.from_numpy(np.concatenate(labs)).to(dev)
    say("batched: 512 problems, default chunking")
    base = kkm.kkm_fit_batched(probs, l0, gram_prec=kkm.BF16, k_store=kkm.F32, max_iter=30,
                               check_convergence=False)
    torch.cuda.synchronize()
    lab_b = base["labels"].cpu().numpy()
    off = np.concatenate([[0], np.cumsum([s["n"] for s in specs])])
    nn = np.array([s["n"] for s in specs])
    pick = sorted({int(np.argmax(nn)), int(np.argmin(nn)), int(np.argsort(nn)[256]), 0, 511})
    for b in pick:
        say("  single run of problem", b, "n=%d d=%d k=%d" % (specs[b]["n"], specs[b]["d"], specs[b]["k"]))
        p = probs[b]
        one = kkm.kkm_fit_ex(p["X"], p["k"], l0[off[b]:off[b + 1]], kkm.GAUSS, p["gamma"],
                             gram_prec=kkm.BF16, k_store=kkm.F32, max_iter=30,
                             check_convergence=False)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(lab_b[off[b]:off[b + 1]], one["labels"].cpu().numpy())
        assert base["objective"][b] == one["objective"] and base["iters"][b] == one["iters"]
    say("batched: tuned chunking")
    tuned = kkm.kkm_fit_batched(autotune.apply(probs, autotune.load(torch=torch), 0), l0,
                                gram_prec=kkm.BF16, k_store=kkm.F32, max_iter=30,
                                check_convergence=False)
    torch.cuda.synchronize()
    agree = (tuned["labels"] == base["labels"]).float().mean().item()
    assert agree >= 0.999, agree
    np.testing.assert_allclose(tuned["objective"], base["objective"], rtol=1e-4)
    # the timed configuration (BF16 product, FP32 K, tuned chunk heights, the
    # captured graph) against the FP64 oracle on the points the product
    # multiplies (bfloat16-rounded): the smallest problem of each d and the
    # smallest overall, whole runs of 30 steps
    from quantref import bf16_round
    lab_t = tuned["labels"].cpu().numpy()
    order = np.argsort(nn)
    sub = sorted({int(order[0])} | {int(next(b for b in order if specs[b]["d"] == dd))
                                     for dd in (32, 64, 128, 256)})
    for b in sub:
        sp = specs[b]
        say("  oracle run of problem", b, "n=%d d=%d k=%d" % (sp["n"], sp["d"], sp["k"]))
        X, _ = datagen.gmm(sp["n"], sp["d"], sp["k"], sp["sigma"], sp["seed"])
        K_or = oracle.kernel_matrix(bf16_round(X), oracle.GAUSS, sp["gamma"])
        lab0 = labs[b]
        ref = oracle.fit(K_or, sp["k"], lab0, 30, check_convergence=False)
        recs = oracle.trajectory(K_or, sp["k"], lab0, 30, check_convergence=False)
        tie = any((st["gap"] < 1e-6 * 4).any() for _, st in recs)
        if not tie:
            np.testing.assert_array_equal(lab_t[off[b]:off[b + 1]], ref["labels"], err_msg="problem %d" % b)
        scale = np.abs(np.diag(K_or)).sum() + np.abs(K_or).max() * sp["n"]
        assert abs(tuned["objective"][b] - ref["objective"]) <= 1e-5 * scale, b
        assert oracle.adjusted_rand_index(lab_t[off[b]:off[b + 1]], ref["labels"]) >= 0.99, b
    del probs
    torch.cuda.empty_cache()
