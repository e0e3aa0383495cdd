"""The matrix-free step (kernel values recomputed on the MFMA inside the step,
no stored K) against the FP64 oracle, on the GPU.

* FP32 product: teacher-forced steps against the oracle's steps on K from the
  definition, with the FP32 parity rules of the stored-K path (distances,
  labels away from near-ties, sizes, changed count, J, centroid norms): the
  rings workload, the MNIST-shaped and 64-component prefixes, ragged shapes
  over several strips and chunks, k = 1, k = n, empty clusters under both
  policies;
* BF16 product: the same rules against the oracle fed the bfloat16-rounded
  points the product multiplies; FP8: against the oracle fed s_i q_il, with the
  distance bound widened by the FP8 matrix unit's measured accumulation term
  (2^-15 sum |x y| per entry, as for the stored-K FP8 Gram);
* whole runs of kkm_fit_matfree against oracle.fit and against the stored-K
  kkm_fit_ex on the same labels; bitwise repeatability; argument errors;
* the learned warm-start workload's size (n = 100000, d = 128, BF16 product):
  one step, E at sampled rows against the oracle's cluster sums of the rounded
  points, and the properties every row must satisfy.
"""
import sys

import numpy as np
import pytest

import datagen
import oracle
from parity import D_TOL, compare_step, gram_bound
from quantref import bf16_round, fp8_dequantised

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


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def teacher_forced(kkm, X, kern, gamma, coef0, degree, k, labels0, steps, prec=0, empty_policy=0,
                   what=""):
    """Steps of kkm_iterate_matfree from the oracle's labels of each step."""
    import torch
    Xe = {0: X, 1: bf16_round(X), 2: fp8_dequantised(X)}[prec]
    K_or = oracle.kernel_matrix(Xe, kern, gamma, coef0, degree)
    Xd = to_dev(X)
    cur = np.ascontiguousarray(labels0, dtype=np.int32)
    flips = 0
    for t in range(steps):
        orc = oracle.step(K_or, k, cur, empty_policy)
        say("  matfree step", t, what)
        lab, cnt, ch, J, D, C, dg = kkm.kkm_iterate_matfree(
            Xd, to_dev(cur), k, kern, gamma, coef0, degree, gram_prec=prec,
            empty_policy=empty_policy, D_out=True, ctilde_out=True, diagK_out=True)
        torch.cuda.synchronize()
        if t == 0:
            # K_ii from the squared norm of the rounded row, within the FP32 bound
            bd = np.diag(gram_bound(Xe, kern, gamma, coef0, degree, K_or))
            assert (np.abs(dg.cpu().numpy() - np.diag(K_or)) <= bd).all(), what
        if prec == 2:
            fp8_step_check(Xe, K_or, kern, gamma, coef0, degree, k, cur, orc, D.cpu().numpy(),
                           lab.cpu().numpy(), cnt.cpu().numpy(), int(ch.item()), what)
        else:
            flips += compare_step(K_or, k, cur, orc, D.cpu().numpy(), lab.cpu().numpy(),
                                  cnt.cpu().numpy(), int(ch.item()), float(J.item()),
                                  C.cpu().numpy(), what="%s step %d" % (what, t))
        if orc["n_changed"] == 0:
            break
        cur = orc["labels"]
    return flips


def fp8_step_check(Xe, K_or, kern, gamma, coef0, degree, k, cur, orc, D, lab, cnt, ch, what):
    """FP8 product: D_ic is built from K_ii, the mean of K over cluster c's row
    entries and the mean over its block, so a per-entry bound B on K (FP32
    accumulation plus the matrix unit's 2^-15 sum |x y|, times 4) bounds its
    error by B_ii + 2 max_j B_ij + max B; labels may differ only where the
    oracle's gap is below twice that."""
    B = gram_bound(Xe, kern, gamma, coef0, degree, K_or, 2.0 ** -15)
    bd = np.diag(B) + 2 * B.max(axis=1) + B.max()
    fin = np.isfinite(orc["D"])
    assert np.array_equal(np.isfinite(D), fin), what
    err = np.where(fin, np.abs(D.astype(np.float64) - np.where(fin, orc["D"], 0)), 0)
    sc = np.abs(np.diag(K_or)) + 2 * np.abs(K_or).max(axis=1) + np.abs(K_or).max()
    assert (err <= 2 * bd[:, None] + D_TOL * sc[:, None]).all(), what
    near = orc["gap"] < 2 * (2 * bd + D_TOL * sc)
    assert not ((lab != orc["labels"]) & ~near).any(), what
    assert np.array_equal(cnt, np.bincount(lab, minlength=k)), what
    assert ch == int((lab != cur).sum()), what


def test_matfree_rings(kkm):
    w = datagen.WORKLOADS["rings"]
    X, _ = w.points()
    flips = teacher_forced(kkm, X, w.kernel, w.gamma, w.coef0, w.degree, w.k, w.labels0(),
                           w.max_iter, what="rings")
    assert flips <= 2


def test_matfree_mnist_like_prefix(kkm):
    w = datagen.WORKLOADS["mnist_like"]
    X, _ = w.points(rows=2500)
    teacher_forced(kkm, X, w.kernel, w.gamma, w.coef0, w.degree, w.k, w.labels0(rows=2500), 6,
                   what="mnist_like[:2500]")


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_matfree_gmm_prefix(kkm, prec):
    w = datagen.WORKLOADS["gmm200k"]
    X, _ = w.points(rows=3000)
    teacher_forced(kkm, X, w.kernel, w.gamma, w.coef0, w.degree, w.k, w.labels0(rows=3000), 4,
                   prec=prec, what="gmm200k[:3000] prec %d" % prec)


@pytest.mark.parametrize("prec", [1, 2])
def test_matfree_learned_workload_prefix(kkm, prec):
    w = datagen.WORKLOADS["learned100k"]
    X, _ = w.points(rows=4100)
    teacher_forced(kkm, X, w.kernel, w.gamma, w.coef0, w.degree, w.k, w.labels0(rows=4100), 4,
                   prec=prec, what="learned100k[:4100] prec %d" % prec)


# ragged n over one to several 128-point strips and 128-position chunks, odd d
@pytest.mark.parametrize("n,d,k", [(1, 2, 1), (7, 3, 2), (65, 4, 7), (129, 33, 5), (1025, 5, 3),
                                   (2049, 70, 33), (3000, 6, 1)])
@pytest.mark.parametrize("kernel", ["linear", "poly", "gauss"])
def test_matfree_shapes(kkm, n, d, k, kernel):
    rng = np.random.default_rng(2000 + n + d)
    X = rng.normal(0, 1, (n, d)).astype(np.float32)
    code = {"linear": kkm.LINEAR, "poly": kkm.POLY, "gauss": kkm.GAUSS}[kernel]
    gamma = 1.0 / d if kernel != "linear" else 1.0
    teacher_forced(kkm, X, code, gamma, 1.0 if kernel == "poly" else 0.0, 2 if kernel == "poly" else 1,
                   k, rng.integers(0, k, n).astype(np.int32), 4, what="n=%d d=%d %s" % (n, d, kernel))


def test_matfree_singletons_and_empty_clusters(kkm):
    rng = np.random.default_rng(5)
    X = rng.normal(0, 1, (40, 3)).astype(np.float32)
    teacher_forced(kkm, X, kkm.POLY, 1.0, 1.0, 2, 40, np.arange(40, dtype=np.int32), 1, what="k=n")
    lab = rng.integers(0, 3, 40).astype(np.int32)
    lab[:5] = 4
    for pol in (0, 1):
        teacher_forced(kkm, X, kkm.POLY, 1.0, 1.0, 2, 6, lab, 4, empty_policy=pol,
                       what="empty policy %d" % pol)


def test_matfree_fit_matches_oracle_and_stored_K(kkm):
    import torch
    w = datagen.WORKLOADS["rings"]
    X, _ = w.points()
    l0 = w.labels0()
    K_or = oracle.kernel_matrix(X, w.kernel, w.gamma, w.coef0, w.degree)
    ref = oracle.fit(K_or, w.k, l0, w.max_iter)
    say("fit matfree rings")
    r = kkm.kkm_fit_matfree(to_dev(X), w.k, to_dev(l0), w.kernel, w.gamma, w.coef0, w.degree,
                            max_iter=w.max_iter, check_convergence=True)
    s = kkm.kkm_fit_ex(to_dev(X), w.k, to_dev(l0), w.kernel, w.gamma, w.coef0, w.degree,
                       max_iter=w.max_iter, check_convergence=True)
    torch.cuda.synchronize()
    recs = oracle.trajectory(K_or, w.k, l0, w.max_iter)
    tie = any((st["gap"] < 1e-6 * 4).any() for _, st in recs)
    if not tie:
        np.testing.assert_array_equal(r["labels"].cpu().numpy(), ref["labels"])
        assert r["iters"] == ref["iters"]
    scale = np.abs(np.diag(K_or)).sum()
    assert abs(r["objective"] - ref["objective"]) <= 2e-5 * scale
    np.testing.assert_allclose(r["J_trace"], ref["J_trace"], rtol=0, atol=2e-5 * scale)
    # the stored-K form from the same labels: the same labels, J to FP32 order
    assert oracle.adjusted_rand_index(r["labels"].cpu().numpy(), s["labels"].cpu().numpy()) == 1.0
    assert abs(r["objective"] - s["objective"]) <= 2e-5 * scale


def test_matfree_fixed_iterations_zero_and_errors(kkm):
    import torch
    rng = np.random.default_rng(9)
    X = rng.normal(0, 1, (500, 4)).astype(np.float32)
    l0 = rng.integers(0, 5, 500).astype(np.int32)
    K_or = oracle.kernel_matrix(X, oracle.GAUSS, 0.3)
    r = kkm.kkm_fit_matfree(to_dev(X), 5, to_dev(l0), kkm.GAUSS, 0.3, max_iter=7,
                            check_convergence=False)
    assert r["iters"] == 7
    ref = oracle.fit(K_or, 5, l0, 7, check_convergence=False)
    assert abs(r["objective"] - ref["objective"]) <= 2e-5 * 500
    r0 = kkm.kkm_fit_matfree(to_dev(X), 5, to_dev(l0), kkm.GAUSS, 0.3, max_iter=0)
    assert r0["iters"] == 0
    np.testing.assert_array_equal(r0["labels"].cpu().numpy(), l0)
    assert abs(r0["objective"] - oracle.objective(K_or, 5, l0)) <= 2e-5 * 500
    bad = l0.copy()
    bad[3] = 7
    with pytest.raises(kkm.KKMError) as e:
        kkm.kkm_fit_matfree(to_dev(X), 5, to_dev(bad), kkm.GAUSS, 0.3, max_iter=3)
    assert e.value.status == -2
    with pytest.raises(kkm.KKMError) as e:
        kkm.kkm_fit_matfree(to_dev(X), 5, to_dev(l0), kkm.GAUSS, -1.0, max_iter=3)
    assert e.value.status == -1
    Xn = X.copy()
    Xn[10, 1] = np.nan
    with pytest.raises(kkm.KKMError) as e:
        kkm.kkm_fit_matfree(to_dev(Xn), 5, to_dev(l0), kkm.GAUSS, 0.3, max_iter=3)
    assert e.value.status == -6
    torch.cuda.synchronize()


def test_matfree_is_deterministic(kkm):
    import torch
    w = datagen.WORKLOADS["gmm200k"]
    X, _ = w.points(rows=5000)
    Xd = to_dev(X)
    l0 = to_dev(w.labels0(rows=5000))
    a = kkm.kkm_iterate_matfree(Xd, l0, w.k, w.kernel, w.gamma, gram_prec=kkm.BF16, D_out=True,
                                ctilde_out=True)
    b = kkm.kkm_iterate_matfree(Xd, l0, w.k, w.kernel, w.gamma, gram_prec=kkm.BF16, D_out=True,
                                ctilde_out=True)
    torch.cuda.synchronize()
    for x, y in zip(a[:6], b[:6]):
        assert torch.equal(x, y)


def test_matfree_learned_workload_full_size(kkm):
    """n = 100000, d = 128, k = 32, BF16 product: one step from the random
    labels.  E = K V^T recovered at sampled rows (and the last rows) from the
    step's distances and centroid norms, against the oracle's cluster sums of
    the bfloat16-rounded points (no K formed); on every row the properties
    that hold at any size."""
    import torch
    w = datagen.WORKLOADS["learned100k"]
    X, _ = w.points()
    l0 = w.labels0()
    n = w.n
    say("matfree full size", n, w.d, w.k)
    lab, cnt, ch, J_in, D, C, dg = kkm.kkm_iterate_matfree(
        to_dev(X), to_dev(l0), w.k, w.kernel, w.gamma, gram_prec=kkm.BF16, D_out=True,
        ctilde_out=True, diagK_out=True)
    torch.cuda.synchronize()
    D = D.cpu().numpy().astype(np.float64)
    C = C.cpu().numpy().astype(np.float64)
    dgl = dg.cpu().numpy().astype(np.float64)
    lab = lab.cpu().numpy()
    assert np.all(dgl == 1.0)
    counts_in = np.bincount(l0, minlength=w.k).astype(np.float64)
    live = counts_in > 0
    E = 0.5 * (dgl[:, None] + C[None, :] - D)
    assert np.array_equal(lab, np.argmin(D, axis=1).astype(np.int32))
    assert np.array_equal(cnt.cpu().numpy(), np.bincount(lab, minlength=w.k))
    assert int(ch.item()) == int((lab != l0).sum())
    j_rows = D[np.arange(n), l0]
    assert abs(float(J_in.item()) - j_rows.sum()) <= 1e-9 * np.abs(j_rows).sum()
    scale = np.abs(dgl).max() + 2 * np.abs(E[:, live]).max() + np.abs(C[live]).max()
    cmean = np.array([E[l0 == c, c].mean() if live[c] else 0.0 for c in range(w.k)])
    assert (np.abs(cmean - C)[live] / scale).max() <= D_TOL
    rng = np.random.default_rng(77)
    R = np.unique(np.concatenate([rng.integers(0, n, 48), np.arange(n - 8, n)]))
    S_or = oracle.cluster_row_sums(bf16_round(X), l0, w.k, R, w.kernel, w.gamma)
    E_or = np.where(live[None, :], S_or / np.maximum(counts_in, 1)[None, :], 0.0)
    sig = np.abs(dgl[R]) + (2 * np.abs(E_or[:, live]) + np.abs(C[live])[None, :]).max(axis=1)
    err = (np.abs(E[R][:, live] - E_or[:, live]) / sig[:, None]).max()
    say("  E error %.3g sigma" % err)
    assert err <= D_TOL, "E error %.3g sigma" % err
