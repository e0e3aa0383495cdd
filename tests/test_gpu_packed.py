"""The strip-packed symmetric K (the upper triangle in strips of W columns,
W = 1024 for FP32 and bfloat16) and the step that reads each stored
entry once, on the GPU.

* layout: every stored entry of the packed K equals the dense K's entry bit
  for bit (the same tiles, the same products), over one to several strips,
  ragged n, FP32 and bfloat16 storage, all three kernels;
* teacher-forced steps against the FP64 oracle with the FP32 parity rules of
  the dense path: FP32 storage against K from the definition; bfloat16
  storage against the oracle's step on the stored bfloat16 values (exact
  inputs); prefixes of the benchmark workloads and shapes over several
  strips and chunks, k from 1 to 128, empty clusters under both policies;
* whole runs of kkm_fit_packed against the dense kkm_fit_ex and oracle.fit;
  bitwise repeatability; argument errors;
* the benchmark's size (n = 200000, d = 1024, k = 64, FP32): one step, E at
  sampled rows against the oracle's cluster sums from the points, and the
  properties every row must satisfy.
"""
import sys

import numpy as np
import pytest

import datagen
import oracle
from parity import D_TOL, compare_step

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


def lgw(kkm, k_store):
    return 10  # 1024-column strips for either storage type


def row_offset(i, lg, ns):
    """Start of row i in the packed layout: rows of strips b < s_i hold
    (ns - b) W entries each, rows of strip s_i (ns - s_i) W."""
    W = 1 << lg
    s = i >> lg
    return W * W * (s * ns - s * (s - 1) // 2) + (i - s * W) * (ns - s) * W


def unpack(kkm, Kp, n, k_store):
    """Dense n x n matrix from the packed entries (float64); entries left of a
    row's strip come from the mirrored stored entry."""
    lg = lgw(kkm, k_store)
    W = 1 << lg
    ns = (n + W - 1) // W
    v = Kp.float().cpu().numpy().astype(np.float64)
    D = np.zeros((n, n))
    for i in range(n):
        s = i >> lg
        o = row_offset(i, lg, ns)
        D[i, s * W:] = v[o:o + n - s * W]
    for i in range(n):
        s = i >> lg
        D[i, :s * W] = D[:s * W, i]
    return D


@pytest.mark.parametrize("n,d", [(1, 3), (7, 2), (1025, 5), (2049, 33), (3000, 16), (4100, 8)])
@pytest.mark.parametrize("kernel", ["linear", "poly", "gauss"])
@pytest.mark.parametrize("store", ["f32", "bf16"])
def test_packed_gram_equals_dense(kkm, n, d, kernel, store):
    import torch
    rng = np.random.default_rng(n + d)
    X = rng.normal(0, 1, (n, d)).astype(np.float32)
    code = {"linear": kkm.LINEAR, "poly": kkm.POLY, "gauss": kkm.GAUSS}[kernel]
    ks = kkm.F32 if store == "f32" else kkm.BF16
    gp = kkm.F32 if store == "f32" else kkm.BF16
    gamma = 1.0 / d if kernel != "linear" else 1.0
    c0, deg = (1.0, 2) if kernel == "poly" else (0.0, 1)
    say("packed gram", n, d, kernel, store)
    Kd, dd = kkm.kkm_gram(to_dev(X), code, gamma, c0, deg, gram_prec=gp, k_store=ks)
    Kp, dp = kkm.kkm_gram_packed(to_dev(X), code, gamma, c0, deg, gram_prec=gp, k_store=ks)
    torch.cuda.synchronize()
    assert torch.equal(dd, dp)
    dense = Kd.float().cpu().numpy().astype(np.float64)
    np.testing.assert_array_equal(unpack(kkm, Kp, n, ks), dense)


def teacher_forced(kkm, X, kern, gamma, coef0, degree, k, labels0, steps, store="f32",
                   empty_policy=0, what=""):
    """Steps of kkm_iterate_packed from the oracle's labels of each step."""
    import torch
    ks = kkm.F32 if store == "f32" else kkm.BF16
    Xd = to_dev(X)
    Kp, dg = kkm.kkm_gram_packed(Xd, kern, gamma, coef0, degree, gram_prec=ks, k_store=ks)
    if store == "f32":
        K_or = oracle.kernel_matrix(X, kern, gamma, coef0, degree)
    else:
        # exact inputs: the oracle steps on the stored bfloat16 values
        Kd, _ = kkm.kkm_gram(Xd, kern, gamma, coef0, degree, gram_prec=ks, k_store=ks)
        torch.cuda.synchronize()
        K_or = Kd.float().cpu().numpy().astype(np.float64)
        del Kd
    cur = np.ascontiguousarray(labels0, dtype=np.int32)
    flips = 0
    for t in range(steps):
        orc = oracle.step(K_or, k, cur, empty_policy)
        say("  packed step", t, what)
        lab, cnt, ch, J, D, C = kkm.kkm_iterate_packed(Kp, dg, to_dev(cur), k, empty_policy,
                                                       D_out=True, ctilde_out=True)
        torch.cuda.synchronize()
        flips += compare_step(K_or, k, cur, orc, D.cpu().numpy(), lab.cpu().numpy(),
                              cnt.cpu().numpy(), int(ch.item()), float(J.item()), C.cpu().numpy(),
                              what="%s step %d" % (what, t))
        if orc["n_changed"] == 0:
            break
        cur = orc["labels"]
    return flips


def test_packed_rings(kkm):
    w = datagen.WORKLOADS["rings"]
    X, _ = w.points()
    flips = teacher_forced(kkm, X, w.kernel, w.gamma, w.coef0, w.degree, w.k, w.labels0(),
                           w.max_iter, what="rings")
    assert flips <= 2


def test_packed_mnist_like_prefix(kkm):
    w = datagen.WORKLOADS["mnist_like"]
    X, _ = w.points(rows=2500)
    teacher_forced(kkm, X, w.kernel, w.gamma, w.coef0, w.degree, w.k, w.labels0(rows=2500), 6,
                   what="mnist_like[:2500]")


@pytest.mark.parametrize("store", ["f32", "bf16"])
def test_packed_gmm_prefix(kkm, store):
    w = datagen.WORKLOADS["gmm200k"]
    X, _ = w.points(rows=4500)
    teacher_forced(kkm, X, w.kernel, w.gamma, w.coef0, w.degree, w.k, w.labels0(rows=4500), 4,
                   store=store, what="gmm200k[:4500] %s" % store)


# one to five strips, ragged n, k from 1 to the packed form's limit
@pytest.mark.parametrize("n,d,k", [(1, 2, 1), (65, 4, 7), (1025, 5, 3), (2049, 7, 33),
                                   (3000, 6, 1), (4099, 9, 128), (5000, 3, 64)])
@pytest.mark.parametrize("store", ["f32", "bf16"])
def test_packed_shapes(kkm, n, d, k, store):
    rng = np.random.default_rng(3000 + n + d)
    X = rng.normal(0, 1, (n, d)).astype(np.float32)
    teacher_forced(kkm, X, kkm.GAUSS, 1.0 / d, 0.0, 1, k, rng.integers(0, k, n).astype(np.int32),
                   4, store=store, what="n=%d d=%d k=%d %s" % (n, d, k, store))


def test_packed_empty_clusters_and_poly(kkm):
    rng = np.random.default_rng(15)
    X = rng.normal(0, 1, (2300, 5)).astype(np.float32)
    lab = rng.integers(0, 3, 2300).astype(np.int32)
    lab[:50] = 4
    for pol in (0, 1):
        teacher_forced(kkm, X, kkm.POLY, 0.2, 1.0, 2, 6, lab, 4, empty_policy=pol,
                       what="empty policy %d" % pol)


def test_packed_fit_matches_dense_and_oracle(kkm):
    """Whole runs from the same labels: where no near-tie occurs on the
    oracle's trajectory, the packed run, the dense run and the oracle's run
    end with the same labels after the same number of steps; the objectives
    agree to the FP32 bar.  The same for bfloat16 storage against the oracle
    run on the stored bfloat16 values."""
    import torch
    w = datagen.WORKLOADS["gmm200k"]
    n = 3000
    X, _ = w.points(rows=n)
    l0 = w.labels0(rows=n)
    Xd = to_dev(X)
    for store in ("f32", "bf16"):
        ks = kkm.F32 if store == "f32" else kkm.BF16
        if store == "f32":
            K_or = oracle.kernel_matrix(X, w.kernel, w.gamma)
        else:
            Kd, _ = kkm.kkm_gram(Xd, w.kernel, w.gamma, gram_prec=ks, k_store=ks)
            torch.cuda.synchronize()
            K_or = Kd.float().cpu().numpy().astype(np.float64)
            del Kd
        ref = oracle.fit(K_or, w.k, l0, 50)
        say("fit packed", store)
        r = kkm.kkm_fit_packed(Xd, w.k, to_dev(l0), w.kernel, w.gamma, gram_prec=ks, k_store=ks,
                               max_iter=50)
        s = kkm.kkm_fit_ex(Xd, w.k, to_dev(l0), w.kernel, w.gamma, gram_prec=ks, k_store=ks,
                           max_iter=50)
        torch.cuda.synchronize()
        recs = oracle.trajectory(K_or, w.k, l0, 50)
        tie = any((st["gap"] < 1e-6 * 4).any() for _, st in recs)
        say("  iterations: packed %d dense %d oracle %d (near-tie on the way: %s)" % (
            r["iters"], s["iters"], ref["iters"], tie))
        if not tie:
            np.testing.assert_array_equal(r["labels"].cpu().numpy(), ref["labels"])
            np.testing.assert_array_equal(s["labels"].cpu().numpy(), ref["labels"])
            assert r["iters"] == ref["iters"] == s["iters"]
        scale = np.abs(np.diag(K_or)).sum()
        assert abs(r["objective"] - ref["objective"]) <= 2e-5 * scale
        np.testing.assert_allclose(r["J_trace"][:len(ref["J_trace"])], ref["J_trace"][:len(r["J_trace"])],
                                   rtol=0, atol=2e-5 * scale)


def test_packed_is_deterministic_and_errors(kkm):
    import torch
    w = datagen.WORKLOADS["gmm200k"]
    n = 5000
    X, _ = w.points(rows=n)
    Xd = to_dev(X)
    l0 = to_dev(w.labels0(rows=n))
    Kp, dg = kkm.kkm_gram_packed(Xd, w.kernel, w.gamma)
    a = kkm.kkm_iterate_packed(Kp, dg, l0, w.k, D_out=True, ctilde_out=True)
    b = kkm.kkm_iterate_packed(Kp, dg, l0, w.k, D_out=True, ctilde_out=True)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    with pytest.raises(kkm.KKMError) as e:
        kkm.kkm_iterate_packed(Kp, dg, to_dev(np.zeros(n, np.int32)), 129)
    assert e.value.status == -5
    bad = w.labels0(rows=n).copy()
    bad[7] = 99
    with pytest.raises(kkm.KKMError) as e:
        kkm.kkm_fit_packed(Xd, w.k, to_dev(bad), w.kernel, w.gamma, max_iter=3)
    assert e.value.status == -2
    r0 = kkm.kkm_fit_packed(Xd, w.k, l0, w.kernel, w.gamma, max_iter=0)
    assert r0["iters"] == 0


def test_packed_gmm200k_full_size(kkm):
    """n = 200000, d = 1024, k = 64, FP32 packed (81 GB): one step from the
    random labels; E recovered at sampled rows (and the last rows) against the
    oracle's cluster sums from the points; on every row the properties that
    hold at any size."""
    import torch
    w = datagen.WORKLOADS["gmm200k"]
    X, _ = w.points()
    l0 = w.labels0()
    n = w.n
    say("packed full size", n, w.d, w.k)
    Kp, dg = kkm.kkm_gram_packed(to_dev(X), w.kernel, w.gamma)
    lab, cnt, ch, J_in, D, C = kkm.kkm_iterate_packed(Kp, dg, to_dev(l0), w.k, D_out=True,
                                                      ctilde_out=True)
    torch.cuda.synchronize()
    del Kp
    torch.cuda.empty_cache()
    D = D.cpu().numpy().astype(np.float64)
    C = C.cpu().numpy().astype(np.float64)
    dgl = dg.cpu().numpy().astype(np.float64)
    lab = lab.cpu().numpy()
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
    rng = np.random.default_rng(91)
    R = np.unique(np.concatenate([rng.integers(0, n, 48), np.arange(n - 8, n), np.arange(8)]))
    S_or = oracle.cluster_row_sums(X, l0, w.k, R, w.kernel, w.gamma)
    E_or = np.where(live[None, :], S_or / np.maximum(counts_in, 1)[None, :], 0.0)
    sig = np.abs(dgl[R]) + (2 * np.abs(E_or[:, live]) + np.abs(C[live])[None, :]).max(axis=1)
    err = (np.abs(E[R][:, live] - E_or[:, live]) / sig[:, None]).max()
    say("  E error %.3g sigma" % err)
    assert err <= D_TOL, "E error %.3g sigma" % err
