"""HIP path vs the FP64 oracle on the GPU, through the C ABI.

Teacher-forced: at every step the oracle's labels of that step are fed to
kkm_iterate, and its distances, labels, sizes, changed count and objective are
compared with the oracle's step (rules in tests/parity.py).  Sizes span
several 128-row Gram tiles, several 1024-column sweep strips and ragged tails.
"""
import sys

import numpy as np
import pytest

import datagen
import oracle

from parity import compare_step, gram_bound

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


def gram_case(kkm, X, kernel, gamma, coef0, degree, what, shape=0):
    import torch
    say("gram", what, X.shape, kernel, "shape", shape)
    Xd = to_dev(X)
    K, diag = kkm.kkm_gram(Xd, kernel, gamma, coef0, degree, shape=shape)
    torch.cuda.synchronize()
    Kg = K.cpu().numpy().astype(np.float64)
    dg = diag.cpu().numpy()
    K_or = oracle.kernel_matrix(X, kernel, gamma, coef0, degree)
    assert np.array_equal(Kg, Kg.T), what + ": K not exactly symmetric"
    np.testing.assert_array_equal(dg, np.diag(Kg).astype(np.float32))
    bound = gram_bound(X, kernel, gamma, coef0, degree, K_or)
    ratio = np.abs(Kg - K_or) / bound
    assert ratio.max() <= 1.0, "%s: K error %.3g of the FP32 bound at %s" % (
        what, ratio.max(), np.unravel_index(ratio.argmax(), ratio.shape))
    if kernel == kkm.GAUSS:
        assert np.all(dg == 1.0)
    return K, diag, K_or


def run_teacher_forced(kkm, K, diag, K_or, k, labels0, steps, empty_policy=0, what=""):
    import torch
    cur = np.ascontiguousarray(labels0, dtype=np.int32)
    flips = 0
    for t in range(steps):
        orc = oracle.step(K_or, k, cur, empty_policy)
        say("  step", t, what)
        lab, cnt, ch, J, D, C = kkm.kkm_iterate(K, diag, to_dev(cur), k, empty_policy,
                                                D_out=True, ctilde_out=True)
        torch.cuda.synchronize()
        flips += compare_step(K_or, k, cur, orc, D.cpu().numpy(), lab.cpu().numpy(),
                              cnt.cpu().numpy(), int(ch.item()), float(J.item()),
                              C.cpu().numpy(), what="%s step %d" % (what, t))
        if orc["n_changed"] == 0:
            break
        cur = orc["labels"]
    return flips


@pytest.mark.parametrize("n,d", [(1, 1), (7, 3), (63, 5), (65, 16), (129, 33), (300, 2),
                                 (1000, 16), (1100, 64)])
@pytest.mark.parametrize("kernel", ["linear", "poly", "gauss"])
@pytest.mark.parametrize("tiles", ["triangle", "full"])
def test_gram_parity_shapes(kkm, n, d, kernel, tiles):
    """Both tile shapes of the product (the SYRK triangle with mirrored stores,
    and the GEMM square where every tile stores its own block) against the
    oracle's K from the definition."""
    rng = np.random.default_rng(n * 131 + d)
    X = rng.normal(0, 1, (n, d)).astype(np.float32)
    code = {"linear": kkm.LINEAR, "poly": kkm.POLY, "gauss": kkm.GAUSS}[kernel]
    gamma = 1.0 / d if kernel != "linear" else 1.0
    shape = kkm.GRAM_TRIANGLE if tiles == "triangle" else kkm.GRAM_FULL
    gram_case(kkm, X, code, gamma, 1.0 if kernel == "poly" else 0.0, 2 if kernel == "poly" else 1,
              "n=%d d=%d %s" % (n, d, kernel), shape=shape)


def test_gram_parity_strided_rows(kkm):
    import torch
    rng = np.random.default_rng(7)
    base = rng.normal(0, 1, (301, 23)).astype(np.float32)
    Xd = to_dev(base)[:, 2:19]  # ldx=23, d=17, unaligned rows
    X = base[:, 2:19].copy()
    K, diag = kkm.kkm_gram(Xd, kkm.GAUSS, 0.1)
    torch.cuda.synchronize()
    K_or = oracle.kernel_matrix(X, oracle.GAUSS, 0.1)
    r = np.abs(K.cpu().numpy() - K_or) / gram_bound(X, 2, 0.1, 0, 1, K_or)
    assert r.max() <= 1.0


def test_rings_teacher_forced(kkm):
    w = datagen.WORKLOADS["rings"]
    X, _ = w.points()
    K, diag, K_or = gram_case(kkm, X, w.kernel, w.gamma, w.coef0, w.degree, "rings")
    flips = run_teacher_forced(kkm, K, diag, K_or, w.k, w.labels0(), w.max_iter, what="rings")
    assert flips <= 2


def test_mnist_like_subsample_teacher_forced(kkm):
    w = datagen.WORKLOADS["mnist_like"]
    X, _ = w.points(rows=2500)
    K, diag, K_or = gram_case(kkm, X, w.kernel, w.gamma, w.coef0, w.degree, "mnist_like[:2500]")
    run_teacher_forced(kkm, K, diag, K_or, w.k, w.labels0(rows=2500), 8, what="mnist_like")


def test_gmm_subsample_teacher_forced(kkm):
    w = datagen.WORKLOADS["gmm200k"]
    X, _ = w.points(rows=3000)
    K, diag, K_or = gram_case(kkm, X, w.kernel, w.gamma, w.coef0, w.degree, "gmm200k[:3000]")
    run_teacher_forced(kkm, K, diag, K_or, w.k, w.labels0(rows=3000), 6, what="gmm")


@pytest.mark.parametrize("n,d,k", [(1, 2, 1), (7, 3, 2), (65, 4, 7), (1025, 5, 3), (2049, 8, 33),
                                   (3000, 6, 1)])
def test_tail_shapes_teacher_forced(kkm, n, d, k):
    rng = np.random.default_rng(1000 + n)
    X = rng.normal(0, 1, (n, d)).astype(np.float32)
    K, diag, K_or = gram_case(kkm, X, kkm.GAUSS, 0.5, 0, 1, "tail n=%d" % n)
    run_teacher_forced(kkm, K, diag, K_or, k, rng.integers(0, k, n).astype(np.int32), 6,
                       what="tail n=%d k=%d" % (n, k))


def test_singletons_and_empty_clusters(kkm):
    import torch
    rng = np.random.default_rng(5)
    X = rng.normal(0, 1, (40, 3)).astype(np.float32)
    K, diag, K_or = gram_case(kkm, X, kkm.POLY, 1.0, 1.0, 2, "singletons")
    # k = n, one point per cluster
    run_teacher_forced(kkm, K, diag, K_or, 40, np.arange(40, dtype=np.int32), 1, what="k=n")
    # clusters 3 and 5 empty, both policies
    lab = rng.integers(0, 3, 40).astype(np.int32)
    lab[:5] = 4
    for pol in (0, 1):
        run_teacher_forced(kkm, K, diag, K_or, 6, lab, 4, empty_policy=pol,
                           what="empty policy %d" % pol)


def test_iterate_is_deterministic(kkm):
    import torch
    w = datagen.WORKLOADS["gmm200k"]
    X, _ = w.points(rows=5000)
    K, diag = kkm.kkm_gram(to_dev(X), w.kernel, w.gamma)
    l0 = to_dev(w.labels0(rows=5000))
    a = kkm.kkm_iterate(K, diag, l0, w.k, D_out=True, ctilde_out=True)
    b = kkm.kkm_iterate(K, diag, l0, w.k, D_out=True, ctilde_out=True)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_fit_matches_oracle_run(kkm):
    import torch
    w = datagen.WORKLOADS["rings"]
    X, _ = w.points()
    l0 = w.labels0()
    K_or = oracle.kernel_matrix(X, w.kernel, w.gamma, w.coef0, w.degree)
    ref = oracle.fit(K_or, w.k, l0, w.max_iter)
    say("fit rings")
    r = kkm.kkm_fit_ex(to_dev(X), w.k, to_dev(l0), w.kernel, w.gamma, w.coef0, w.degree,
                       max_iter=w.max_iter, check_convergence=True)
    torch.cuda.synchronize()
    # whole-run equality holds when no near-tie occurred on the trajectory
    recs = oracle.trajectory(K_or, w.k, l0, w.max_iter)
    tie = any((st["gap"] < 1e-6 * 4).any() for _, st in recs)
    if not tie:
        np.testing.assert_array_equal(r["labels"].cpu().numpy(), ref["labels"])
        assert r["iters"] == ref["iters"]
    scale = np.abs(np.diag(K_or)).sum()
    assert abs(r["objective"] - ref["objective"]) <= 1e-5 * scale * 2
    np.testing.assert_allclose(r["J_trace"], ref["J_trace"], rtol=0, atol=2e-5 * scale)


def test_fit_fixed_iterations_and_zero(kkm):
    import torch
    rng = np.random.default_rng(9)
    X = rng.normal(0, 1, (500, 4)).astype(np.float32)
    l0 = rng.integers(0, 5, 500).astype(np.int32)
    K_or = oracle.kernel_matrix(X, oracle.GAUSS, 0.3)
    r = kkm.kkm_fit_ex(to_dev(X), 5, to_dev(l0), kkm.GAUSS, 0.3, max_iter=7,
                       check_convergence=False)
    assert r["iters"] == 7
    ref = oracle.fit(K_or, 5, l0, 7, check_convergence=False)
    assert abs(r["objective"] - ref["objective"]) <= 2e-5 * 500
    r0 = kkm.kkm_fit_ex(to_dev(X), 5, to_dev(l0), kkm.GAUSS, 0.3, max_iter=0)
    assert r0["iters"] == 0
    np.testing.assert_array_equal(r0["labels"].cpu().numpy(), l0)
    assert abs(r0["objective"] - oracle.objective(K_or, 5, l0)) <= 2e-5 * 500


def test_error_paths(kkm):
    import torch
    rng = np.random.default_rng(11)
    X = rng.normal(0, 1, (300, 4)).astype(np.float32)
    Xd = to_dev(X)
    bad = rng.integers(0, 3, 300).astype(np.int32)
    bad[17] = 3
    with pytest.raises(kkm.KKMError) as e:
        kkm.kkm_fit(Xd, 3, to_dev(bad), kkm.GAUSS, 0.5, max_iter=5)
    assert e.value.status == -2
    K, diag = kkm.kkm_gram(Xd, kkm.GAUSS, 0.5)
    lab, cnt, ch, J, _, _ = kkm.kkm_iterate(K, diag, to_dev(bad), 3)
    torch.cuda.synchronize()
    assert int(ch.item()) == -1
    Xn = X.copy()
    Xn[5, 2] = np.nan
    with pytest.raises(kkm.KKMError) as e:
        kkm.kkm_fit(to_dev(Xn), 3, to_dev(np.zeros(300, np.int32)), kkm.GAUSS, 0.5, max_iter=2)
    assert e.value.status == -6
    with pytest.raises(kkm.KKMError) as e:
        kkm.kkm_fit(Xd, 0, to_dev(np.zeros(300, np.int32)), kkm.GAUSS, 0.5)
    assert e.value.status == -1


@pytest.mark.parametrize("gp,ks", [(0, 0), (0, 1), (1, 0), (1, 1), (2, 0), (2, 1)])
@pytest.mark.parametrize("n,d", [(1, 3), (129, 33), (700, 100), (1100, 64)])
def test_full_shape_equals_triangle(kkm, gp, ks, n, d):
    """The GEMM shape (every tile) gives bit for bit the K and diag(K) of the
    SYRK shape (upper triangle, mirrored), for every precision pair."""
    import torch
    X = np.random.default_rng(n + d).normal(0, 1, (n, d)).astype(np.float32)
    Xd = to_dev(X)
    for kern, g in ((kkm.GAUSS, 1.0 / d), (kkm.POLY, 0.1)):
        a, da = kkm.kkm_gram(Xd, kern, g, 1.0, 2, gram_prec=gp, k_store=ks)
        b, db = kkm.kkm_gram(Xd, kern, g, 1.0, 2, gram_prec=gp, k_store=ks, shape=kkm.GRAM_FULL)
        torch.cuda.synchronize()
        assert torch.equal(a, b), (gp, ks, kern)
        assert torch.equal(da, db)


@pytest.mark.parametrize("gp,ks", [(1, 0), (1, 1), (2, 0), (2, 1)])
@pytest.mark.parametrize("n,d", [(1, 3), (129, 33), (300, 100), (700, 256), (1100, 64), (2600, 200),
                                 (513, 1030)])
def test_256_tile_equals_128_tile(kkm, gp, ks, n, d):
    """The BF16 / FP8 triangle in 256 x 256 tiles gives bit for bit the K and
    diag(K) of the 128 x 128 tiles (same slabs, same order per entry); n from
    one point to several tiles with ragged edges (2600 = 10 * 256 + 40), d
    from one slab to 17 with a ragged last slab."""
    import torch
    X = np.random.default_rng(7 * n + d).normal(0, 1, (n, d)).astype(np.float32)
    Xd = to_dev(X)
    say("256 tile", n, d, gp, ks)
    for kern, g, c0 in ((kkm.GAUSS, 1.0 / d, 0.0), (kkm.POLY, 0.1, 1.0), (kkm.LINEAR, 1.0, 0.0)):
        a, da = kkm.kkm_gram(Xd, kern, g, c0, 2, gram_prec=gp, k_store=ks, shape=kkm.GRAM_TRIANGLE_128)
        b, db = kkm.kkm_gram(Xd, kern, g, c0, 2, gram_prec=gp, k_store=ks, shape=kkm.GRAM_TRIANGLE_256)
        torch.cuda.synchronize()
        assert torch.equal(a, b), (gp, ks, kern, (a != b).sum().item())
        assert torch.equal(da, db)


def test_gram_shape_values(kkm):
    """An FP32 product ignores the tile-size request (always 128 x 128: same K
    bit for bit); an unknown shape is rejected before any work."""
    import torch
    X = np.random.default_rng(3).normal(0, 1, (300, 40)).astype(np.float32)
    Xd = to_dev(X)
    a, da = kkm.kkm_gram(Xd, kkm.GAUSS, 0.05)
    for shape in (kkm.GRAM_TRIANGLE_128, kkm.GRAM_TRIANGLE_256):
        b, db = kkm.kkm_gram(Xd, kkm.GAUSS, 0.05, shape=shape)
        torch.cuda.synchronize()
        assert torch.equal(a, b) and torch.equal(da, db), shape
    with pytest.raises(kkm.KKMError) as e:
        kkm.kkm_gram(Xd, kkm.GAUSS, 0.05, shape=7)
    assert e.value.status == -1
