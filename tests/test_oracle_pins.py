"""Pins for the FP64 oracle: checks against facts fixed by the paper and by
mathematics, independent of the oracle's own code.

* hand-worked examples (tests/golden/hand_examples.json);
* linear kernel == classical Lloyd with explicit centroids (Sec. 2.1), and ==
  scikit-learn's Lloyd (a library routine);
* degree-2 polynomial kernel == Lloyd on the explicit feature expansion
  phi(x) = (c, sqrt(2 c gamma) x, gamma vec(x x^T)) (Sec. 3.2 with Eq. mtx_dist);
* centroid norms == diag(V K V^T) with a dense V (Eq. c_norm);
* objective never increases: J_{t+1} <= A_t <= J_t;
* brute force over all partitions for n <= 10: the optimum is a fixed point and
  no run ends below it;
* special cases: k=1, singletons, a well-separated truth partition, empty
  clusters, the Gaussian diagonal, symmetry and positive semi-definiteness.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import datagen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_examples.json")
KCODE = {"linear": oracle.LINEAR, "poly": oracle.POLY, "gauss": oracle.GAUSS}


def blobs(n, d, k, sep, seed):
    rng = np.random.default_rng(seed)
    mu = rng.normal(0, sep, (k, d))
    lab = rng.integers(0, k, n)
    X = (mu[lab] + rng.normal(0, 1, (n, d))).astype(np.float32)
    return X, lab.astype(np.int32)


def explicit_lloyd_step(F, k, labels):
    """Lloyd phases 1-3 with explicit centroids in the feature space of F (rows).

    Returns (labels_out, D) with D_ic = ||F_i - mean_{j in c} F_j||^2 (+inf if empty)."""
    F = F.astype(np.float64)
    n = F.shape[0]
    D = np.full((n, k), np.inf)
    for c in range(k):
        m = labels == c
        if m.any():
            mu = F[m].mean(axis=0)
            D[:, c] = ((F - mu) ** 2).sum(axis=1)
    return np.argmin(D, axis=1).astype(np.int32), D


# ---------------------------------------------------------------- golden


@pytest.mark.parametrize("ex", json.load(open(GOLDEN))["examples"], ids=lambda e: e["name"])
def test_hand_worked_examples(ex):
    X = np.array(ex["points"], dtype=np.float32)
    K = oracle.kernel_matrix(X, KCODE[ex["kernel"]], ex["gamma"], ex["coef0"], ex["degree"])
    if "K" in ex:
        np.testing.assert_allclose(K, np.array(ex["K"]), rtol=1e-12, atol=1e-15)
    labels = np.array(ex["labels0"], dtype=np.int32)
    for st in ex["steps"]:
        r = oracle.step(K, ex["k"], labels)
        np.testing.assert_allclose(r["D"], np.array(st["D"], dtype=np.float64), rtol=1e-12, atol=1e-12)
        assert r["labels"].tolist() == st["labels_out"]
        assert r["J_in"] == pytest.approx(st["J_in"], rel=1e-12, abs=1e-12)
        assert r["A"] == pytest.approx(st["A"], rel=1e-12, abs=1e-12)
        assert r["n_changed"] == st["n_changed"]
        labels = r["labels"]


# ---------------------------------------------------------------- kernel values


def test_gaussian_closed_form_values():
    # ||x - y||^2 = 25 for (0,0),(3,4); gamma = 1/25 gives exp(-1)
    x = np.array([0.0, 0.0], np.float32)
    y = np.array([3.0, 4.0], np.float32)
    assert oracle.kappa(x, y, oracle.GAUSS, 1.0 / 25.0) == pytest.approx(math.exp(-1.0), rel=1e-14)
    assert oracle.kappa(x, x, oracle.GAUSS, 0.7) == 1.0
    # polynomial (x.y + 1)^2 at x.y = 11 (1*3 + 2*4) is 144
    a = np.array([1.0, 2.0], np.float32)
    b = np.array([3.0, 4.0], np.float32)
    assert oracle.kappa(a, b, oracle.POLY, 1.0, 1.0, 2) == 144.0
    assert oracle.kappa(a, b, oracle.POLY, 0.5, 2.0, 3) == (0.5 * 11 + 2.0) ** 3
    assert oracle.kappa(a, b, oracle.LINEAR) == 11.0


def test_linear_kernel_matrix_is_gram_product():
    X, _ = blobs(60, 7, 3, 2.0, 1)
    K = oracle.kernel_matrix(X, oracle.LINEAR)
    Xd = X.astype(np.float64)
    np.testing.assert_allclose(K, Xd @ Xd.T, rtol=1e-12, atol=1e-12)


def test_gaussian_matrix_matches_norm_expansion():
    # Eq. (gauss): exp(-gamma (B_ii + B_jj - 2 B_ij)) with B = P P^T (a different route)
    X, _ = blobs(50, 5, 3, 1.0, 2)
    g = 0.3
    K = oracle.kernel_matrix(X, oracle.GAUSS, g)
    Xd = X.astype(np.float64)
    B = Xd @ Xd.T
    nb = np.diag(B)
    ref = np.exp(-g * np.maximum(nb[:, None] + nb[None, :] - 2 * B, 0.0))
    np.testing.assert_allclose(K, ref, rtol=1e-10, atol=1e-13)
    assert np.all(np.diag(K) == 1.0)


@pytest.mark.parametrize("kern,g,c,r", [(oracle.GAUSS, 0.5, 0.0, 1), (oracle.POLY, 1.0, 1.0, 2),
                                        (oracle.LINEAR, 1.0, 0.0, 1)])
def test_kernel_matrix_symmetric_psd(kern, g, c, r):
    X, _ = blobs(120, 4, 3, 1.5, 3)
    K = oracle.kernel_matrix(X, kern, g, c, r)
    assert np.array_equal(K, K.T)
    ev = np.linalg.eigvalsh(K)
    assert ev.min() >= -1e-12 * np.abs(K).max() * K.shape[0]


def test_kernel_rows_and_cluster_row_sums_agree_with_matrix():
    X, _ = blobs(90, 6, 4, 1.0, 4)
    lab = np.random.default_rng(5).integers(0, 4, 90).astype(np.int32)
    K = oracle.kernel_matrix(X, oracle.GAUSS, 0.2)
    rows = np.array([0, 17, 89])
    np.testing.assert_array_equal(oracle.kernel_rows(X, rows, oracle.GAUSS, 0.2), K[rows])
    S = oracle.cluster_row_sums(X, lab, 4, rows, oracle.GAUSS, 0.2)
    for a, r in enumerate(rows):
        for c in range(4):
            assert S[a, c] == pytest.approx(K[r, lab == c].sum(), rel=1e-13)


# ---------------------------------------------------------------- distance identity


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_linear_kernel_is_classical_lloyd(seed):
    X, _ = blobs(240, 3, 5, 3.0, 10 + seed)
    k = 5
    K = oracle.kernel_matrix(X, oracle.LINEAR)
    labels = datagen.uniform_labels(240, k, 100 + seed)
    for _ in range(15):
        r = oracle.step(K, k, labels)
        ref_lab, ref_D = explicit_lloyd_step(X, k, labels)
        scale = np.abs(ref_D[np.isfinite(ref_D)]).max()
        fin = np.isfinite(ref_D)
        np.testing.assert_array_equal(np.isfinite(r["D"]), fin)
        np.testing.assert_allclose(r["D"][fin], ref_D[fin], rtol=0, atol=1e-10 * scale)
        clear = r["gap"] > 1e-9 * scale
        np.testing.assert_array_equal(r["labels"][clear], ref_lab[clear])
        J_ref = ref_D[np.arange(240), labels].sum()
        assert r["J_in"] == pytest.approx(J_ref, rel=1e-12)
        if r["n_changed"] == 0:
            break
        labels = r["labels"]


def test_linear_kernel_matches_sklearn_lloyd():
    sk = pytest.importorskip("sklearn.cluster")
    X, _ = blobs(300, 4, 4, 4.0, 21)
    k = 4
    labels0 = datagen.uniform_labels(300, k, 22)
    Xd = X.astype(np.float64)
    init = np.stack([Xd[labels0 == c].mean(axis=0) for c in range(k)])
    K = oracle.kernel_matrix(X, oracle.LINEAR)
    res = oracle.fit(K, k, labels0, 100)
    assert np.all(np.bincount(res["labels"], minlength=k) > 0)  # sklearn relocates empties
    km = sk.KMeans(n_clusters=k, init=init, n_init=1, max_iter=100, tol=0.0,
                   algorithm="lloyd").fit(Xd)
    np.testing.assert_array_equal(km.labels_, res["labels"])
    assert res["objective"] == pytest.approx(km.inertia_, rel=1e-9)


@pytest.mark.parametrize("gamma,coef0", [(1.0, 1.0), (0.5, 2.0)])
def test_poly2_kernel_equals_explicit_features(gamma, coef0):
    # (gamma x.y + c)^2 = <phi(x), phi(y)> with phi(x) = (c, sqrt(2 c gamma) x, gamma vec(x x^T))
    X, _ = blobs(150, 3, 4, 1.0, 31)
    X = (X / 3.0).astype(np.float32)
    n, d = X.shape
    Xd = X.astype(np.float64)
    F = np.concatenate([np.full((n, 1), coef0), math.sqrt(2 * coef0 * gamma) * Xd,
                        gamma * np.einsum("ni,nj->nij", Xd, Xd).reshape(n, d * d)], axis=1)
    K = oracle.kernel_matrix(X, oracle.POLY, gamma, coef0, 2)
    np.testing.assert_allclose(K, F @ F.T, rtol=1e-12, atol=1e-12)
    k = 4
    labels = datagen.uniform_labels(n, k, 32)
    for _ in range(12):
        r = oracle.step(K, k, labels)
        ref_lab, ref_D = explicit_lloyd_step(F, k, labels)
        scale = np.abs(ref_D[np.isfinite(ref_D)]).max()
        fin = np.isfinite(ref_D)
        np.testing.assert_allclose(r["D"][fin], ref_D[fin], rtol=0, atol=1e-10 * scale)
        clear = r["gap"] > 1e-9 * scale
        np.testing.assert_array_equal(r["labels"][clear], ref_lab[clear])
        if r["n_changed"] == 0:
            break
        labels = r["labels"]


def test_centroid_norms_equal_diag_VKVt():
    # Eq. (c_norm): ||c_j||^2 = (V K V^T)_jj with V_ji = 1/|L_j| (Eq. v_init)
    X, _ = blobs(130, 5, 6, 1.0, 41)
    k = 6
    K = oracle.kernel_matrix(X, oracle.GAUSS, 0.1)
    labels = datagen.uniform_labels(130, k, 42)
    V = np.zeros((k, 130))
    for c in range(k):
        m = labels == c
        V[c, m] = 1.0 / m.sum()
    r = oracle.step(K, k, labels)
    KVt = K @ V.T  # E_ic = (1/|c|) sum_{j in c} K_ij
    cn = r["D"] - np.diag(K)[:, None] + 2.0 * KVt  # what remains is the centroid norm, every row
    ref = np.diag(V @ K @ V.T)
    np.testing.assert_allclose(cn, np.broadcast_to(ref, cn.shape), rtol=1e-11, atol=1e-12)
    # J = sum_i K_ii - sum_c |c| ||c_c||^2
    cnt = np.bincount(labels, minlength=k)
    assert r["J_in"] == pytest.approx(np.trace(K) - (cnt * ref).sum(), rel=1e-11)


# ---------------------------------------------------------------- loop properties


@pytest.mark.parametrize("kern,g,c,r,seed", [(oracle.GAUSS, 1.0, 0.0, 1, 0),
                                             (oracle.POLY, 1.0, 1.0, 2, 1),
                                             (oracle.LINEAR, 1.0, 0.0, 1, 2),
                                             (oracle.GAUSS, 0.05, 0.0, 1, 3)])
def test_objective_non_increasing(kern, g, c, r, seed):
    X, _ = blobs(200, 4, 6, 1.5, 50 + seed)
    k = 6
    K = oracle.kernel_matrix(X, kern, g, c, r)
    labels = datagen.uniform_labels(200, k, 60 + seed)
    slack = 1e-12
    prev_A = None
    for _ in range(40):
        st = oracle.step(K, k, labels)
        J, A = st["J_in"], st["A"]
        assert A <= J + slack * abs(J)
        if prev_A is not None:
            assert J <= prev_A + slack * abs(prev_A)
        prev_A = A
        if st["n_changed"] == 0:
            break
        labels = st["labels"]


def test_fit_traces_consistent():
    X, _ = blobs(150, 3, 4, 2.0, 70)
    K = oracle.kernel_matrix(X, oracle.GAUSS, 0.3)
    l0 = datagen.uniform_labels(150, 4, 71)
    res = oracle.fit(K, 4, l0, 50)
    assert res["changed_trace"][-1] == 0
    assert res["objective"] == pytest.approx(oracle.objective(K, 4, res["labels"]), rel=1e-14)
    assert res["J_trace"][-1] == res["objective"]
    assert np.all(np.diff(res["J_trace"]) <= 1e-12 * abs(res["J_trace"][0]))
    # fixed iteration count without the convergence check
    res2 = oracle.fit(K, 4, l0, 7, check_convergence=False)
    assert res2["iters"] == 7
    res0 = oracle.fit(K, 4, l0, 0)
    assert res0["iters"] == 0 and np.array_equal(res0["labels"], l0)
    assert res0["objective"] == pytest.approx(oracle.objective(K, 4, l0), rel=1e-14)


def _partitions(n, kmax):
    """All set partitions of range(n) into at most kmax blocks (restricted growth strings)."""
    def rec(i, labels, m):
        if i == n:
            yield list(labels)
            return
        for c in range(min(m + 1, kmax)):
            labels.append(c)
            yield from rec(i + 1, labels, max(m, c + 1))
            labels.pop()
    yield from rec(0, [], 0)


def _scatter_objective(K, labels):
    """Within-cluster scatter in feature space written with K only:
    sum_c [ sum_{i in c} K_ii - (1/|c|) sum_{i,j in c} K_ij ]."""
    total = 0.0
    for c in set(labels):
        idx = [i for i, l in enumerate(labels) if l == c]
        sub = K[np.ix_(idx, idx)]
        total += np.trace(sub) - sub.sum() / len(idx)
    return total


@pytest.mark.parametrize("n,k,seed", [(9, 3, 0), (10, 3, 1), (8, 4, 2)])
def test_bruteforce_optimum(n, k, seed):
    rng = np.random.default_rng(80 + seed)
    mu = rng.normal(0, 4, (k, 2))
    X = (mu[rng.integers(0, k, n)] + rng.normal(0, 0.5, (n, 2))).astype(np.float32)
    K = oracle.kernel_matrix(X, oracle.GAUSS, 0.2)
    best, best_lab = math.inf, None
    count = 0
    for lab in _partitions(n, k):
        count += 1
        J = _scatter_objective(K, lab)
        if J < best:
            best, best_lab = J, lab
    assert count == sum(_stirling2(n, j) for j in range(1, k + 1))
    best_lab = np.array(best_lab, dtype=np.int32)
    kk = int(best_lab.max()) + 1
    st = oracle.step(K, kk, best_lab)
    assert st["n_changed"] == 0  # the global optimum is a fixed point
    assert st["J_in"] == pytest.approx(best, rel=1e-12)
    reached = math.inf
    for s in range(50):
        res = oracle.fit(K, k, datagen.uniform_labels(n, k, 1000 + s), 100)
        assert res["objective"] >= best - 1e-12 * abs(best)
        reached = min(reached, res["objective"])
    assert reached == pytest.approx(best, rel=1e-12)


def _stirling2(n, j):
    return sum((-1) ** i * math.comb(j, i) * (j - i) ** n for i in range(j + 1)) // math.factorial(j)


# ---------------------------------------------------------------- special cases


def test_single_cluster_closed_form():
    X, _ = blobs(77, 3, 2, 1.0, 90)
    K = oracle.kernel_matrix(X, oracle.GAUSS, 0.4)
    st = oracle.step(K, 1, np.zeros(77, np.int32))
    assert st["n_changed"] == 0
    assert st["J_in"] == pytest.approx(np.trace(K) - K.sum() / 77, rel=1e-12)


def test_singletons_have_zero_objective():
    X, _ = blobs(12, 3, 3, 1.0, 91)
    K = oracle.kernel_matrix(X, oracle.POLY, 1.0, 1.0, 2)
    lab = np.arange(12, dtype=np.int32)
    st = oracle.step(K, 12, lab)
    assert st["n_changed"] == 0
    assert abs(st["J_in"]) <= 1e-12 * np.abs(K).max()
    assert np.all(np.abs(st["D"][np.arange(12), lab]) <= 1e-12 * np.abs(K).max())


def test_truth_partition_of_separated_mixture_is_fixed_point():
    X, truth = datagen.gmm(2000, 32, 8, 0.3, seed=92)
    K = oracle.kernel_matrix(X, oracle.GAUSS, 1.0 / 32)
    st = oracle.step(K, 8, truth)
    assert st["n_changed"] == 0


def test_empty_cluster_policies():
    X, _ = blobs(40, 2, 2, 3.0, 93)
    K = oracle.kernel_matrix(X, oracle.GAUSS, 0.5)
    lab = np.random.default_rng(94).integers(0, 2, 40).astype(np.int32)  # cluster 2 empty
    a = oracle.step(K, 3, lab, empty_policy=oracle.EMPTY_INF)
    assert np.all(np.isinf(a["D"][:, 2])) and a["counts"][2] == 0
    b = oracle.step(K, 3, lab, empty_policy=oracle.EMPTY_ZERO_CENTROID)
    np.testing.assert_array_equal(b["D"][:, 2], np.diag(K))
    np.testing.assert_array_equal(a["D"][:, :2], b["D"][:, :2])
    with pytest.raises(ValueError):
        oracle.step(K, 2, np.full(40, 2, np.int32))


def test_adjusted_rand_index_matches_sklearn():
    skm = pytest.importorskip("sklearn.metrics")
    rng = np.random.default_rng(95)
    for _ in range(20):
        n = int(rng.integers(2, 400))
        a = rng.integers(0, int(rng.integers(1, 9)), n)
        b = np.where(rng.random(n) < 0.7, a, rng.integers(0, 6, n))
        assert oracle.adjusted_rand_index(a, b) == pytest.approx(skm.adjusted_rand_score(a, b), abs=1e-12)
    assert oracle.adjusted_rand_index([0, 0, 1, 1], [5, 5, 3, 3]) == 1.0
