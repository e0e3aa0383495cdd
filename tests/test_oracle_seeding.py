"""Pins of the kernel-space k-means++ reference (no GPU)."""
import numpy as np

import oracle
from oracle import mlp, seeding


def test_linear_kernel_is_feature_space_kmeanspp():
    """With kappa(x, y) = x.y the kernel distances K_ii + K_ss - 2K_is are the
    squared Euclidean distances, so the seeding must equal k-means++ on the
    points themselves (computed there from direct differences)."""
    rng = np.random.default_rng(7)
    compared = 0
    for n, d, k in ((40, 3, 5), (200, 8, 12), (7, 2, 7)):
        X = rng.normal(0, 1, (n, d))
        u = rng.random(k)
        s1, l1, _ = seeding.kernel_kmeanspp(X @ X.T, k, u)
        s2, l2, m2 = mlp.kmeanspp(X, k, u)
        close = m2 < 1e-12
        if not close.any():
            np.testing.assert_array_equal(s1, s2)
            np.testing.assert_array_equal(l1, l2)
            compared += 1
    assert compared == 3


def test_hand_computed_draws():
    """Points 0, 1, 3 on a line, linear kernel.  Seed 0 = row floor(0 * 3) = 0;
    squared distances to it 0, 1, 9 (running sums 0, 1, 10): u = 0.05 puts the
    target at 0.5 -> row 1; u = 0.15 puts it at 1.5 -> row 2."""
    X = np.array([[0.0], [1.0], [3.0]])
    K = X @ X.T
    s, lab, _ = seeding.kernel_kmeanspp(K, 2, [0.0, 0.05])
    assert list(s) == [0, 1] and list(lab) == [0, 1, 1]
    s, lab, _ = seeding.kernel_kmeanspp(K, 2, [0.0, 0.15])
    assert list(s) == [0, 2] and list(lab) == [0, 0, 1]
    # a third seed: distances to the nearest of {0, 2} are 0, 1, 0 -> row 1
    s, lab, _ = seeding.kernel_kmeanspp(K, 3, [0.0, 0.15, 0.7])
    assert list(s) == [0, 2, 1] and list(lab) == [0, 2, 1]


def test_gaussian_seeds_distinct_and_labels_nearest():
    """Gaussian kernel: distinct points give distinct seeds (a chosen seed has
    dmin 0 and is never drawn again), every seed labels itself, and each label
    is the seed of smallest kernel distance."""
    rng = np.random.default_rng(3)
    X = rng.normal(0, 1, (150, 4)).astype(np.float32)
    K = oracle.kernel_matrix(X, oracle.GAUSS, 0.5)
    s, lab, _ = seeding.kernel_kmeanspp(K, 10, rng.random(10))
    assert len(set(s.tolist())) == 10
    np.testing.assert_array_equal(lab[s], np.arange(10))
    Kd = np.asarray(K, np.float64)
    D = np.diag(Kd)[:, None] + np.diag(Kd)[s][None, :] - 2.0 * Kd[:, s]
    assert np.all(D[np.arange(150), lab] <= D.min(axis=1) + 1e-12)
