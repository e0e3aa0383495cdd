"""Pins for the FP64 reference of the learned feature map: gradients against
central finite differences and against torch autograd in FP64 (a library
routine), the loss and GELU against closed forms, Adam against its first-step
closed form, and feature-space Lloyd against classical K-means."""
import math

import numpy as np
import pytest

import datagen

from oracle import mlp

DIMS = dict(d=6, h1=9, h2=7, out=5)


def small_problem(seed=0, B=8):
    rng = np.random.default_rng(seed)
    theta = datagen.mlp_init_params(**DIMS, seed=seed).astype(np.float64)
    theta += rng.normal(0, 0.05, theta.shape)  # non-zero biases too
    X = rng.normal(0, 1, (B, DIMS["d"]))
    A = rng.normal(0, 1, (B, B))
    K = np.exp(-0.1 * ((X[:, None, :] - X[None, :, :]) ** 2).sum(-1))  # symmetric kernel values
    return theta, X, K + 0 * A


def test_gelu_closed_forms():
    assert mlp.gelu(np.array(0.0)) == 0.0
    assert mlp.gelu(np.array(1.0)) == pytest.approx(0.5 * (1 + math.erf(1 / math.sqrt(2))), rel=1e-15)
    z = np.linspace(-4, 4, 81)
    h = 1e-6
    np.testing.assert_allclose(mlp.gelu_grad(z), (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h),
                               rtol=0, atol=1e-9)


def test_gradient_matches_finite_differences():
    theta, X, K = small_problem(1)
    L, g = mlp.loss_and_grad(theta, X, K, **DIMS)
    rng = np.random.default_rng(2)
    idx = rng.choice(theta.size, 60, replace=False)
    h = 1e-6
    for i in idx:
        tp = theta.copy(); tp[i] += h
        tm = theta.copy(); tm[i] -= h
        fd = (mlp.loss_and_grad(tp, X, K, **DIMS)[0] - mlp.loss_and_grad(tm, X, K, **DIMS)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, np.abs(g).max())


def test_gradient_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    theta, X, K = small_problem(3)
    L, g = mlp.loss_and_grad(theta, X, K, **DIMS)
    t = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    shapes = mlp.param_shapes(**DIMS)
    parts, off = [], 0
    for s in shapes:
        size = int(np.prod(s))
        parts.append(t[off:off + size].reshape(s))
        off += size
    W1, b1, W2, b2, W3, b3 = parts
    x = torch.tensor(X, dtype=torch.float64)
    gelu = torch.nn.functional.gelu  # exact erf form by default
    phi = gelu(gelu(x @ W1.T + b1) @ W2.T + b2) @ W3.T + b3
    B = x.shape[0]
    loss = ((phi @ phi.T - torch.tensor(K)) ** 2).sum() / (B * B)
    loss.backward()
    assert L == pytest.approx(loss.item(), rel=1e-12)
    np.testing.assert_allclose(g, t.grad.numpy(), rtol=1e-10, atol=1e-12)


def test_loss_closed_form_and_zero_at_fit():
    # one output feature, linear map: Phi = X w, K = Phi Phi^T exactly -> loss 0, gradient 0
    theta, X, _ = small_problem(4)
    phi, _ = mlp.forward(theta, X, **DIMS)
    K = phi @ phi.T
    L, g = mlp.loss_and_grad(theta, X, K, **DIMS)
    assert L == pytest.approx(0.0, abs=1e-24)
    assert np.abs(g).max() <= 1e-12
    L2, _ = mlp.loss_and_grad(theta, X, K + 0.5, **DIMS)
    assert L2 == pytest.approx(0.25, rel=1e-12)  # every entry off by 0.5


def test_bf16_operand_rounding_is_small_and_exact_on_bf16_values():
    theta, X, K = small_problem(5)
    L, g = mlp.loss_and_grad(theta, X, K, **DIMS)
    Lb, gb = mlp.loss_and_grad(theta, X, K, **DIMS, bf16_operands=True)
    assert abs(Lb - L) <= 2e-2 * abs(L) and np.abs(gb - g).max() <= 3e-2 * np.abs(g).max()
    assert mlp.bf16(np.array([1.0 + 2 ** -8])) == 1.0  # tie to even
    assert mlp.bf16(np.array([1.0 + 3 * 2 ** -8])) == 1.0 + 2 ** -6


def test_adam_first_step():
    theta = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -0.1, 0.0])
    t1, m, v = mlp.adam_step(theta, np.zeros(3), np.zeros(3), g, 1, lr=0.01)
    # bias-corrected first step moves every coordinate by lr * sign(g) (up to eps)
    np.testing.assert_allclose(t1, theta - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_kmeanspp_samples_proportional_to_d2():
    # second seed after a fixed first one: frequencies follow dmin / sum(dmin)
    rng = np.random.default_rng(8)
    F = rng.normal(0, 1, (12, 3))
    p = ((F - F[0]) ** 2).sum(axis=1)
    p = p / p.sum()
    draws = 20000
    counts = np.zeros(12)
    u = rng.random((draws, 2))
    u[:, 0] = 0.0  # first seed = row 0
    for t in range(draws):
        seeds, _, _ = mlp.kmeanspp(F, 2, u[t])
        counts[seeds[1]] += 1
    assert counts[0] == 0
    chi2 = ((counts[1:] - draws * p[1:]) ** 2 / (draws * p[1:])).sum()
    assert chi2 < 40.0  # 10 degrees of freedom; p-value ~ 1e-5 at 40


def test_kmeanspp_separated_blobs_and_labels():
    rng = np.random.default_rng(9)
    mu = np.array([[0.0, 0.0], [100.0, 0.0], [0.0, 100.0]])
    F = mu[np.repeat(np.arange(3), 50)] + rng.normal(0, 1, (150, 2))
    seeds, lab, margins = mlp.kmeanspp(F, 3, rng.random(3))
    assert len({int(s) // 50 for s in seeds}) == 3  # one seed per blob
    D = ((F[:, None] - F[seeds][None]) ** 2).sum(-1)
    np.testing.assert_array_equal(lab, np.argmin(D, axis=1))
    assert np.all(margins[1:] >= 0)


def test_feature_lloyd_matches_sklearn():
    sk = pytest.importorskip("sklearn.cluster")
    rng = np.random.default_rng(6)
    mu = rng.normal(0, 4, (5, 8))
    F = mu[rng.integers(0, 5, 400)] + rng.normal(0, 1, (400, 8))
    l0 = rng.integers(0, 5, 400).astype(np.int32)
    lab, it = mlp.lloyd(F, 5, l0, 100)
    init = np.stack([F[l0 == c].mean(axis=0) for c in range(5)])
    km = sk.KMeans(n_clusters=5, init=init, n_init=1, max_iter=100, tol=0.0, algorithm="lloyd").fit(F)
    np.testing.assert_array_equal(km.labels_, lab)
