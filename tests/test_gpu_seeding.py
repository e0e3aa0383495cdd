"""k-means++ seeding on the kernel matrix (GPU) against the FP64 reference.

The GPU computes the kernel distances K_ii + K_ss - 2K_is in FP32 from its own
K; the reference runs on the same K values in FP64.  A draw may differ only
where the reference's target lay next to a running-sum boundary (margin); labels
may differ only where two seeds are equally near."""
import sys

import numpy as np
import pytest

import datagen
import oracle
from oracle import seeding

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


def check(kkm, X, k, kernel, gamma, k_store, seed):
    import torch
    say("kernel k-means++", X.shape, k, kernel, k_store)
    K, diag = kkm.kkm_gram(to_dev(X), kernel, gamma, 1.0, 2, k_store=k_store)
    u = np.random.default_rng(seed).random(k)
    s_gpu, lab_gpu = kkm.kkm_kernel_kmeanspp(K, diag, k, u)
    torch.cuda.synchronize()
    Kh = K.float().cpu().numpy().astype(np.float64)
    s_ref, lab_ref, margins = seeding.kernel_kmeanspp(Kh, k, u)
    s_gpu = s_gpu.cpu().numpy()
    diff = np.nonzero(s_gpu != s_ref)[0]
    if diff.size:
        assert margins[diff[0]] < 1e-5, (diff[0], margins[diff[0]])
        return
    lab_gpu = lab_gpu.cpu().numpy()
    dg = np.diag(Kh)
    D = np.maximum(dg[:, None] + dg[s_ref][None, :] - 2.0 * Kh[:, s_ref], 0.0)
    srt = np.sort(D, axis=1)
    near = (srt[:, 1] - srt[:, 0]) <= 1e-5 * np.maximum(srt[:, 1], 1e-30) if k > 1 else np.zeros(len(X), bool)
    bad = (lab_gpu != lab_ref) & ~near
    assert not bad.any(), np.nonzero(bad)[0][:10]


@pytest.mark.parametrize("k_store", [0, 1])
def test_gaussian_mixture(kkm, k_store):
    X, _ = datagen.gmm(3000, 24, 17, 0.4, 71)
    check(kkm, X, 17, kkm.GAUSS, 1.0 / 24, k_store, 72)


def test_polynomial_and_ragged(kkm):
    X, _ = datagen.gmm(1029, 9, 5, 0.3, 73)
    check(kkm, X, 7, kkm.POLY, 0.2, 0, 74)


def test_every_point_a_seed(kkm):
    rng = np.random.default_rng(75)
    X = rng.normal(0, 1, (5, 3)).astype(np.float32)
    import torch
    K, diag = kkm.kkm_gram(to_dev(X), kkm.GAUSS, 0.5)
    s, lab = kkm.kkm_kernel_kmeanspp(K, diag, 5, rng.random(5))
    torch.cuda.synchronize()
    s = s.cpu().numpy()
    assert sorted(s.tolist()) == list(range(5))
    np.testing.assert_array_equal(lab.cpu().numpy()[s], np.arange(5))
    s1, lab1 = kkm.kkm_kernel_kmeanspp(K[:1, :1], diag[:1], 1, [0.3])
    torch.cuda.synchronize()
    assert s1.item() == 0 and lab1.item() == 0


def test_bad_arguments(kkm):
    import torch
    K, diag = kkm.kkm_gram(to_dev(np.ones((4, 2), np.float32)), kkm.LINEAR)
    with pytest.raises(kkm.KKMError):
        kkm.kkm_kernel_kmeanspp(K, diag, 5, np.zeros(5))      # k > n
    with pytest.raises(kkm.KKMError):
        kkm.kkm_kernel_kmeanspp(K, diag, 2, [0.5, 1.0])       # u outside [0, 1)
    torch.cuda.synchronize()


def test_refine_equals_fit_loop(kkm):
    """kkm_gram + kkm_refine reproduces kkm_fit_ex bit for bit (the same loop on
    the same K), for both storage types."""
    import torch
    X, _ = datagen.gmm(2500, 16, 6, 0.5, 76)
    l0 = to_dev(datagen.uniform_labels(2500, 6, 77))
    Xd = to_dev(X)
    for gp, ks in ((0, 0), (1, 1)):
        a = kkm.kkm_fit_ex(Xd, 6, l0, kkm.GAUSS, 1.0 / 16, gram_prec=gp, k_store=ks, max_iter=40)
        K, diag = kkm.kkm_gram(Xd, kkm.GAUSS, 1.0 / 16, gram_prec=gp, k_store=ks)
        b = kkm.kkm_refine(K, diag, 6, l0, max_iter=40)
        torch.cuda.synchronize()
        assert torch.equal(a["labels"], b["labels"])
        assert a["iters"] == b["iters"] and a["objective"] == b["objective"]
        np.testing.assert_array_equal(a["J_trace"], b["J_trace"])


def test_kernel_seeded_refine_matches_oracle(kkm):
    """Seeds from K, then the exact loop: the whole run against the oracle's
    seeding followed by its fit on the same K values."""
    import torch
    X, _ = datagen.gmm(1500, 12, 8, 0.4, 78)
    u = np.random.default_rng(79).random(8)
    K, diag = kkm.kkm_gram(to_dev(X), kkm.GAUSS, 1.0 / 12)
    seeds, lab0 = kkm.kkm_kernel_kmeanspp(K, diag, 8, u)
    r = kkm.kkm_refine(K, diag, 8, lab0, max_iter=50)
    torch.cuda.synchronize()
    Kh = K.cpu().numpy().astype(np.float64)
    s_ref, l_ref, margins = seeding.kernel_kmeanspp(Kh, 8, u)
    if (seeds.cpu().numpy() != s_ref).any():
        pytest.skip("a draw landed on a running-sum boundary (margin %.2g)" % margins.min())
    ref = oracle.fit(Kh, 8, l_ref, 50)
    recs = oracle.trajectory(Kh, 8, l_ref, 50)
    tie = any((st["gap"] < 4e-6).any() for _, st in recs)
    if not tie:
        np.testing.assert_array_equal(r["labels"].cpu().numpy(), ref["labels"])
        assert r["iters"] == ref["iters"]
    assert abs(r["objective"] - ref["objective"]) <= 1e-5 * 1500
