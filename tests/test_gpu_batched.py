"""Batched form on the GPU, through the C ABI.

Each problem of a batch must reproduce its own single-problem run
(kkm_fit_ex) bit for bit when chunk_rows is left at its default, the graph
replay must reproduce the direct launches, and a subset is checked against
the FP64 oracle.  The batches mix sizes across Gram tiles, sweep strips and
ragged tails, d and k, and all three kernel functions.
"""
import sys

import numpy as np
import pytest

import datagen
import oracle

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


# (n, d, k, kernel, gamma, coef0, degree)
SPECS = [
    (1, 3, 1, "gauss", 0.5, 0.0, 1),
    (5, 1, 2, "linear", 1.0, 0.0, 1),
    (100, 32, 5, "gauss", 1 / 32, 0.0, 1),
    (257, 64, 17, "poly", 1 / 64, 1.0, 2),
    (700, 100, 9, "gauss", 1 / 100, 0.0, 1),
    (1500, 256, 64, "gauss", 1 / 256, 0.0, 1),
    (1025, 7, 3, "linear", 1.0, 0.0, 1),
    (3000, 32, 40, "gauss", 1 / 32, 0.0, 1),
    (4100, 128, 12, "poly", 1 / 128, 0.5, 3),
    (130, 33, 2, "gauss", 1 / 33, 0.0, 1),
]
KERNELS = {"linear": 0, "poly": 1, "gauss": 2}


def build(kkm, specs, seed):
    probs, labs, host = [], [], []
    for b, (n, d, k, kern, g, c0, deg) in enumerate(specs):
        X, _ = datagen.gmm(n, d, max(k, 2), 0.3, seed + b)
        l0 = datagen.uniform_labels(n, k, seed + 1000 + b)
        probs.append(dict(X=to_dev(X), k=k, kernel=KERNELS[kern], gamma=g, coef0=c0,
                          degree=deg))
        labs.append(l0)
        host.append((X, l0))
    return probs, to_dev(np.concatenate(labs)), host


def split(labels, specs):
    out, off = [], 0
    for s in specs:
        out.append(labels[off:off + s[0]])
        off += s[0]
    return out


PAIRS = [(0, 0), (1, 0), (1, 1), (2, 0)]  # (gram_prec, k_store)


@pytest.mark.parametrize("gp,ks", PAIRS)
def test_each_problem_matches_its_single_run(kkm, gp, ks):
    import torch
    probs, l0, _ = build(kkm, SPECS, 500)
    say("batched", len(probs), "problems gram_prec", gp, "k_store", ks)
    r = kkm.kkm_fit_batched(probs, l0, gram_prec=gp, k_store=ks, max_iter=25)
    torch.cuda.synchronize()
    got = split(r["labels"].cpu().numpy(), SPECS)
    l0s = split(l0, SPECS)
    for b, p in enumerate(probs):
        say("  single", b, SPECS[b])
        one = kkm.kkm_fit_ex(p["X"], p["k"], l0s[b], p["kernel"], p["gamma"], p["coef0"],
                             p["degree"], gram_prec=gp, k_store=ks, max_iter=25)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(got[b], one["labels"].cpu().numpy(), err_msg="problem %d" % b)
        assert r["iters"][b] == one["iters"], b
        assert r["objective"][b] == one["objective"], (b, r["objective"][b], one["objective"])


def test_graph_replay_equals_direct_launches(kkm):
    import torch
    probs, l0, _ = build(kkm, SPECS, 600)
    a = kkm.kkm_fit_batched(probs, l0, gram_prec=1, max_iter=30, use_graph=True)
    b = kkm.kkm_fit_batched(probs, l0, gram_prec=1, max_iter=30, use_graph=False)
    c = kkm.kkm_fit_batched(probs, l0, gram_prec=1, max_iter=30, use_graph=True)
    torch.cuda.synchronize()
    for x in (b, c):
        assert torch.equal(a["labels"], x["labels"])
        np.testing.assert_array_equal(a["iters"], x["iters"])
        np.testing.assert_array_equal(a["objective"], x["objective"])
    # problems retire at different steps
    assert len(set(a["iters"].tolist())) > 1


def test_fixed_iterations_and_zero(kkm):
    import torch
    specs = SPECS[2:6]
    probs, l0, _ = build(kkm, specs, 700)
    l0s = split(l0, specs)
    for mi, conv in ((0, True), (7, False), (3, True)):
        r = kkm.kkm_fit_batched(probs, l0, max_iter=mi, check_convergence=conv)
        torch.cuda.synchronize()
        got = split(r["labels"].cpu().numpy(), specs)
        for b, p in enumerate(probs):
            one = kkm.kkm_fit_ex(p["X"], p["k"], l0s[b], p["kernel"], p["gamma"], p["coef0"],
                                 p["degree"], max_iter=mi, check_convergence=conv)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(got[b], one["labels"].cpu().numpy())
            assert r["iters"][b] == one["iters"]
            assert r["objective"][b] == one["objective"]
        if mi == 0:
            assert torch.equal(r["labels"], l0)
            assert (r["iters"] == 0).all()


def test_subset_against_oracle(kkm):
    """FP32 product and K: each problem's run against the FP64 oracle's run."""
    import torch
    specs = [s for s in SPECS if s[0] <= 1500]
    probs, l0, host = build(kkm, specs, 800)
    r = kkm.kkm_fit_batched(probs, l0, max_iter=30)
    torch.cuda.synchronize()
    got = split(r["labels"].cpu().numpy(), specs)
    for b, (n, d, k, kern, g, c0, deg) in enumerate(specs):
        X, lab0 = host[b]
        say("  oracle", b, specs[b])
        K_or = oracle.kernel_matrix(X, KERNELS[kern], g, c0, deg)
        ref = oracle.fit(K_or, k, lab0, 30)
        recs = oracle.trajectory(K_or, k, lab0, 30)
        scale = np.abs(np.diag(K_or)).sum() + np.abs(K_or).max() * n
        tie = any((st["gap"] < 1e-6 * max(1.0, np.abs(K_or).max()) * 4).any() for _, st in recs)
        if not tie:
            np.testing.assert_array_equal(got[b], ref["labels"], err_msg="problem %d" % b)
            assert r["iters"][b] == ref["iters"], b
        assert abs(r["objective"][b] - ref["objective"]) <= 1e-5 * scale, b


def test_timed_configuration_subset_against_oracle(kkm):
    """The configuration the benchmark times: BF16 product, K stored FP32, sweep
    heights from the tuned table.  Each problem's run against the FP64 oracle's
    run on the bfloat16-rounded points (the product's exact input; the GPU then
    differs only by FP32 accumulation and summation order)."""
    import torch
    from quantref import bf16_round
    from paper_2501_05587_amd import autotune
    table = autotune.load(path=autotune.default_path("gfx950"))
    specs = [s for s in SPECS if s[0] <= 3000]
    probs, l0, host = build(kkm, specs, 900)
    tuned = autotune.apply(probs, table, 0)
    heights = [p["chunk_rows"] for p in tuned]
    say("  tuned heights", heights)
    assert any(h > 0 for h in heights)  # the table covers these sizes
    r = kkm.kkm_fit_batched(tuned, l0, gram_prec=kkm.BF16, k_store=kkm.F32, max_iter=30)
    torch.cuda.synchronize()
    got = split(r["labels"].cpu().numpy(), specs)
    for b, (n, d, k, kern, g, c0, deg) in enumerate(specs):
        X, lab0 = host[b]
        say("  oracle", b, specs[b], "height", heights[b])
        K_or = oracle.kernel_matrix(bf16_round(X), KERNELS[kern], g, c0, deg)
        ref = oracle.fit(K_or, k, lab0, 30)
        recs = oracle.trajectory(K_or, k, lab0, 30)
        scale = np.abs(np.diag(K_or)).sum() + np.abs(K_or).max() * n
        tie = any((st["gap"] < 1e-6 * max(1.0, np.abs(K_or).max()) * 4).any() for _, st in recs)
        if not tie:
            np.testing.assert_array_equal(got[b], ref["labels"], err_msg="problem %d" % b)
            assert r["iters"][b] == ref["iters"], b
        assert abs(r["objective"][b] - ref["objective"]) <= 1e-5 * scale, b


def test_chunk_rows_and_caller_workspace(kkm):
    """A tuned chunk length changes only the summation order; a workspace
    from the caller gives the same run as one the call allocates."""
    import torch
    specs = SPECS[3:9]
    probs, l0, _ = build(kkm, specs, 900)
    base = kkm.kkm_fit_batched(probs, l0, max_iter=15, check_convergence=False)
    for L in (8, 100, 4096):
        tuned = [dict(p, chunk_rows=L) for p in probs]
        r = kkm.kkm_fit_batched(tuned, l0, max_iter=15, check_convergence=False)
        torch.cuda.synchronize()
        agree = (r["labels"] == base["labels"]).float().mean().item()
        assert agree >= 0.995, (L, agree)
        np.testing.assert_allclose(r["objective"], base["objective"], rtol=2e-4)
    nbytes = kkm.kkm_fit_batched_workspace_bytes(probs)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    r = kkm.kkm_fit_batched(probs, l0, max_iter=15, check_convergence=False, ws=ws)
    torch.cuda.synchronize()
    assert torch.equal(r["labels"], base["labels"])
    np.testing.assert_array_equal(r["objective"], base["objective"])


def test_zero_centroid_policy_matches_single_run(kkm):
    import torch
    specs = [(300, 16, 40, "gauss", 0.05, 0.0, 1), (90, 8, 30, "gauss", 0.1, 0.0, 1)]
    probs, l0, _ = build(kkm, specs, 1000)
    r = kkm.kkm_fit_batched(probs, l0, empty_policy=kkm.EMPTY_ZERO_CENTROID, max_iter=20)
    torch.cuda.synchronize()
    got = split(r["labels"].cpu().numpy(), specs)
    l0s = split(l0, specs)
    for b, p in enumerate(probs):
        one = kkm.kkm_fit_ex(p["X"], p["k"], l0s[b], p["kernel"], p["gamma"], empty_policy=1,
                             max_iter=20)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(got[b], one["labels"].cpu().numpy())
        assert r["objective"][b] == one["objective"]


def test_errors(kkm):
    import torch
    specs = SPECS[2:5]
    probs, l0, _ = build(kkm, specs, 1100)
    bad = l0.clone()
    bad[specs[0][0] + 3] = specs[1][2]  # a label == k in problem 1
    with pytest.raises(kkm.KKMError) as e:
        kkm.kkm_fit_batched(probs, bad, max_iter=5)
    assert e.value.status == -2 and "problem 1" in str(e.value)
    with pytest.raises(kkm.KKMError) as e:
        kkm.kkm_fit_batched(probs, bad, max_iter=0)
    assert e.value.status == -2
    Xn = probs[2]["X"].clone()
    Xn[5, 0] = float("nan")
    with pytest.raises(kkm.KKMError) as e:
        kkm.kkm_fit_batched(probs[:2] + [dict(probs[2], X=Xn)], l0, max_iter=5)
    assert e.value.status == -6
    torch.cuda.synchronize()
