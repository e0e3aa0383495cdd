"""kkm_iterate_noalloc (the step on the library's per-device scratch array)
against kkm_iterate with a workspace, through the C ABI: the same kernels on
the same inputs, so every output must be bitwise equal.  Two calls in a row,
the second on a smaller problem, so the second runs on whatever the first
left in the shared array; then a problem whose scratch would exceed the
array is rejected before any device work."""
import sys

import numpy as np
import pytest

import datagen

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


def one_case(kkm, n, k, k_store, seed):
    import torch
    w = datagen.WORKLOADS["gmm200k"]
    X, _ = w.points(rows=n)
    Xd = torch.from_numpy(X).cuda()
    K, dg = kkm.kkm_gram(Xd, w.kernel, w.gamma, k_store=k_store)
    lab = torch.from_numpy(np.random.default_rng(seed).integers(0, k, n).astype(np.int32)).cuda()
    say("no-alloc step: n=%d k=%d k_store=%d" % (n, k, k_store))
    ref = kkm.kkm_iterate(K, dg, lab, k, D_out=True, ctilde_out=True)
    got = kkm.kkm_iterate_noalloc(K, dg, lab, k, D_out=True, ctilde_out=True)
    torch.cuda.synchronize()
    for a, b, nm in zip(ref, got, ("labels", "counts", "n_changed", "J_in", "D", "ctilde")):
        assert torch.equal(a, b), nm
    return got


def test_noalloc_matches_workspace_entry_point(kkm):
    assert kkm.iterate_noalloc_max_bytes() >= kkm.iterate_workspace_bytes(200000, 64)
    # the larger problem first, then a smaller one over what it left behind
    one_case(kkm, 20000, 64, kkm.F32, 1)
    one_case(kkm, 3001, 13, kkm.BF16, 2)
    got = one_case(kkm, 777, 5, kkm.F32, 3)
    assert int(got[2].item()) >= 0


def test_noalloc_rejects_oversized_problem(kkm):
    import torch
    n, k = 300000, 64
    assert kkm.iterate_workspace_bytes(n, k) > kkm.iterate_noalloc_max_bytes()
    # the size check comes before anything touches the (tiny) buffers passed
    t = torch.zeros(16, dtype=torch.float32, device="cuda")
    lab = torch.zeros(16, dtype=torch.int32, device="cuda")
    st = kkm.lib().kkm_iterate_noalloc(t.data_ptr(), kkm.F32, n, t.data_ptr(), n, k, lab.data_ptr(),
                                       0, lab.data_ptr() + 4, lab.data_ptr() + 8, t.data_ptr(),
                                       t.data_ptr(), None, None, None)
    assert st == -5
    assert b"scratch" in kkm.lib().kkm_last_error()
