"""The C ABI on a host without a GPU: the library loads, exports every entry
point include/kkm.h declares, and rejects bad arguments before any device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kkm.h")


def declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:kkm_status|size_t|int64_t|const char \*)\s*(kkm_\w+)\(", txt, re.M)))


@pytest.fixture(scope="module")
def lib():
    import paper_2501_05587_amd as kkm
    return kkm.lib()


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert {"kkm_gram", "kkm_iterate", "kkm_fit"} <= set(names)
    for nm in names:
        assert hasattr(lib, nm), nm


def test_binding_names_match_header():
    import paper_2501_05587_amd as kkm
    assert set(kkm.EXPORTS) == set(declared())


def test_argument_validation_without_device_work(lib):
    vp = ctypes.c_void_p
    # kkm_gram: n = 0
    assert lib.kkm_gram(None, 0, 4, 4, 2, 1.0, 0.0, 1, 0, 0, None, 0, None, None, 0, None) == -1
    assert b"bad sizes" in lib.kkm_last_error()
    # Gaussian with gamma <= 0 and a bad degree
    fake = vp(16)
    assert lib.kkm_gram(fake, 8, 4, 4, 2, -1.0, 0.0, 1, 0, 0, fake, 8, fake, None, 0, None) == -1
    assert lib.kkm_gram(fake, 8, 4, 4, 1, 1.0, 1.0, 0, 0, 0, fake, 8, fake, None, 0, None) == -1
    assert lib.kkm_gram(fake, 8, 4, 4, 7, 1.0, 1.0, 1, 0, 0, fake, 8, fake, None, 0, None) == -1
    # ldx < d, ldk < n
    assert lib.kkm_gram(fake, 8, 4, 3, 2, 1.0, 0.0, 1, 0, 0, fake, 8, fake, None, 0, None) == -1
    assert lib.kkm_gram(fake, 8, 4, 4, 2, 1.0, 0.0, 1, 0, 0, fake, 7, fake, None, 0, None) == -1
    # kkm_iterate: k > n, aliasing, k too large
    z = None
    assert lib.kkm_iterate(fake, 0, 8, fake, 8, 9, fake, 0, vp(32), fake, fake, fake, z, z, z, 0, z) == -1
    assert lib.kkm_iterate(fake, 0, 8, fake, 8, 2, fake, 0, fake, fake, fake, fake, z, z, z, 0, z) == -1
    assert lib.kkm_iterate(fake, 0, 5000, fake, 5000, 2000, fake, 0, vp(32), fake, fake, fake, z, z,
                           z, 0, z) == -5
    assert lib.kkm_iterate(fake, 0, 8, fake, 8, 2, fake, 9, vp(32), fake, fake, fake, z, z, z, 0, z) == -1
    # kkm_fit: k = 0, negative max_iter
    J = ctypes.c_double()
    it = ctypes.c_int32()
    assert lib.kkm_fit(fake, 8, 4, 4, 0, 2, 1.0, 0.0, 1, fake, 5, 1, fake, ctypes.byref(J),
                       ctypes.byref(it), None, 0, None) == -1
    assert lib.kkm_fit(fake, 8, 4, 4, 2, 2, 1.0, 0.0, 1, fake, -1, 1, fake, ctypes.byref(J),
                       ctypes.byref(it), None, 0, None) == -1


def test_workspace_sizes(lib):
    import paper_2501_05587_amd as kkm
    assert kkm.iterate_workspace_bytes(0, 3) == 0
    small = kkm.iterate_workspace_bytes(1000, 4)
    big = kkm.iterate_workspace_bytes(200000, 64)
    assert 0 < small < big
    # partial sums stay a small fraction of the n x n matrix they summarise
    assert big < 0.002 * 200000 ** 2 * 4
    assert kkm.gram_workspace_bytes(1000, 16) >= 1000 * 4
