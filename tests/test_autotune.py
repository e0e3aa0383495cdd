"""Host logic of the batched-form autotuner (no GPU): buckets and lookup."""
import numpy as np

from paper_2501_05587_amd import autotune


class _Rows:
    def __init__(self, n):
        self.shape = (n, 3)


def test_buckets_cover_the_ranges():
    assert autotune.bucket(1, 1) == (8, 1)
    assert autotune.bucket(256, 4) == (8, 1)
    assert autotune.bucket(257, 5) == (9, 2)
    assert autotune.bucket(16384, 16) == (14, 2)
    assert autotune.bucket(16385, 17) == (15, 3)
    assert autotune.bucket(100, 64) == (8, 3)
    assert autotune.bucket(100, 65) == (8, 4)
    # every n in (2^(a-1), 2^a] shares a bucket
    for a in range(9, 16):
        for n in (2 ** (a - 1) + 1, 2 ** a):
            assert autotune.bucket(n, 3)[0] == a


def test_apply_fills_chunk_rows_from_the_table():
    table = {"f32": {autotune.key(1000, 10): {"chunk_rows": 128}},
             "bf16": {autotune.key(1000, 10): {"chunk_rows": 512}}}
    probs = [dict(X=_Rows(1000), k=10), dict(X=_Rows(1000), k=50), dict(X=_Rows(5000), k=10)]
    got = autotune.apply(probs, table, k_store=0)
    assert [p["chunk_rows"] for p in got] == [128, 0, 0]
    got = autotune.apply(probs, table, k_store=1)
    assert [p["chunk_rows"] for p in got] == [512, 0, 0]
    assert "chunk_rows" not in probs[0]  # the input dicts are left alone
    assert autotune.apply(probs, {}, 0)[0]["chunk_rows"] == 0


def test_candidates_are_powers_of_two():
    c = np.array(autotune.CANDIDATES)
    assert (c & (c - 1) == 0).all() and (np.diff(c) > 0).all()
