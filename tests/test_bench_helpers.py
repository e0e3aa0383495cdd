"""Host-side helpers of bench.py (no GPU): the adjusted Rand index, the HBM
traffic entry that must read null once a kernel's sources change, and the
one-GPU guard."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_ari_against_scikit_learn():
    metrics = pytest.importorskip("sklearn.metrics")
    rng = np.random.default_rng(4)
    for n, ka, kb in ((50, 3, 4), (1000, 10, 7), (300, 1, 5)):
        a = rng.integers(0, ka, n)
        b = np.where(rng.random(n) < 0.7, a, rng.integers(0, kb, n))
        assert bench.ari(a, b) == pytest.approx(metrics.adjusted_rand_score(a, b), abs=1e-12)


def test_ari_invariants():
    a = np.array([0, 0, 1, 1, 2, 2, 2])
    assert bench.ari(a, a) == 1.0
    assert bench.ari(a, (a + 5) * 3) == 1.0  # renamed labels
    assert bench.ari(np.zeros(9, int), np.zeros(9, int)) == 1.0


def test_traffic_reads_null_when_sources_or_size_change(monkeypatch):
    name = "spmm_row_sweep"
    t = bench.TRAFFIC[name]
    expected = (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]) * 1024.0
    current = bench.sources_sha(t["sources"])
    monkeypatch.setitem(bench.TRAFFIC, name, dict(t, sha256=current))
    assert bench.traffic_bytes(name, t["n"]) == pytest.approx(expected)
    assert bench.traffic_bytes(name, t["n"] + 1) is None
    monkeypatch.setitem(bench.TRAFFIC, name, dict(t, sha256="0" * 64))
    assert bench.traffic_bytes(name, t["n"]) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_rowpart_bytes_closed_form():
    # whole strips: every row of strip s has ns - s - 1 strips to its right,
    # W k 4 (0 + 1 + ... + ns - 1) bytes in all
    W, k = 1024, 64
    for ns in (1, 2, 7, 196):
        n = ns * W
        assert bench.rowpart_bytes(n, k, W) == W * k * 4 * ns * (ns - 1) // 2
    # a ragged last strip: its rows have no strip to their right
    assert bench.rowpart_bytes(3 * W - 5, k, W) == bench.rowpart_bytes(3 * W, k, W)
    assert bench.rowpart_bytes(1, 3, W) == 0.0


def test_traffic_of_an_unrecorded_kernel_is_null():
    assert bench.traffic_bytes("no_such_kernel", 200000) is None
