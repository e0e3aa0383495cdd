"""The host reference roundings, pinned to the formats' definitions."""
import numpy as np

from quantref import bf16_round, e4m3_round, fp8_rowscaled


def e4m3_values():
    """All finite non-negative OCP E4M3 values from the bit layout (bias 7;
    exponent 15 with mantissa 7 is NaN)."""
    out = []
    for e in range(16):
        for m in range(8):
            if e == 15 and m == 7:
                continue
            out.append(m * 2.0 ** -9 if e == 0 else (1 + m / 8) * 2.0 ** (e - 7))
    return np.array(sorted(out))


def test_e4m3_value_set():
    v = e4m3_values()
    assert v.max() == 448.0 and v[1] == 2.0 ** -9 and len(v) == 127
    np.testing.assert_array_equal(e4m3_round(v), v)
    np.testing.assert_array_equal(e4m3_round(-v), -v)


def test_e4m3_ties_to_even_and_nearest():
    v = e4m3_values()
    mid = (v[:-1] + v[1:]) / 2
    got = e4m3_round(mid)
    # a tie goes to the neighbour whose 3-bit mantissa is even
    for lo, hi, g in zip(v[:-1], v[1:], got):
        assert g in (lo, hi)
    codes = {x: i for i, x in enumerate(v)}  # consecutive values alternate mantissa parity
    assert all(codes[g] % 2 == 0 for g in got)
    rng = np.random.default_rng(0)
    x = rng.uniform(-448, 448, 5000)
    r = e4m3_round(x)
    idx = np.searchsorted(v, np.abs(x))
    lo = v[np.clip(idx - 1, 0, len(v) - 1)]
    hi = v[np.clip(idx, 0, len(v) - 1)]
    best = np.minimum(np.abs(np.abs(x) - lo), np.abs(np.abs(x) - hi))
    assert np.all(np.abs(np.abs(r) - np.abs(x)) <= best + 1e-12)


def test_bf16_round():
    x = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -2.5, 3.0e38, 1e-40], np.float32)
    r = bf16_round(x)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == np.float32(1 + 2 ** -6) and r[3] == -2.5
    assert (r.view(np.uint32) & 0xFFFF == 0).all()
    rng = np.random.default_rng(1)
    y = rng.normal(0, 3, 10000).astype(np.float32)
    assert np.all(np.abs(bf16_round(y) - y) <= np.abs(y) * 2.0 ** -8)


def test_fp8_rowscale():
    X = np.array([[0.0, 1.0, -3.5], [0, 0, 0], [1e-3, 2e-3, 5e-4]], np.float32)
    q, s = fp8_rowscaled(X)
    assert s[0] == np.float32(3.5 / 448) and s[1] == 1.0
    assert np.abs(q).max() == 448.0 and q[1].tolist() == [0, 0, 0]
    np.testing.assert_allclose(q * s[:, None], X, rtol=2 ** -4, atol=0)
