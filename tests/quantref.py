"""Host reference roundings for the precision forms (written from the formats'
definitions; used only to prepare test inputs and expected values).

* bfloat16: the upper 16 bits of an IEEE float32, round to nearest, ties to even.
* OCP FP8 E4M3 (FN): 1 sign, 4 exponent bits (bias 7), 3 mantissa bits, largest
  finite 448, subnormal step 2^-9; round to nearest, ties to even.
* Row scaling: s_i = max_l |x_il| / 448 and x_il / s_i computed as
  x_il * (448 / max_l |x_il|) in float32, clamped to [-448, 448], rounded to E4M3.
"""
import numpy as np


def bf16_round(x):
    """float32 array -> float32 array of the nearest bfloat16 values (ties to even)."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def e4m3_round(y):
    """Nearest OCP E4M3 value (ties to even) of |y| <= 448, as float64."""
    y = np.asarray(y, dtype=np.float64)
    a = np.abs(y)
    e = np.floor(np.log2(np.maximum(a, 2.0 ** -6)))
    step = 2.0 ** (e - 3)
    return np.sign(y) * (np.round(a / step) * step)


def fp8_rowscaled(X):
    """(q, s): E4M3 values q [n, d] (float64) and float32 row scales s [n]."""
    X = np.asarray(X, dtype=np.float32)
    amax = np.abs(X).max(axis=1)
    pos = amax > 0
    s = np.where(pos, amax / np.float32(448.0), np.float32(1.0)).astype(np.float32)
    inv = np.where(pos, np.float32(448.0) / np.where(pos, amax, 1), np.float32(1.0)).astype(np.float32)
    y = np.clip((X * inv[:, None]).astype(np.float32), np.float32(-448.0), np.float32(448.0))
    return e4m3_round(y), s


def fp8_dequantised(X):
    """float32 points s_i * q_il that the FP8 product multiplies (rounded to float32)."""
    q, s = fp8_rowscaled(X)
    return (q * s[:, None].astype(np.float64)).astype(np.float32)
