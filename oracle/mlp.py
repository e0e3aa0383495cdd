"""FP64 reference of the learned feature map and its warm start.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Plain numpy, written from
the definitions:

* phi_theta: R^d -> R^h1 -> R^h2 -> R^out, z = W a + b per layer, GELU after the
  first two layers (exact erf form, GELU(z) = z/2 (1 + erf(z / sqrt 2))), the last
  layer linear.  Parameters live in one flat vector, in the order
  W1 [h1, d], b1 [h1], W2 [h2, h1], b2 [h2], W3 [out, h2], b3 [out] (row-major).
* loss on a batch of B points with kernel values K_B (B x B):
      L = (1/B^2) || Phi Phi^T - K_B ||_F^2 ,   Phi = phi_theta(X_B) (B x out),
  so dL/dPhi = (4/B^2) (Phi Phi^T - K_B) Phi (K_B symmetric); the rest is the
  chain rule through the layers.
* Adam (Kingma and Ba, 2015) with bias correction.
* Lloyd iterations with explicit centroids on feature vectors (the cheap
  iterations of the warm start): d_ic = ||f_i - mean_{j in c} f_j||^2, argmin
  with the lowest index on ties, an empty cluster at +inf.

`bf16_operands=True` rounds every matrix-product operand to bfloat16 (round to
nearest even) before the product, where the GPU's matrix units take bfloat16
inputs; accumulation stays FP64 here.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf


def param_shapes(d, h1=512, h2=512, out=256):
    return [(h1, d), (h1,), (h2, h1), (h2,), (out, h2), (out,)]


def param_count(d, h1=512, h2=512, out=256):
    return sum(int(np.prod(s)) for s in param_shapes(d, h1, h2, out))


def unpack(theta, d, h1=512, h2=512, out=256):
    parts, off = [], 0
    for s in param_shapes(d, h1, h2, out):
        size = int(np.prod(s))
        parts.append(theta[off:off + size].reshape(s))
        off += size
    return parts


def bf16(x):
    """Nearest bfloat16 value (ties to even) of x taken as float32."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def _op(x, bf):
    return bf16(x) if bf else np.asarray(x, dtype=np.float64)


def forward(theta, X, d, h1=512, h2=512, out=256, bf16_operands=False):
    """Returns (Phi, cache) with every layer's input and pre-activation."""
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(theta, np.float64), d, h1, h2, out)
    a0 = np.asarray(X, dtype=np.float64)
    z1 = _op(a0, bf16_operands) @ _op(W1, bf16_operands).T + b1
    a1 = gelu(z1)
    z2 = _op(a1, bf16_operands) @ _op(W2, bf16_operands).T + b2
    a2 = gelu(z2)
    phi = _op(a2, bf16_operands) @ _op(W3, bf16_operands).T + b3
    return phi, dict(a0=a0, z1=z1, a1=a1, z2=z2, a2=a2)


def loss_and_grad(theta, XB, KB, d, h1=512, h2=512, out=256, bf16_operands=False):
    """L = (1/B^2) ||Phi Phi^T - K_B||_F^2 and dL/dtheta (flat, FP64)."""
    theta = np.asarray(theta, np.float64)
    W1, b1, W2, b2, W3, b3 = unpack(theta, d, h1, h2, out)
    B = XB.shape[0]
    phi, c = forward(theta, XB, d, h1, h2, out, bf16_operands)
    G = phi @ phi.T - np.asarray(KB, np.float64)
    L = float((G * G).sum()) / (B * B)
    dphi = (4.0 / (B * B)) * (G @ phi)
    bf = bf16_operands
    # layer 3 (linear)
    gW3 = _op(dphi, bf).T @ _op(c["a2"], bf)
    gb3 = dphi.sum(axis=0)
    da2 = _op(dphi, bf) @ _op(W3, bf)
    dz2 = da2 * gelu_grad(c["z2"])
    gW2 = _op(dz2, bf).T @ _op(c["a1"], bf)
    gb2 = dz2.sum(axis=0)
    da1 = _op(dz2, bf) @ _op(W2, bf)
    dz1 = da1 * gelu_grad(c["z1"])
    gW1 = _op(dz1, bf).T @ _op(c["a0"], bf)
    gb1 = dz1.sum(axis=0)
    grad = np.concatenate([g.ravel() for g in (gW1, gb1, gW2, gb2, gW3, gb3)])
    return L, grad


def adam_step(theta, m, v, grad, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); returns new (theta, m, v)."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mhat = m / (1 - beta1 ** t)
    vhat = v / (1 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def lloyd_step(F, k, labels):
    """One Lloyd step with explicit centroids on feature rows F.
    Returns (labels_out, D, n_changed)."""
    F = np.asarray(F, np.float64)
    n = F.shape[0]
    D = np.full((n, k), np.inf)
    for c in range(k):
        m = labels == c
        if m.any():
            mu = F[m].mean(axis=0)
            D[:, c] = ((F - mu) ** 2).sum(axis=1)
    out = np.argmin(D, axis=1).astype(np.int32)
    return out, D, int((out != labels).sum())


def kmeanspp(F, k, uniforms):
    """K-means++ seeding by D^2 sampling (Arthur and Vassilvitskii, 2007) with the
    caller's uniforms u_t in [0,1): seed 0 is row floor(u_0 n); seed t is the
    first row whose running sum of dmin exceeds u_t * sum(dmin), dmin being the
    squared distance to the nearest earlier seed.  Returns (seeds, labels of the
    nearest seed with the lowest index on ties, margins): margins[t] is the
    distance from u_t * total to the nearer cumulative-sum boundary, relative to
    the total (how close the draw came to picking a neighbouring row)."""
    F = np.asarray(F, np.float64)
    n = F.shape[0]
    seeds = [min(int(uniforms[0] * n), n - 1)]
    margins = [np.inf]
    dmin = ((F - F[seeds[0]]) ** 2).sum(axis=1)
    for t in range(1, k):
        cum = np.cumsum(dmin)
        total = cum[-1]
        target = uniforms[t] * total
        i = int(np.searchsorted(cum, target, side="right"))
        i = min(i, n - 1)
        lo = cum[i - 1] if i > 0 else 0.0
        margins.append(min(target - lo, cum[i] - target) / total if total > 0 else np.inf)
        seeds.append(i)
        dmin = np.minimum(dmin, ((F - F[i]) ** 2).sum(axis=1))
    S = F[seeds]
    D = ((F[:, None, :] - S[None, :, :]) ** 2).sum(axis=2)
    return np.array(seeds, np.int32), np.argmin(D, axis=1).astype(np.int32), np.array(margins)


def lloyd(F, k, labels0, max_iter):
    """Lloyd to convergence (no label changes) or max_iter steps; returns (labels, iters)."""
    cur = np.asarray(labels0, np.int32)
    for t in range(max_iter):
        nxt, _, ch = lloyd_step(F, k, cur)
        cur = nxt
        if ch == 0:
            return cur, t + 1
    return cur, max_iter
