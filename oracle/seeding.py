"""FP64 reference of k-means++ seeding on the kernel matrix (a warm start that
needs no learned features).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Plain numpy.

K-means++ (Arthur and Vassilvitskii, 2007; the paper's Sec. 2.1 names it as an
initialisation) run in the feature space of the kernel: the squared distance of
point i to a chosen seed s is ||phi(x_i) - phi(x_s)||^2 = K_ii + K_ss - 2 K_is
(the kernel trick of Sec. 2.2 applied to two single points), clamped at 0 against
rounding.  Seed 0 is row floor(u_0 n); seed t is the first row whose running sum
of dmin (the squared distance to the nearest earlier seed) exceeds u_t * sum(dmin);
the uniforms come from the caller.  Each point is then labelled with its nearest
seed (lowest seed index on ties).
"""
from __future__ import annotations

import numpy as np


def _dist(K, diag, s):
    return np.maximum(diag + diag[s] - 2.0 * K[s], 0.0)


def kernel_kmeanspp(K, k, uniforms):
    """Returns (seeds int32 [k], labels int32 [n], margins [k]); margins[t] is the
    distance of u_t * total to the nearer running-sum boundary, relative to the
    total (how close draw t came to picking a neighbouring row)."""
    K = np.asarray(K, np.float64)
    n = K.shape[0]
    diag = np.diag(K).copy()
    seeds = [min(int(uniforms[0] * n), n - 1)]
    margins = [np.inf]
    dmin = _dist(K, diag, seeds[0])
    for t in range(1, k):
        cum = np.cumsum(dmin)
        total = cum[-1]
        if total > 0:
            target = uniforms[t] * total
            i = min(int(np.searchsorted(cum, target, side="right")), n - 1)
            lo = cum[i - 1] if i > 0 else 0.0
            margins.append(min(target - lo, cum[i] - target) / total)
        else:  # every point coincides with a seed
            i = min(int(uniforms[t] * n), n - 1)
            margins.append(np.inf)
        seeds.append(i)
        dmin = np.minimum(dmin, _dist(K, diag, i))
    D = np.stack([_dist(K, diag, s) for s in seeds], axis=1)
    return np.array(seeds, np.int32), np.argmin(D, axis=1).astype(np.int32), np.array(margins)
