"""Seeded synthetic inputs for the Kernel K-means workloads.

This module only draws numbers: points, ground-truth components and initial
labels.  It holds none of the method's arithmetic, so both the FP64 oracle and
the HIP library can be fed from it without sharing any computation.

Every generator is deterministic in its seed and draws rows in fixed blocks of
``BLOCK_ROWS`` rows, each block from its own PCG64 stream keyed by
``(seed, block)``.  The first ``m`` rows of a workload therefore do not depend
on how many rows are requested, so a subsample is exactly a prefix of the full
draw.

Workloads (the paper evaluates on libSVM datasets that are not available here;
these synthetic sets stand in for them with the same shapes and value ranges):

* ``rings``     n=1000, d=16, k=4: four concentric 2-D rings (radii 1..4, 250
                points each, uniform angle, radial noise N(0, 0.05^2)); dims
                2..15 are N(0, 0.01^2).  Gaussian kernel, gamma=1.
* ``mnist_like`` n=60000, d=784, k=10: ten means U[0,1]^784, points =
                mean + N(0, 0.1^2) clipped to [0,1], then each entry zeroed with
                probability 0.8 (an MNIST-shaped stand-in: the paper's MNIST set
                has n=60000, d=780).  Polynomial kernel (x.y+1)^2 as in the
                paper's experiments.
* ``gmm``       equal-weight Gaussian mixtures with means N(0,1)^d and isotropic
                spread sigma (the n=200000, d=1024, k=64 precision workload; the
                batched instances; the learned warm-start set in R^128).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

BLOCK_ROWS = 8192

# kernel type codes, identical to the C-ABI enum values
LINEAR, POLY, GAUSS = 0, 1, 2


def _block_rng(seed: int, block: int) -> np.random.Generator:
    return np.random.default_rng([int(seed), int(block)])


def _means_rng(seed: int) -> np.random.Generator:
    return np.random.default_rng([int(seed), 0x6D65616E])  # tag "mean"


def uniform_labels(n: int, k: int, seed: int) -> np.ndarray:
    """Initial labels drawn iid uniform in [0, k) (a random cluster per point,
    as the paper's initialisation does), int32, block-keyed like the points."""
    out = np.empty(n, dtype=np.int32)
    for b in range(0, (n + BLOCK_ROWS - 1) // BLOCK_ROWS):
        lo, hi = b * BLOCK_ROWS, min(n, (b + 1) * BLOCK_ROWS)
        out[lo:hi] = _block_rng(seed, b).integers(0, k, hi - lo, dtype=np.int32)
    return out


def rings(n_per_ring: int = 250, radii=(1.0, 2.0, 3.0, 4.0), d: int = 16,
          radial_sd: float = 0.05, extra_sd: float = 0.01, seed: int = 1):
    """Concentric rings in dims 0-1 plus small Gaussian noise in the rest.

    Returns (X float32 [n, d], truth int32 [n]); ring-major order."""
    rng = _block_rng(seed, 0)
    n = n_per_ring * len(radii)
    X = np.empty((n, d), dtype=np.float64)
    truth = np.empty(n, dtype=np.int32)
    for r_idx, r in enumerate(radii):
        sl = slice(r_idx * n_per_ring, (r_idx + 1) * n_per_ring)
        theta = rng.uniform(0.0, 2.0 * math.pi, n_per_ring)
        rho = r + rng.normal(0.0, radial_sd, n_per_ring)
        X[sl, 0] = rho * np.cos(theta)
        X[sl, 1] = rho * np.sin(theta)
        X[sl, 2:] = rng.normal(0.0, extra_sd, (n_per_ring, d - 2))
        truth[sl] = r_idx
    return X.astype(np.float32), truth


def mnist_like(n: int = 60000, d: int = 784, n_comp: int = 10, noise_sd: float = 0.1,
               zero_frac: float = 0.8, seed: int = 2, rows: int | None = None):
    """Ten-component [0,1]-valued mixture with 80% of entries zeroed.

    ``rows`` (default n) returns only the first ``rows`` points of the size-n draw.
    Returns (X float32 [rows, d], truth int32 [rows])."""
    rows = n if rows is None else rows
    means = _means_rng(seed).uniform(0.0, 1.0, (n_comp, d)).astype(np.float32)
    X = np.empty((rows, d), dtype=np.float32)
    truth = np.empty(rows, dtype=np.int32)
    for b in range(0, (rows + BLOCK_ROWS - 1) // BLOCK_ROWS):
        # a block is always drawn whole (sized by n), then cut to the prefix
        lo, hi = b * BLOCK_ROWS, min(n, (b + 1) * BLOCK_ROWS)
        m = hi - lo
        rng = _block_rng(seed, b)
        comp = rng.integers(0, n_comp, m, dtype=np.int32)
        noise = rng.standard_normal((m, d), dtype=np.float32) * np.float32(noise_sd)
        x = np.clip(means[comp] + noise, 0.0, 1.0)
        keep = rng.random((m, d), dtype=np.float32) >= np.float32(zero_frac)
        take = min(hi, rows) - lo
        X[lo:lo + take] = np.where(keep, x, np.float32(0.0))[:take]
        truth[lo:lo + take] = comp[:take]
    return X, truth


def gmm_means(d: int, n_comp: int, seed: int) -> np.ndarray:
    """Component means N(0,1)^d, float32 [n_comp, d]."""
    return _means_rng(seed).standard_normal((n_comp, d), dtype=np.float32)


def gmm(n: int, d: int, n_comp: int, sigma: float, seed: int, means: np.ndarray | None = None,
        rows: int | None = None):
    """Equal-weight isotropic Gaussian mixture: x = mu_c + sigma * N(0, I).

    ``means`` defaults to ``gmm_means(d, n_comp, seed)``; pass the means of another
    draw to sample fresh points of the same mixture.  ``rows`` returns a prefix.
    Returns (X float32 [rows, d], truth int32 [rows])."""
    rows = n if rows is None else rows
    if means is None:
        means = gmm_means(d, n_comp, seed)
    X = np.empty((rows, d), dtype=np.float32)
    truth = np.empty(rows, dtype=np.int32)
    for b in range(0, (rows + BLOCK_ROWS - 1) // BLOCK_ROWS):
        lo, hi = b * BLOCK_ROWS, min(n, (b + 1) * BLOCK_ROWS)
        m = hi - lo
        rng = _block_rng(seed, b)
        comp = rng.integers(0, n_comp, m, dtype=np.int32)
        noise = rng.standard_normal((m, d), dtype=np.float32)
        take = min(hi, rows) - lo
        X[lo:lo + take] = means[comp[:take]] + np.float32(sigma) * noise[:take]
        truth[lo:lo + take] = comp[:take]
    return X, truth


@dataclasses.dataclass(frozen=True)
class Workload:
    """One named workload: data recipe, kernel and loop protocol."""
    name: str
    n: int
    d: int
    k: int
    kernel: int
    gamma: float
    coef0: float
    degree: int
    max_iter: int
    check_convergence: bool
    data_seed: int
    label_seed: int
    means_seed: int | None = None  # the mixture's means (default: data_seed)
    train_seed: int | None = None  # fresh training draws of the same mixture
    init_seed: int | None = None   # initial parameters of the feature network

    def means(self):
        return gmm_means(self.d, self.k, self.data_seed if self.means_seed is None else self.means_seed)

    def points(self, rows: int | None = None):
        rows = self.n if rows is None else rows
        if self.name == "rings":
            X, t = rings(seed=self.data_seed)
            return X[:rows], t[:rows]
        if self.name == "mnist_like":
            return mnist_like(n=self.n, d=self.d, seed=self.data_seed, rows=rows)
        if self.name in ("gmm200k", "learned100k"):
            return gmm(self.n, self.d, self.k, 0.5, self.data_seed, means=self.means(), rows=rows)
        raise KeyError(self.name)

    def labels0(self, rows: int | None = None):
        rows = self.n if rows is None else rows
        return uniform_labels(self.n, self.k, self.label_seed)[:rows]


WORKLOADS = {
    "rings": Workload("rings", 1000, 16, 4, GAUSS, 1.0, 0.0, 1, 50, True, 1, 101),
    "mnist_like": Workload("mnist_like", 60000, 784, 10, POLY, 1.0, 1.0, 2, 30, False, 2, 102),
    "gmm200k": Workload("gmm200k", 200000, 1024, 64, GAUSS, 1.0 / 1024, 0.0, 1, 30, False, 3, 103),
    # the learned warm-start test set: fresh draws of the 32-component mixture
    # in R^128 (sigma 0.5) that the feature network is trained on; means seed
    # 5000, training draws 5001, test points 5002, initial labels 5003
    "learned100k": Workload("learned100k", 100000, 128, 32, GAUSS, 1.0 / 128, 0.0, 1, 300, True,
                            5002, 5003, means_seed=5000, train_seed=5001, init_seed=5005),
}


def batched_instances(count: int = 512, seed_base: int = 4000):
    """Parameters of the uneven batched instances: n ~ U{256..16384},
    d ~ U{32,64,128,256}, k ~ U{2..64}; each a k-component mixture with
    sigma=0.3 and Gaussian kernel gamma=1/d.  Returns a list of dicts; points
    are drawn lazily with ``gmm(n, d, k, 0.3, seed)``."""
    out = []
    for b in range(count):
        rng = np.random.default_rng([seed_base + b, 0x696E7374])  # tag "inst"
        n = int(rng.integers(256, 16384 + 1))
        d = int(rng.choice([32, 64, 128, 256]))
        k = int(rng.integers(2, 64 + 1))
        out.append(dict(n=n, d=d, k=k, sigma=0.3, gamma=1.0 / d, seed=seed_base + b,
                        label_seed=seed_base + b + 100000))
    return out


def mlp_init_params(d: int, h1: int = 512, h2: int = 512, out: int = 256, seed: int = 0):
    """Initial parameters of the feature network, flat float32 in the order
    W1 [h1, d], b1 [h1], W2 [h2, h1], b2 [h2], W3 [out, h2], b3 [out]:
    W ~ U(-1/sqrt(fan_in), 1/sqrt(fan_in)), b = 0."""
    rng = np.random.default_rng([int(seed), 0x6D6C70])  # tag "mlp"
    parts = []
    for rows, cols in ((h1, d), (h2, h1), (out, h2)):
        lim = 1.0 / math.sqrt(cols)
        parts.append(rng.uniform(-lim, lim, rows * cols))
        parts.append(np.zeros(rows))
    return np.concatenate(parts).astype(np.float32)


def training_pairs_rows(pairs: float = 1e7) -> int:
    """Smallest m with m (m - 1) / 2 >= pairs: the training points whose
    distinct pairs carry that many kernel values."""
    m = int(math.ceil((1 + math.sqrt(1 + 8 * pairs)) / 2))
    while m * (m - 1) // 2 < pairs:
        m += 1
    return m


def batch_indices(m: int, batch: int, steps: int, seed: int):
    """Training batches: `steps` rows of `batch` distinct indices in [0, m), int32."""
    rng = np.random.default_rng([int(seed), 0x62617463])  # tag "batc"
    return np.stack([rng.choice(m, batch, replace=False) for _ in range(steps)]).astype(np.int32)


def uniforms(count: int, seed: int):
    """Uniform draws in [0, 1) (k-means++ seeding), float64."""
    return np.random.default_rng([int(seed), 0x756E6966]).random(count)  # tag "unif"
