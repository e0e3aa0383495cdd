"""Comparison rules between the HIP path and the FP64 oracle.

Tolerances (the paper fixes no precision; these follow the FP32 arithmetic):
* distances: |D_gpu - D_or| <= 1e-5 * sigma_i with the per-point condition
  scale sigma_i = |K_ii| + max_c (2 |E_ic| + |C_c|) (E = K V^T, C = centroid
  norms), the largest magnitude among the terms D_ic is built from;
* labels: equal, except at points whose oracle gap between the best and the
  second-best distance is below 1e-6 * sigma_i (FP32 cannot order them);
* objective: |J_gpu - J_or| <= 1e-5 * (sum_i |K_ii| + sum_c |c| |C_c|);
* integers (cluster sizes, changed count) exact given the labels.
"""
import numpy as np

D_TOL = 1e-5
GAP_TOL = 1e-6
J_TOL = 1e-5


def oracle_terms(K, k, labels, D_or):
    """E = K V^T and the centroid norms implied by the oracle's D, FP64."""
    n = K.shape[0]
    cnt = np.bincount(labels, minlength=k).astype(np.float64)
    V = np.zeros((k, n))
    for c in range(k):
        if cnt[c] > 0:
            V[c, labels == c] = 1.0 / cnt[c]
    E = K @ V.T
    diag = np.diag(K)
    C = np.zeros(k)
    for c in range(k):
        if cnt[c] > 0:
            C[c] = D_or[0, c] - diag[0] + 2.0 * E[0, c]
    return E, C, cnt


def sigma(K, E, C, cnt):
    live = cnt > 0
    t = 2.0 * np.abs(E[:, live]) + np.abs(C[live])[None, :]
    return np.abs(np.diag(K)) + (t.max(axis=1) if live.any() else 0.0)


def compare_step(K_or, k, labels_in, orc, D_gpu, labels_gpu, counts_gpu, n_changed_gpu, J_gpu,
                 ctilde_gpu=None, what=""):
    """Assert one teacher-forced step agrees.  Returns the number of near-tie
    points whose labels were allowed to differ."""
    D_or = orc["D"]
    E, C, cnt = oracle_terms(K_or, k, labels_in, D_or)
    sig = sigma(K_or, E, C, cnt)
    fin = np.isfinite(D_or)
    assert np.array_equal(np.isfinite(D_gpu), fin), what + ": infinite pattern differs"
    err = np.where(fin, np.abs(D_gpu.astype(np.float64) - np.where(fin, D_or, 0.0)), 0.0)
    worst = (err / sig[:, None]).max()
    assert worst <= D_TOL, "%s: distance error %.3g sigma > %.1g" % (what, worst, D_TOL)
    if ctilde_gpu is not None:
        live = cnt > 0
        cs = np.abs(np.diag(K_or)).max() + 2 * np.abs(E).max() + np.abs(C).max()
        cerr = np.abs(ctilde_gpu[live].astype(np.float64) - C[live]).max() / cs if live.any() else 0
        assert cerr <= D_TOL, "%s: centroid-norm error %.3g" % (what, cerr)
    near = orc["gap"] < GAP_TOL * sig
    bad = (labels_gpu != orc["labels"]) & ~near
    assert not bad.any(), "%s: %d labels differ away from ties (first %s)" % (
        what, int(bad.sum()), np.nonzero(bad)[0][:5])
    assert np.array_equal(counts_gpu, np.bincount(labels_gpu, minlength=k)), what + ": counts"
    assert n_changed_gpu == int((labels_gpu != labels_in).sum()), what + ": n_changed"
    jscale = np.abs(np.diag(K_or)).sum() + (cnt * np.abs(C)).sum()
    assert abs(J_gpu - orc["J_in"]) <= J_TOL * jscale, "%s: J %r vs %r" % (what, J_gpu, orc["J_in"])
    return int((labels_gpu != orc["labels"]).sum())


def gram_bound(X, kernel, gamma, coef0, degree, K_or, dot_rel=0.0):
    """Per-entry bound on |K_fp32 - K_exact| for an FP32 dot product of any
    summation order, pushed through the kernel function (first order), times 4.
    dot_rel adds a further relative error of the dot product (a matrix unit
    whose internal accumulation keeps fewer bits than FP32)."""
    u = 2.0 ** -24
    Xd = np.abs(X.astype(np.float64))
    d = X.shape[1]
    dot_abs = Xd @ Xd.T
    dot_err = ((d + 2) * u + dot_rel) * dot_abs
    if kernel == 0:
        b = dot_err
    elif kernel == 1:
        Xs = X.astype(np.float64)
        t = gamma * (Xs @ Xs.T) + coef0
        t_err = gamma * dot_err + u * (np.abs(t) + np.abs(coef0))
        b = degree * np.abs(t) ** max(degree - 1, 0) * t_err + (degree + 1) * u * np.abs(K_or)
    else:
        nr = (Xd * Xd).sum(axis=1)
        sq_err = (d + 4) * u * (nr[:, None] + nr[None, :] + 2 * dot_abs) + 2 * dot_rel * dot_abs
        b = np.abs(K_or) * (gamma * sq_err + 4 * u)
    return 4.0 * b + 1e-30


def gram_bound_pairs(X, I, J, kernel, gamma, coef0, degree, K_or, dot_rel=0.0):
    """gram_bound for selected entries (I[t], J[t]) only, K_or the exact values
    there: the same per-entry rule without forming the n x n matrices."""
    u = 2.0 ** -24
    Xd = np.abs(X.astype(np.float64))
    d = X.shape[1]
    dot_abs = (Xd[I] * Xd[J]).sum(axis=1)
    dot_err = ((d + 2) * u + dot_rel) * dot_abs
    if kernel == 0:
        b = dot_err
    elif kernel == 1:
        Xs = X.astype(np.float64)
        t = gamma * (Xs[I] * Xs[J]).sum(axis=1) + coef0
        t_err = gamma * dot_err + u * (np.abs(t) + np.abs(coef0))
        b = degree * np.abs(t) ** max(degree - 1, 0) * t_err + (degree + 1) * u * np.abs(K_or)
    else:
        nr = (Xd * Xd).sum(axis=1)
        sq_err = (d + 4) * u * (nr[I] + nr[J] + 2 * dot_abs) + 2 * dot_rel * dot_abs
        b = np.abs(K_or) * (gamma * sq_err + 4 * u)
    return 4.0 * b + 1e-30
