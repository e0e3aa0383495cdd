"""FP64 CPU oracle for Kernel K-means.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline leg of the benchmark, never by the product path.  It shares no code
with the HIP library.  The arithmetic lives in ``kkm_oracle.c`` (plain C, FP64);
this module marshals numpy arrays into it and adds the adjusted Rand index
written from its definition.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np

from . import build as _build

LINEAR, POLY, GAUSS = 0, 1, 2
EMPTY_INF, EMPTY_ZERO_CENTROID = 0, 1

_lib = None

_f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_i64, _i32, _d, _int = ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_int


def _nullable(p):
    return ctypes.c_void_p


def lib():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = ctypes.CDLL(path)
        L.oracle_threads.restype = _int
        L.oracle_threads.argtypes = []
        L.oracle_set_threads.restype = None
        L.oracle_set_threads.argtypes = [_int]
        L.oracle_kappa.restype = _d
        L.oracle_kappa.argtypes = [_f32p, _f32p, _i64, _int, _d, _d, _int]
        L.oracle_kernel_matrix.restype = None
        L.oracle_kernel_matrix.argtypes = [_f32p, _i64, _i64, _i64, _int, _d, _d, _int, _f64p]
        L.oracle_kernel_rows.restype = None
        L.oracle_kernel_rows.argtypes = [_f32p, _i64, _i64, _i64, _int, _d, _d, _int,
                                         _i64p, _i64, _f64p]
        L.oracle_step.restype = _int
        L.oracle_step.argtypes = [_f64p, _i64, _i32, _i32p, _int, _i32p, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(_d),
                                  ctypes.POINTER(_d), ctypes.POINTER(_i64)]
        L.oracle_objective.restype = _int
        L.oracle_objective.argtypes = [_f64p, _i64, _i32, _i32p, _int, ctypes.POINTER(_d)]
        L.oracle_fit.restype = _int
        L.oracle_fit.argtypes = [_f64p, _i64, _i32, _i32p, _i32, _int, _int, _i32p,
                                 ctypes.POINTER(_d), ctypes.POINTER(_i32), ctypes.c_void_p,
                                 ctypes.c_void_p]
        L.oracle_cluster_row_sums.restype = _int
        L.oracle_cluster_row_sums.argtypes = [_f32p, _i64, _i64, _i64, _int, _d, _d, _int,
                                              _i32p, _i32, _i64p, _i64, _f64p]
        _lib = L
    return _lib


def threads() -> int:
    """Number of OpenMP threads the oracle's loops use."""
    return int(lib().oracle_threads())


def set_threads(t: int) -> None:
    """Threads of the oracle's following OpenMP loops (timing only)."""
    lib().oracle_set_threads(int(t))


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _x(X):
    X = np.ascontiguousarray(X, dtype=np.float32)
    assert X.ndim == 2
    return X


def kappa(x, y, kernel=GAUSS, gamma=1.0, coef0=0.0, degree=1) -> float:
    """kappa(x, y) from the definitions of Sec. 3.2 (FP64)."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    return lib().oracle_kappa(x, y, x.shape[0], kernel, gamma, coef0, degree)


def kernel_matrix(X, kernel=GAUSS, gamma=1.0, coef0=0.0, degree=1) -> np.ndarray:
    """K_ij = kappa(x_i, x_j), FP64 [n, n]."""
    X = _x(X)
    n, d = X.shape
    K = np.empty((n, n), dtype=np.float64)
    lib().oracle_kernel_matrix(X, n, d, d, kernel, gamma, coef0, degree, K)
    return K


def kernel_rows(X, rows, kernel=GAUSS, gamma=1.0, coef0=0.0, degree=1) -> np.ndarray:
    """kappa(x_r, x_j) for the selected rows r, FP64 [len(rows), n]."""
    X = _x(X)
    n, d = X.shape
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.empty((rows.shape[0], n), dtype=np.float64)
    lib().oracle_kernel_rows(X, n, d, d, kernel, gamma, coef0, degree, rows, rows.shape[0], out)
    return out


def step(K, k, labels_in, empty_policy=EMPTY_INF, want_D=True, want_gap=True):
    """One batch reassignment step from the definition of the feature-space
    distance.  Returns a dict with labels, D, gap, counts, J_in, A, n_changed."""
    K = np.ascontiguousarray(K, dtype=np.float64)
    n = K.shape[0]
    labels_in = np.ascontiguousarray(labels_in, dtype=np.int32)
    out = np.empty(n, dtype=np.int32)
    D = np.empty((n, k), dtype=np.float64) if want_D else None
    gap = np.empty(n, dtype=np.float64) if want_gap else None
    counts = np.empty(k, dtype=np.int32)
    J, A, ch = _d(), _d(), _i64()
    rc = lib().oracle_step(K, n, k, labels_in, empty_policy, out, _ptr(D), _ptr(gap),
                           _ptr(counts), ctypes.byref(J), ctypes.byref(A), ctypes.byref(ch))
    if rc != 0:
        raise ValueError("label outside [0, k)")
    return dict(labels=out, D=D, gap=gap, counts=counts, J_in=J.value, A=A.value,
                n_changed=int(ch.value))


def objective(K, k, labels, empty_policy=EMPTY_INF) -> float:
    K = np.ascontiguousarray(K, dtype=np.float64)
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    J = _d()
    if lib().oracle_objective(K, K.shape[0], k, labels, empty_policy, ctypes.byref(J)) != 0:
        raise ValueError("label outside [0, k)")
    return J.value


def fit(K, k, labels0, max_iter, check_convergence=True, empty_policy=EMPTY_INF):
    """The full loop.  Returns dict(labels, objective, iters, J_trace, changed_trace)."""
    K = np.ascontiguousarray(K, dtype=np.float64)
    n = K.shape[0]
    labels0 = np.ascontiguousarray(labels0, dtype=np.int32)
    out = np.empty(n, dtype=np.int32)
    Jt = np.zeros(max_iter + 1, dtype=np.float64)
    Ct = np.zeros(max(max_iter, 1), dtype=np.int64)
    J, it = _d(), _i32()
    rc = lib().oracle_fit(K, n, k, labels0, max_iter, int(bool(check_convergence)), empty_policy,
                          out, ctypes.byref(J), ctypes.byref(it), _ptr(Jt), _ptr(Ct))
    if rc != 0:
        raise ValueError("label outside [0, k)")
    t = int(it.value)
    return dict(labels=out, objective=J.value, iters=t, J_trace=Jt[:t + 1].copy(),
                changed_trace=Ct[:t].copy())


def trajectory(K, k, labels0, max_iter, check_convergence=True, empty_policy=EMPTY_INF):
    """Per-step records [(labels_in, step_result), ...] of the loop, for
    teacher-forced comparisons one step at a time."""
    cur = np.ascontiguousarray(labels0, dtype=np.int32)
    recs = []
    for _ in range(max_iter):
        r = step(K, k, cur, empty_policy)
        recs.append((cur, r))
        cur = r["labels"]
        if check_convergence and r["n_changed"] == 0:
            break
    return recs


def cluster_row_sums(X, labels, k, rows, kernel=GAUSS, gamma=1.0, coef0=0.0, degree=1):
    """sum_{j: a(j)=c} kappa(x_r, x_j) for selected rows r, FP64 [len(rows), k],
    without forming K (for checks at sizes where K does not fit the host)."""
    X = _x(X)
    n, d = X.shape
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.empty((rows.shape[0], k), dtype=np.float64)
    if lib().oracle_cluster_row_sums(X, n, d, d, kernel, gamma, coef0, degree, labels, k,
                                     rows, rows.shape[0], out) != 0:
        raise ValueError("label outside [0, k)")
    return out


def adjusted_rand_index(a, b) -> float:
    """Adjusted Rand index (Hubert and Arabie, 1985) from its definition:
    pair counts of the contingency table, corrected for chance."""
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    n = a.shape[0]
    if n < 2:
        return 1.0
    _, ai = np.unique(a, return_inverse=True)
    _, bi = np.unique(b, return_inverse=True)
    table = np.zeros((ai.max() + 1, bi.max() + 1), dtype=np.int64)
    np.add.at(table, (ai, bi), 1)

    def pairs(x):
        x = x.astype(np.float64)
        return float(np.sum(x * (x - 1.0) / 2.0))

    sum_ij = pairs(table)
    sum_a = pairs(table.sum(axis=1))
    sum_b = pairs(table.sum(axis=0))
    total = n * (n - 1) / 2.0
    expected = sum_a * sum_b / total
    max_index = 0.5 * (sum_a + sum_b)
    if max_index == expected:  # both labellings are a single cluster or all singletons
        return 1.0
    return (sum_ij - expected) / (max_index - expected)
