"""ctypes binding of libkkm.so: argument marshalling only.

Every computation runs in the HIP library; this module checks tensor
devices/dtypes/shapes, passes raw device pointers and torch's current HIP
stream, and turns a non-zero status into an exception.  torch is imported
first so that the library binds to the HIP runtime torch already loaded.
"""
from __future__ import annotations

import ctypes
import os

import torch

LINEAR, POLY, GAUSS = 0, 1, 2
F32, BF16, FP8_ROWSCALED = 0, 1, 2
EMPTY_INF, EMPTY_ZERO_CENTROID = 0, 1
MAX_K = 1024

_STATUS = {0: "KKM_OK", -1: "KKM_ERR_ARG", -2: "KKM_ERR_LABEL", -3: "KKM_ERR_NOMEM",
           -4: "KKM_ERR_HIP", -5: "KKM_ERR_UNSUPPORTED", -6: "KKM_ERR_NONFINITE"}

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libkkm.so")

EXPORTS = ("kkm_gram", "kkm_gram_ex", "kkm_gram_workspace_bytes", "kkm_iterate", "kkm_iterate_workspace_bytes",
           "kkm_iterate_noalloc", "kkm_iterate_noalloc_max_bytes",
           "kkm_iterate_matfree", "kkm_iterate_matfree_workspace_bytes", "kkm_fit_matfree",
           "kkm_packed_elements", "kkm_gram_packed", "kkm_iterate_packed",
           "kkm_iterate_packed_workspace_bytes", "kkm_fit_packed",
           "kkm_fit", "kkm_fit_ex", "kkm_mlp_param_count", "kkm_mlp_forward",
           "kkm_mlp_forward_workspace_bytes", "kkm_mlp_loss_grad", "kkm_mlp_train_workspace_bytes",
           "kkm_mlp_adam", "kkm_mlp_train", "kkm_feature_lloyd", "kkm_feature_lloyd_workspace_bytes",
           "kkm_feature_kmeanspp", "kkm_feature_kmeanspp_workspace_bytes",
           "kkm_mlp_train_fresh", "kkm_mlp_train_fresh_workspace_bytes",
           "kkm_fit_batched", "kkm_fit_batched_workspace_bytes",
           "kkm_kernel_kmeanspp", "kkm_kernel_kmeanspp_workspace_bytes", "kkm_refine",
           "kkm_warm_start", "kkm_warm_start_workspace_bytes", "kkm_mlp_forward_layers",
           "kkm_timing_enable", "kkm_timing_read", "kkm_timing_spans", "kkm_last_error")


class KKMError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (_STATUS.get(status, status), message))
        self.status = status


_lib = None
_vp, _i64, _i32, _d, _sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t


class KkmInstance(ctypes.Structure):
    """The C struct kkm_instance (one problem of a batch)."""
    _fields_ = [("X", _vp), ("n", _i64), ("d", _i64), ("ldx", _i64), ("k", _i32),
                ("kernel_type", _i32), ("gamma", _d), ("coef0", _d), ("degree", _i32),
                ("chunk_rows", _i32)]


def lib():
    """Load libkkm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libkkm.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        L.kkm_last_error.restype = ctypes.c_char_p
        L.kkm_last_error.argtypes = []
        L.kkm_gram_workspace_bytes.restype = _sz
        L.kkm_gram_workspace_bytes.argtypes = [_i64, _i64, _i32]
        L.kkm_iterate_workspace_bytes.restype = _sz
        L.kkm_iterate_workspace_bytes.argtypes = [_i64, _i32]
        L.kkm_gram_ex.restype = ctypes.c_int
        L.kkm_gram_ex.argtypes = [_vp, _i64, _i64, _i64, _i32, _d, _d, _i32, _i32, _i32, _i32,
                                  _vp, _i64, _vp, _vp, _sz, _vp]
        L.kkm_gram.restype = ctypes.c_int
        L.kkm_gram.argtypes = [_vp, _i64, _i64, _i64, _i32, _d, _d, _i32, _i32, _i32, _vp, _i64,
                               _vp, _vp, _sz, _vp]
        L.kkm_iterate.restype = ctypes.c_int
        L.kkm_iterate.argtypes = [_vp, _i32, _i64, _vp, _i64, _i32, _vp, _i32, _vp, _vp, _vp, _vp,
                                  _vp, _vp, _vp, _sz, _vp]
        L.kkm_iterate_noalloc.restype = ctypes.c_int
        L.kkm_iterate_noalloc.argtypes = [_vp, _i32, _i64, _vp, _i64, _i32, _vp, _i32, _vp, _vp, _vp,
                                          _vp, _vp, _vp, _vp]
        L.kkm_iterate_noalloc_max_bytes.restype = _sz
        L.kkm_iterate_noalloc_max_bytes.argtypes = []
        L.kkm_iterate_matfree_workspace_bytes.restype = _sz
        L.kkm_iterate_matfree_workspace_bytes.argtypes = [_i64, _i64, _i32, _i32]
        L.kkm_iterate_matfree.restype = ctypes.c_int
        L.kkm_iterate_matfree.argtypes = [_vp, _i64, _i64, _i64, _i32, _d, _d, _i32, _i32, _i32, _vp,
                                          _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]
        L.kkm_fit_matfree.restype = ctypes.c_int
        L.kkm_fit_matfree.argtypes = [_vp, _i64, _i64, _i64, _i32, _i32, _d, _d, _i32, _i32, _i32,
                                      _vp, _i32, _i32, _vp, ctypes.POINTER(_d), ctypes.POINTER(_i32),
                                      _vp, _vp, _vp, _vp]
        L.kkm_packed_elements.restype = _sz
        L.kkm_packed_elements.argtypes = [_i64, _i32]
        L.kkm_iterate_packed_workspace_bytes.restype = _sz
        L.kkm_iterate_packed_workspace_bytes.argtypes = [_i64, _i32, _i32]
        L.kkm_gram_packed.restype = ctypes.c_int
        L.kkm_gram_packed.argtypes = [_vp, _i64, _i64, _i64, _i32, _d, _d, _i32, _i32, _i32, _vp, _vp,
                                      _vp, _sz, _vp]
        L.kkm_iterate_packed.restype = ctypes.c_int
        L.kkm_iterate_packed.argtypes = [_vp, _i32, _vp, _i64, _i32, _vp, _i32, _vp, _vp, _vp, _vp,
                                         _vp, _vp, _vp, _sz, _vp]
        L.kkm_fit_packed.restype = ctypes.c_int
        L.kkm_fit_packed.argtypes = [_vp, _i64, _i64, _i64, _i32, _i32, _d, _d, _i32, _i32, _i32,
                                     _i32, _vp, _i32, _i32, _vp, ctypes.POINTER(_d),
                                     ctypes.POINTER(_i32), _vp, _vp, _vp, _vp, _vp]
        L.kkm_fit.restype = ctypes.c_int
        L.kkm_fit.argtypes = [_vp, _i64, _i64, _i64, _i32, _i32, _d, _d, _i32, _vp, _i32, _i32,
                              _vp, ctypes.POINTER(_d), ctypes.POINTER(_i32), _vp, _i64, _vp]
        L.kkm_fit_ex.restype = ctypes.c_int
        L.kkm_fit_ex.argtypes = [_vp, _i64, _i64, _i64, _i32, _i32, _d, _d, _i32, _i32, _i32, _i32,
                                 _vp, _i32, _i32, _vp, ctypes.POINTER(_d), ctypes.POINTER(_i32),
                                 _vp, _i64, _vp, _vp, _vp, _vp]
        L.kkm_mlp_param_count.restype = _i64
        L.kkm_mlp_param_count.argtypes = [_i64, _i64, _i64, _i64]
        L.kkm_mlp_forward_workspace_bytes.restype = _sz
        L.kkm_mlp_forward_workspace_bytes.argtypes = [_i64, _i64, _i64, _i64, _i64]
        L.kkm_mlp_train_workspace_bytes.restype = _sz
        L.kkm_mlp_train_workspace_bytes.argtypes = [_i64, _i64, _i64, _i64, _i64]
        L.kkm_mlp_forward.restype = ctypes.c_int
        L.kkm_mlp_forward.argtypes = [_vp, _i64, _i64, _i64, _i64, _vp, _i64, _i64, _vp, _i64, _vp,
                                      _sz, _vp]
        L.kkm_mlp_forward_layers.restype = ctypes.c_int
        L.kkm_mlp_forward_layers.argtypes = [_vp, _i64, _i64, _i64, _i64, _vp, _i64, _i64, _vp, _vp,
                                             _vp, _i64, _vp]
        L.kkm_mlp_loss_grad.restype = ctypes.c_int
        L.kkm_mlp_loss_grad.argtypes = [_vp, _i64, _i64, _i64, _i64, _vp, _i64, _i64, _vp, _i64,
                                        _vp, _vp, _vp, _sz, _vp]
        L.kkm_mlp_adam.restype = ctypes.c_int
        L.kkm_mlp_adam.argtypes = [_vp, _vp, _vp, _vp, _i64, _i32, _d, _d, _d, _d, _vp]
        L.kkm_mlp_train.restype = ctypes.c_int
        L.kkm_mlp_train.argtypes = [_vp, _vp, _vp, _i64, _i64, _i64, _i64, _vp, _i64, _i64, _vp,
                                    _i64, _vp, _i64, _i32, _i32, _d, _d, _d, _d, _vp, _vp, _sz, _vp]
        L.kkm_mlp_train_fresh_workspace_bytes.restype = _sz
        L.kkm_mlp_train_fresh_workspace_bytes.argtypes = [_i64, _i64, _i64, _i64, _i64]
        L.kkm_mlp_train_fresh.restype = ctypes.c_int
        L.kkm_mlp_train_fresh.argtypes = [_vp, _vp, _vp, _i64, _i64, _i64, _i64, _vp, _i64, _i64,
                                          _i32, _i32, _i32, _d, _d, _i32, _d, _d, _d, _d, _vp, _vp,
                                          _sz, _vp]
        L.kkm_feature_lloyd_workspace_bytes.restype = _sz
        L.kkm_feature_lloyd_workspace_bytes.argtypes = [_i64, _i64, _i32]
        L.kkm_feature_lloyd.restype = ctypes.c_int
        L.kkm_feature_lloyd.argtypes = [_vp, _i64, _i64, _i64, _i32, _vp, _i32, _vp,
                                        ctypes.POINTER(_i32), _vp, ctypes.POINTER(_d), _vp, _sz,
                                        _vp]
        L.kkm_feature_kmeanspp_workspace_bytes.restype = _sz
        L.kkm_feature_kmeanspp_workspace_bytes.argtypes = [_i64, _i64, _i32]
        L.kkm_feature_kmeanspp.restype = ctypes.c_int
        L.kkm_feature_kmeanspp.argtypes = [_vp, _i64, _i64, _i64, _i32, _vp, _vp, _vp, _vp, _sz, _vp]
        L.kkm_refine.restype = ctypes.c_int
        L.kkm_refine.argtypes = [_vp, _i32, _i64, _vp, _i64, _i32, _i32, _vp, _i32, _i32, _vp,
                                 ctypes.POINTER(_d), ctypes.POINTER(_i32), _vp, _vp, _vp, _vp]
        L.kkm_kernel_kmeanspp_workspace_bytes.restype = _sz
        L.kkm_kernel_kmeanspp_workspace_bytes.argtypes = [_i64, _i32]
        L.kkm_kernel_kmeanspp.restype = ctypes.c_int
        L.kkm_kernel_kmeanspp.argtypes = [_vp, _i32, _i64, _vp, _i64, _i32, _vp, _vp, _vp, _vp,
                                          _sz, _vp]
        L.kkm_fit_batched_workspace_bytes.restype = _sz
        L.kkm_fit_batched_workspace_bytes.argtypes = [ctypes.POINTER(KkmInstance), _i32, _i32, _i32]
        L.kkm_fit_batched.restype = ctypes.c_int
        L.kkm_fit_batched.argtypes = [ctypes.POINTER(KkmInstance), _i32, _i32, _i32, _i32, _vp,
                                      _i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _sz, _vp]
        L.kkm_warm_start_workspace_bytes.restype = _sz
        L.kkm_warm_start_workspace_bytes.argtypes = [_i64, _i64, _i64, _i64, _i64, _i32, _i32]
        L.kkm_warm_start.restype = ctypes.c_int
        L.kkm_warm_start.argtypes = [_vp, _i64, _i64, _i64, _i64, _vp, _i64, _i64, _i32, _i32,
                                     _vp, _i32, _i32, _vp, ctypes.POINTER(_d),
                                     ctypes.POINTER(_i32), ctypes.POINTER(_i32), _vp, _sz, _vp]
        L.kkm_timing_enable.restype = ctypes.c_int
        L.kkm_timing_enable.argtypes = [_i32]
        L.kkm_timing_read.restype = ctypes.c_int
        L.kkm_timing_read.argtypes = [_vp, _vp]
        L.kkm_timing_spans.restype = ctypes.c_int
        L.kkm_timing_spans.argtypes = [_i32, _vp, _i64, ctypes.POINTER(_i64)]
        _lib = L
    return _lib


def _check(status: int):
    if status != 0:
        raise KKMError(status, lib().kkm_last_error().decode(errors="replace"))


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype, name, ndim=None):
    if t is None:
        return None
    if not (isinstance(t, torch.Tensor) and t.is_cuda):
        raise TypeError("%s must be a GPU tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if ndim is not None and t.dim() != ndim:
        raise ValueError("%s must have %d dims" % (name, ndim))
    return t


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _rows(t, name):
    """(rows, cols, leading dimension) of a row-major 2-D tensor view."""
    if t.stride(1) != 1:
        raise ValueError("%s must have unit column stride" % name)
    return t.shape[0], t.shape[1], t.stride(0)


def _kstore_dtype(k_store):
    return torch.bfloat16 if k_store == BF16 else torch.float32


def alloc_kernel_matrix(n: int, k_store: int = F32, device="cuda") -> torch.Tensor:
    """Uninitialised [n, n] view of a [n, ldk] buffer with ldk = n rounded up to
    128 (rows start 256-byte aligned in bfloat16 too: the Gram's stores measured
    faster so)."""
    ldk = (n + 127) // 128 * 128
    return torch.empty((n, ldk), dtype=_kstore_dtype(k_store), device=device)[:, :n]


def gram_workspace_bytes(n: int, d: int, gram_prec: int = F32) -> int:
    return int(lib().kkm_gram_workspace_bytes(n, d, gram_prec))


def iterate_workspace_bytes(n: int, k: int) -> int:
    return int(lib().kkm_iterate_workspace_bytes(n, k))


GRAM_TRIANGLE, GRAM_FULL, GRAM_TRIANGLE_128, GRAM_TRIANGLE_256 = 0, 1, 2, 3


def kkm_gram(X, kernel=GAUSS, gamma=1.0, coef0=0.0, degree=1, gram_prec=F32, k_store=F32,
             K=None, diagK=None, ws=None, shape=GRAM_TRIANGLE):
    """K = kappa(X X^T) and diag(K) on the GPU.  Returns (K, diagK).  shape:
    GRAM_TRIANGLE (upper-triangle 128 x 128 tiles, mirrored stores; also
    GRAM_TRIANGLE_128), GRAM_FULL (every tile), or GRAM_TRIANGLE_256 (the
    triangle in 256 x 256 tiles for a BF16 / FP8 product)."""
    _dev(X, torch.float32, "X", 2)
    n, d, ldx = _rows(X, "X")
    if K is None:
        K = alloc_kernel_matrix(n, k_store, X.device)
    _dev(K, _kstore_dtype(k_store), "K", 2)
    if tuple(K.shape) != (n, n):
        raise ValueError("K must be [n, n]")
    _, _, ldk = _rows(K, "K")
    if diagK is None:
        diagK = torch.empty(n, dtype=torch.float32, device=X.device)
    _dev(diagK, torch.float32, "diagK", 1)
    need = gram_workspace_bytes(n, d, gram_prec)
    if ws is None:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=X.device)
    _check(lib().kkm_gram_ex(_ptr(X), n, d, ldx, kernel, gamma, coef0, degree, gram_prec,
                             k_store, shape, _ptr(K), ldk, _ptr(diagK), _ptr(ws), ws.numel(),
                             _stream()))
    return K, diagK


def _iterate_outputs(K, diagK, labels_in, k, k_store, labels_out, counts_out, n_changed, J_in, D_out,
                     ctilde_out):
    """Checks the step's arguments and allocates the outputs not passed in."""
    if k_store is None:
        k_store = BF16 if K.dtype == torch.bfloat16 else F32
    _dev(K, _kstore_dtype(k_store), "K", 2)
    n, _, ldk = _rows(K, "K")
    _dev(diagK, torch.float32, "diagK", 1)
    _dev(labels_in, torch.int32, "labels_in", 1)
    dev = K.device
    if labels_out is None:
        labels_out = torch.empty(n, dtype=torch.int32, device=dev)
    if counts_out is None:
        counts_out = torch.empty(k, dtype=torch.int32, device=dev)
    if n_changed is None:
        n_changed = torch.empty(1, dtype=torch.int64, device=dev)
    if J_in is None:
        J_in = torch.empty(1, dtype=torch.float64, device=dev)
    if D_out is True:
        D_out = torch.empty((n, k), dtype=torch.float32, device=dev)
    if ctilde_out is True:
        ctilde_out = torch.empty(k, dtype=torch.float32, device=dev)
    for t, dt, nm in ((labels_out, torch.int32, "labels_out"), (counts_out, torch.int32, "counts_out"),
                      (n_changed, torch.int64, "n_changed"), (J_in, torch.float64, "J_in")):
        _dev(t, dt, nm)
    if D_out is not None:
        _dev(D_out, torch.float32, "D_out", 2)
        if not D_out.is_contiguous() or tuple(D_out.shape) != (n, k):
            raise ValueError("D_out must be contiguous [n, k]")
    if ctilde_out is not None:
        _dev(ctilde_out, torch.float32, "ctilde_out", 1)
    return k_store, n, ldk, labels_out, counts_out, n_changed, J_in, D_out, ctilde_out


def kkm_iterate(K, diagK, labels_in, k, empty_policy=EMPTY_INF, labels_out=None, counts_out=None,
                n_changed=None, J_in=None, D_out=None, ctilde_out=None, ws=None, k_store=None):
    """One reassignment step.  Returns (labels_out, counts_out, n_changed[1] int64, J_in[1] f64);
    D_out / ctilde_out are filled when passed (True allocates them)."""
    k_store, n, ldk, labels_out, counts_out, n_changed, J_in, D_out, ctilde_out = _iterate_outputs(
        K, diagK, labels_in, k, k_store, labels_out, counts_out, n_changed, J_in, D_out, ctilde_out)
    need = iterate_workspace_bytes(n, k)
    if ws is None:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=K.device)
    _check(lib().kkm_iterate(_ptr(K), k_store, ldk, _ptr(diagK), n, k, _ptr(labels_in),
                             empty_policy, _ptr(labels_out), _ptr(counts_out), _ptr(n_changed),
                             _ptr(J_in), _ptr(D_out), _ptr(ctilde_out), _ptr(ws), ws.numel(),
                             _stream()))
    return labels_out, counts_out, n_changed, J_in, D_out, ctilde_out


def kkm_iterate_noalloc(K, diagK, labels_in, k, empty_policy=EMPTY_INF, labels_out=None,
                        counts_out=None, n_changed=None, J_in=None, D_out=None, ctilde_out=None,
                        k_store=None):
    """kkm_iterate on the library's per-device scratch array (no workspace, no
    allocation inside the library; outputs not passed in are allocated here)."""
    k_store, n, ldk, labels_out, counts_out, n_changed, J_in, D_out, ctilde_out = _iterate_outputs(
        K, diagK, labels_in, k, k_store, labels_out, counts_out, n_changed, J_in, D_out, ctilde_out)
    _check(lib().kkm_iterate_noalloc(_ptr(K), k_store, ldk, _ptr(diagK), n, k, _ptr(labels_in),
                                     empty_policy, _ptr(labels_out), _ptr(counts_out),
                                     _ptr(n_changed), _ptr(J_in), _ptr(D_out), _ptr(ctilde_out),
                                     _stream()))
    return labels_out, counts_out, n_changed, J_in, D_out, ctilde_out


def iterate_noalloc_max_bytes() -> int:
    return int(lib().kkm_iterate_noalloc_max_bytes())


def kkm_fit(X, k, labels0, kernel=GAUSS, gamma=1.0, coef0=0.0, degree=1, max_iter=30,
            check_convergence=True, K_ws=None, labels_out=None):
    """The whole method on the GPU.  Returns (labels_out, objective, iters)."""
    r = kkm_fit_ex(X, k, labels0, kernel, gamma, coef0, degree, max_iter=max_iter,
                   check_convergence=check_convergence, K_ws=K_ws, labels_out=labels_out)
    return r["labels"], r["objective"], r["iters"]


def kkm_fit_ex(X, k, labels0, kernel=GAUSS, gamma=1.0, coef0=0.0, degree=1, gram_prec=F32,
               k_store=F32, empty_policy=EMPTY_INF, max_iter=30, check_convergence=True,
               K_ws=None, labels_out=None):
    """kkm_fit with precision forms and per-step records.  Returns a dict with
    labels, objective, iters, J_trace, changed_trace and times_ms (Gram, steps, final J)."""
    import numpy as np

    _dev(X, torch.float32, "X", 2)
    n, d, ldx = _rows(X, "X")
    _dev(labels0, torch.int32, "labels0", 1)
    if labels_out is None:
        labels_out = torch.empty(n, dtype=torch.int32, device=X.device)
    ldk = 0
    if K_ws is not None:
        _dev(K_ws, _kstore_dtype(k_store), "K_ws", 2)
        if K_ws.shape[0] != n or K_ws.shape[1] < n:
            raise ValueError("K_ws must have n rows and >= n columns")
        _, _, ldk = _rows(K_ws, "K_ws")
    J = _d()
    it = _i32()
    Jt = np.zeros(max_iter + 1, dtype=np.float64)
    Ct = np.zeros(max(max_iter, 1), dtype=np.int64)
    tm = np.zeros(3, dtype=np.float64)
    _check(lib().kkm_fit_ex(_ptr(X), n, d, ldx, k, kernel, gamma, coef0, degree, gram_prec,
                            k_store, empty_policy, _ptr(labels0), max_iter,
                            int(bool(check_convergence)), _ptr(labels_out), ctypes.byref(J),
                            ctypes.byref(it), _ptr(K_ws), ldk,
                            Jt.ctypes.data_as(_vp), Ct.ctypes.data_as(_vp), tm.ctypes.data_as(_vp),
                            _stream()))
    t = int(it.value)
    return dict(labels=labels_out, objective=J.value, iters=t, J_trace=Jt[:t + 1],
                changed_trace=Ct[:t], times_ms=tm)


def matfree_workspace_bytes(n: int, d: int, k: int, gram_prec: int = F32) -> int:
    return int(lib().kkm_iterate_matfree_workspace_bytes(n, d, k, gram_prec))


def kkm_iterate_matfree(X, labels_in, k, kernel=GAUSS, gamma=1.0, coef0=0.0, degree=1,
                        gram_prec=F32, empty_policy=EMPTY_INF, labels_out=None, counts_out=None,
                        n_changed=None, J_in=None, D_out=None, ctilde_out=None, diagK_out=None,
                        ws=None):
    """One reassignment step that recomputes the kernel values instead of
    reading a stored K.  Returns (labels_out, counts_out, n_changed, J_in,
    D_out, ctilde_out, diagK_out); D_out / ctilde_out / diagK_out are filled
    when passed (True allocates them)."""
    _dev(X, torch.float32, "X", 2)
    n, d, ldx = _rows(X, "X")
    _dev(labels_in, torch.int32, "labels_in", 1)
    dev = X.device
    if labels_out is None:
        labels_out = torch.empty(n, dtype=torch.int32, device=dev)
    if counts_out is None:
        counts_out = torch.empty(k, dtype=torch.int32, device=dev)
    if n_changed is None:
        n_changed = torch.empty(1, dtype=torch.int64, device=dev)
    if J_in is None:
        J_in = torch.empty(1, dtype=torch.float64, device=dev)
    if D_out is True:
        D_out = torch.empty((n, k), dtype=torch.float32, device=dev)
    if ctilde_out is True:
        ctilde_out = torch.empty(k, dtype=torch.float32, device=dev)
    if diagK_out is True:
        diagK_out = torch.empty(n, dtype=torch.float32, device=dev)
    for t, dt, nm in ((labels_out, torch.int32, "labels_out"), (counts_out, torch.int32, "counts_out"),
                      (n_changed, torch.int64, "n_changed"), (J_in, torch.float64, "J_in")):
        _dev(t, dt, nm)
    if D_out is not None:
        _dev(D_out, torch.float32, "D_out", 2)
        if not D_out.is_contiguous() or tuple(D_out.shape) != (n, k):
            raise ValueError("D_out must be contiguous [n, k]")
    if ctilde_out is not None:
        _dev(ctilde_out, torch.float32, "ctilde_out", 1)
    if diagK_out is not None:
        _dev(diagK_out, torch.float32, "diagK_out", 1)
    need = matfree_workspace_bytes(n, d, k, gram_prec)
    if ws is None:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    _check(lib().kkm_iterate_matfree(_ptr(X), n, d, ldx, kernel, gamma, coef0, degree, gram_prec, k,
                                     _ptr(labels_in), empty_policy, _ptr(labels_out),
                                     _ptr(counts_out), _ptr(n_changed), _ptr(J_in), _ptr(D_out),
                                     _ptr(ctilde_out), _ptr(diagK_out), _ptr(ws), ws.numel(),
                                     _stream()))
    return labels_out, counts_out, n_changed, J_in, D_out, ctilde_out, diagK_out


def kkm_fit_matfree(X, k, labels0, kernel=GAUSS, gamma=1.0, coef0=0.0, degree=1, gram_prec=F32,
                    empty_policy=EMPTY_INF, max_iter=30, check_convergence=True, labels_out=None):
    """The whole method with the matrix-free step (no n x n buffer).  Returns a
    dict with labels, objective, iters, J_trace, changed_trace and times_ms
    (prologue, steps, final J)."""
    import numpy as np

    _dev(X, torch.float32, "X", 2)
    n, d, ldx = _rows(X, "X")
    _dev(labels0, torch.int32, "labels0", 1)
    if labels_out is None:
        labels_out = torch.empty(n, dtype=torch.int32, device=X.device)
    J = _d()
    it = _i32()
    Jt = np.zeros(max_iter + 1, dtype=np.float64)
    Ct = np.zeros(max(max_iter, 1), dtype=np.int64)
    tm = np.zeros(3, dtype=np.float64)
    _check(lib().kkm_fit_matfree(_ptr(X), n, d, ldx, k, kernel, gamma, coef0, degree, gram_prec,
                                 empty_policy, _ptr(labels0), max_iter, int(bool(check_convergence)),
                                 _ptr(labels_out), ctypes.byref(J), ctypes.byref(it),
                                 Jt.ctypes.data_as(_vp), Ct.ctypes.data_as(_vp),
                                 tm.ctypes.data_as(_vp), _stream()))
    t = int(it.value)
    return dict(labels=labels_out, objective=J.value, iters=t, J_trace=Jt[:t + 1],
                changed_trace=Ct[:t], times_ms=tm)


def packed_elements(n: int, k_store: int = F32) -> int:
    return int(lib().kkm_packed_elements(n, k_store))


def alloc_packed_kernel_matrix(n: int, k_store=F32, device="cuda"):
    """A 1-d device buffer for the strip-packed upper triangle of K."""
    return torch.empty(packed_elements(n, k_store), dtype=_kstore_dtype(k_store), device=device)


def packed_workspace_bytes(n: int, k: int, k_store: int = F32) -> int:
    return int(lib().kkm_iterate_packed_workspace_bytes(n, k, k_store))


def kkm_gram_packed(X, kernel=GAUSS, gamma=1.0, coef0=0.0, degree=1, gram_prec=F32, k_store=F32,
                    K=None, diagK=None, ws=None):
    """K = kappa(X X^T) in the strip-packed upper layout, and diag(K).  Returns (K, diagK)."""
    _dev(X, torch.float32, "X", 2)
    n, d, ldx = _rows(X, "X")
    if K is None:
        K = alloc_packed_kernel_matrix(n, k_store, X.device)
    _dev(K, _kstore_dtype(k_store), "K", 1)
    if K.numel() < packed_elements(n, k_store):
        raise ValueError("K holds fewer than packed_elements(n) entries")
    if diagK is None:
        diagK = torch.empty(n, dtype=torch.float32, device=X.device)
    _dev(diagK, torch.float32, "diagK", 1)
    need = gram_workspace_bytes(n, d, gram_prec)
    if ws is None:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=X.device)
    _check(lib().kkm_gram_packed(_ptr(X), n, d, ldx, kernel, gamma, coef0, degree, gram_prec,
                                 k_store, _ptr(K), _ptr(diagK), _ptr(ws), ws.numel(), _stream()))
    return K, diagK


def kkm_iterate_packed(K, diagK, labels_in, k, empty_policy=EMPTY_INF, labels_out=None,
                       counts_out=None, n_changed=None, J_in=None, D_out=None, ctilde_out=None,
                       ws=None):
    """One reassignment step on a strip-packed K (1-d, float32 or bfloat16)."""
    k_store = BF16 if K.dtype == torch.bfloat16 else F32
    _dev(K, _kstore_dtype(k_store), "K", 1)
    _dev(diagK, torch.float32, "diagK", 1)
    n = diagK.shape[0]
    if K.numel() < packed_elements(n, k_store):
        raise ValueError("K holds fewer than packed_elements(n) entries")
    _dev(labels_in, torch.int32, "labels_in", 1)
    dev = K.device
    if labels_out is None:
        labels_out = torch.empty(n, dtype=torch.int32, device=dev)
    if counts_out is None:
        counts_out = torch.empty(k, dtype=torch.int32, device=dev)
    if n_changed is None:
        n_changed = torch.empty(1, dtype=torch.int64, device=dev)
    if J_in is None:
        J_in = torch.empty(1, dtype=torch.float64, device=dev)
    if D_out is True:
        D_out = torch.empty((n, k), dtype=torch.float32, device=dev)
    if ctilde_out is True:
        ctilde_out = torch.empty(k, dtype=torch.float32, device=dev)
    for t, dt, nm in ((labels_out, torch.int32, "labels_out"), (counts_out, torch.int32, "counts_out"),
                      (n_changed, torch.int64, "n_changed"), (J_in, torch.float64, "J_in")):
        _dev(t, dt, nm)
    if D_out is not None:
        _dev(D_out, torch.float32, "D_out", 2)
        if not D_out.is_contiguous() or tuple(D_out.shape) != (n, k):
            raise ValueError("D_out must be contiguous [n, k]")
    if ctilde_out is not None:
        _dev(ctilde_out, torch.float32, "ctilde_out", 1)
    need = packed_workspace_bytes(n, k, k_store)
    if ws is None:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    _check(lib().kkm_iterate_packed(_ptr(K), k_store, _ptr(diagK), n, k, _ptr(labels_in),
                                    empty_policy, _ptr(labels_out), _ptr(counts_out),
                                    _ptr(n_changed), _ptr(J_in), _ptr(D_out), _ptr(ctilde_out),
                                    _ptr(ws), ws.numel(), _stream()))
    return labels_out, counts_out, n_changed, J_in, D_out, ctilde_out


def kkm_fit_packed(X, k, labels0, kernel=GAUSS, gamma=1.0, coef0=0.0, degree=1, gram_prec=F32,
                   k_store=F32, empty_policy=EMPTY_INF, max_iter=30, check_convergence=True,
                   K_ws=None, labels_out=None):
    """kkm_fit_ex with K stored strip-packed (half the entries).  Returns a dict
    with labels, objective, iters, J_trace, changed_trace and times_ms (Gram,
    steps, final J)."""
    import numpy as np

    _dev(X, torch.float32, "X", 2)
    n, d, ldx = _rows(X, "X")
    _dev(labels0, torch.int32, "labels0", 1)
    if labels_out is None:
        labels_out = torch.empty(n, dtype=torch.int32, device=X.device)
    if K_ws is not None:
        _dev(K_ws, _kstore_dtype(k_store), "K_ws", 1)
        if K_ws.numel() < packed_elements(n, k_store):
            raise ValueError("K_ws holds fewer than packed_elements(n) entries")
    J = _d()
    it = _i32()
    Jt = np.zeros(max_iter + 1, dtype=np.float64)
    Ct = np.zeros(max(max_iter, 1), dtype=np.int64)
    tm = np.zeros(3, dtype=np.float64)
    _check(lib().kkm_fit_packed(_ptr(X), n, d, ldx, k, kernel, gamma, coef0, degree, gram_prec,
                                k_store, empty_policy, _ptr(labels0), max_iter,
                                int(bool(check_convergence)), _ptr(labels_out), ctypes.byref(J),
                                ctypes.byref(it), _ptr(K_ws), Jt.ctypes.data_as(_vp),
                                Ct.ctypes.data_as(_vp), tm.ctypes.data_as(_vp), _stream()))
    t = int(it.value)
    return dict(labels=labels_out, objective=J.value, iters=t, J_trace=Jt[:t + 1],
                changed_trace=Ct[:t], times_ms=tm)


def kkm_refine(K, diagK, k, labels0, empty_policy=EMPTY_INF, max_iter=30, check_convergence=True,
               labels_out=None):
    """The loop of kkm_fit_ex on a resident K (float32 or bfloat16) and its
    diagonal.  Returns a dict with labels, objective, iters, J_trace,
    changed_trace and times_ms (steps, final objective pass)."""
    import numpy as np
    if not (isinstance(K, torch.Tensor) and K.is_cuda and K.dim() == 2):
        raise TypeError("K must be a 2-d GPU tensor")
    k_store = BF16 if K.dtype == torch.bfloat16 else F32
    _dev(K, _kstore_dtype(k_store), "K", 2)
    n, _, ldk = _rows(K, "K")
    _dev(diagK, torch.float32, "diagK", 1)
    _dev(labels0, torch.int32, "labels0", 1)
    if labels_out is None:
        labels_out = torch.empty(n, dtype=torch.int32, device=K.device)
    J = _d()
    it = _i32()
    Jt = np.zeros(max_iter + 1, dtype=np.float64)
    Ct = np.zeros(max(max_iter, 1), dtype=np.int64)
    tm = np.zeros(2, dtype=np.float64)
    _check(lib().kkm_refine(_ptr(K), k_store, ldk, _ptr(diagK), n, k, empty_policy, _ptr(labels0),
                            max_iter, int(bool(check_convergence)), _ptr(labels_out),
                            ctypes.byref(J), ctypes.byref(it), Jt.ctypes.data_as(_vp),
                            Ct.ctypes.data_as(_vp), tm.ctypes.data_as(_vp), _stream()))
    t = int(it.value)
    return dict(labels=labels_out, objective=J.value, iters=t, J_trace=Jt[:t + 1],
                changed_trace=Ct[:t], times_ms=tm)


def kkm_kernel_kmeanspp(K, diagK, k, uniforms, seeds=None, labels_out=None, ws=None):
    """K-means++ seeds in the kernel's feature space from the kernel matrix K
    (float32 or bfloat16, as kkm_gram writes it) and its diagonal.
    Returns (seeds, labels_out): device int32 [k] and [n]."""
    import numpy as np
    if not (isinstance(K, torch.Tensor) and K.is_cuda and K.dim() == 2):
        raise TypeError("K must be a 2-d GPU tensor")
    k_store = BF16 if K.dtype == torch.bfloat16 else F32
    _dev(K, _kstore_dtype(k_store), "K", 2)
    n, _, ldk = _rows(K, "K")
    _dev(diagK, torch.float32, "diagK", 1)
    u = np.ascontiguousarray(uniforms, dtype=np.float64)
    if u.shape != (k,):
        raise ValueError("need k uniforms")
    if seeds is None:
        seeds = torch.empty(k, dtype=torch.int32, device=K.device)
    if labels_out is None:
        labels_out = torch.empty(n, dtype=torch.int32, device=K.device)
    need = int(lib().kkm_kernel_kmeanspp_workspace_bytes(n, k))
    if ws is None:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=K.device)
    _check(lib().kkm_kernel_kmeanspp(_ptr(K), k_store, ldk, _ptr(diagK), n, k,
                                     u.ctypes.data_as(_vp), _ptr(seeds), _ptr(labels_out),
                                     _ptr(ws), ws.numel(), _stream()))
    return seeds, labels_out


def _instances(problems):
    arr = (KkmInstance * len(problems))()
    for b, p in enumerate(problems):
        X = p["X"]
        _dev(X, torch.float32, "problems[%d].X" % b, 2)
        n, d, ldx = _rows(X, "problems[%d].X" % b)
        arr[b] = KkmInstance(X.data_ptr(), n, d, ldx, int(p["k"]), int(p.get("kernel", GAUSS)),
                             float(p.get("gamma", 1.0)), float(p.get("coef0", 0.0)),
                             int(p.get("degree", 1)), int(p.get("chunk_rows", 0)))
    return arr


def kkm_fit_batched_workspace_bytes(problems, gram_prec=F32, k_store=F32) -> int:
    arr = _instances(problems)
    return int(lib().kkm_fit_batched_workspace_bytes(arr, len(problems), gram_prec, k_store))


def kkm_fit_batched(problems, labels0, gram_prec=F32, k_store=F32, empty_policy=EMPTY_INF,
                    max_iter=30, check_convergence=True, use_graph=True, labels_out=None,
                    ws=None):
    """kkm_fit_ex for many problems in shared launches.

    problems: list of dicts with X (device float32 [n, d], row stride allowed),
    k, kernel, gamma, coef0, degree and optionally chunk_rows.  labels0: int32
    device vector of sum(n) labels, problem after problem.  Returns a dict with
    labels (same layout), objective (float64 [count]), iters (int32 [count])
    and times_ms (Gram, steps, final pass)."""
    import numpy as np

    arr = _instances(problems)
    count = len(problems)
    total = sum(int(a.n) for a in arr)
    _dev(labels0, torch.int32, "labels0", 1)
    if labels0.shape[0] != total:
        raise ValueError("labels0 must hold sum(n) = %d labels" % total)
    if labels_out is None:
        labels_out = torch.empty(total, dtype=torch.int32, device=labels0.device)
    ws_bytes = 0
    if ws is not None:
        _dev(ws, torch.uint8, "ws", 1)
        ws_bytes = ws.numel()
    obj = np.zeros(count, dtype=np.float64)
    its = np.zeros(count, dtype=np.int32)
    tm = np.zeros(3, dtype=np.float64)
    _check(lib().kkm_fit_batched(arr, count, gram_prec, k_store, empty_policy, _ptr(labels0),
                                 max_iter, int(bool(check_convergence)), int(bool(use_graph)),
                                 _ptr(labels_out), obj.ctypes.data_as(_vp), its.ctypes.data_as(_vp),
                                 tm.ctypes.data_as(_vp), _ptr(ws), ws_bytes, _stream()))
    return dict(labels=labels_out, objective=obj, iters=its, times_ms=tm)


def kkm_timing_enable(on: bool = True):
    """Start (clearing old records) or stop event timing of Gram / sweep / step launches."""
    _check(lib().kkm_timing_enable(int(bool(on))))


def kkm_timing_read():
    """{'gram'|'sweep'|'iterate'|'fold': (total_ms, launches)} since timing was enabled."""
    import numpy as np
    ms = np.zeros(4, dtype=np.float64)
    cnt = np.zeros(4, dtype=np.int64)
    _check(lib().kkm_timing_read(ms.ctypes.data_as(_vp), cnt.ctypes.data_as(_vp)))
    return {"gram": (float(ms[0]), int(cnt[0])), "sweep": (float(ms[1]), int(cnt[1])),
            "iterate": (float(ms[2]), int(cnt[2])), "fold": (float(ms[3]), int(cnt[3]))}


_TIMING_CLASS = {"gram": 0, "sweep": 1, "iterate": 2, "fold": 3}


def kkm_timing_spans(cls):
    """Durations in ms (numpy float64, launch order) of the recorded launches of
    class 'gram', 'sweep', 'iterate' or 'fold' since timing was enabled."""
    import numpy as np
    c = _TIMING_CLASS[cls]
    cnt = _i64()
    _check(lib().kkm_timing_spans(c, None, 0, ctypes.byref(cnt)))
    out = np.zeros(max(int(cnt.value), 1), dtype=np.float64)
    _check(lib().kkm_timing_spans(c, out.ctypes.data_as(_vp), out.size, ctypes.byref(cnt)))
    return out[:int(cnt.value)]


# ---------------------------------------------------------------- learned warm start

MLP_DIMS = dict(h1=512, h2=512, out=256)


def mlp_param_count(d, h1=512, h2=512, out=256) -> int:
    return int(lib().kkm_mlp_param_count(d, h1, h2, out))


def kkm_mlp_forward(params, X, h1=512, h2=512, out=256, F=None, ws=None):
    """F = phi_theta(X) on the GPU (params: FP32 device vector)."""
    _dev(params, torch.float32, "params", 1)
    _dev(X, torch.float32, "X", 2)
    n, d, ldx = _rows(X, "X")
    if params.numel() != mlp_param_count(d, h1, h2, out):
        raise ValueError("params has %d entries, expected %d" % (params.numel(),
                                                                 mlp_param_count(d, h1, h2, out)))
    if F is None:
        F = torch.empty((n, out), dtype=torch.float32, device=X.device)
    _dev(F, torch.float32, "F", 2)
    _, _, ldf = _rows(F, "F")
    need = int(lib().kkm_mlp_forward_workspace_bytes(n, d, h1, h2, out))
    if ws is None:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=X.device)
    _check(lib().kkm_mlp_forward(_ptr(params), d, h1, h2, out, _ptr(X), n, ldx, _ptr(F), ldf,
                                 _ptr(ws), ws.numel(), _stream()))
    return F


def kkm_mlp_forward_layers(params, X, h1=512, h2=512, out=256):
    """(H1, H2, F): every layer's output of phi_theta(X) on the GPU."""
    _dev(params, torch.float32, "params", 1)
    _dev(X, torch.float32, "X", 2)
    n, d, ldx = _rows(X, "X")
    if params.numel() != mlp_param_count(d, h1, h2, out):
        raise ValueError("params has %d entries, expected %d" % (params.numel(),
                                                                 mlp_param_count(d, h1, h2, out)))
    H1 = torch.empty((n, h1), dtype=torch.float32, device=X.device)
    H2 = torch.empty((n, h2), dtype=torch.float32, device=X.device)
    F = torch.empty((n, out), dtype=torch.float32, device=X.device)
    _check(lib().kkm_mlp_forward_layers(_ptr(params), d, h1, h2, out, _ptr(X), n, ldx, _ptr(H1),
                                        _ptr(H2), _ptr(F), out, _stream()))
    return H1, H2, F


def kkm_mlp_loss_grad(params, XB, KB, h1=512, h2=512, out=256, grad=None, ws=None):
    """(grad, loss[1] float64) of (1/B^2)||Phi Phi^T - KB||^2 for one batch."""
    _dev(params, torch.float32, "params", 1)
    _dev(XB, torch.float32, "XB", 2)
    _dev(KB, torch.float32, "KB", 2)
    B, d, ldx = _rows(XB, "XB")
    _, _, ldkb = _rows(KB, "KB")
    if grad is None:
        grad = torch.empty_like(params)
    loss = torch.empty(1, dtype=torch.float64, device=XB.device)
    need = int(lib().kkm_mlp_train_workspace_bytes(B, d, h1, h2, out))
    if ws is None:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=XB.device)
    _check(lib().kkm_mlp_loss_grad(_ptr(params), d, h1, h2, out, _ptr(XB), B, ldx, _ptr(KB), ldkb,
                                   _ptr(grad), _ptr(loss), _ptr(ws), ws.numel(), _stream()))
    return grad, loss


def kkm_mlp_adam(params, m, v, grad, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    _check(lib().kkm_mlp_adam(_ptr(params), _ptr(m), _ptr(v), _ptr(grad), params.numel(), t, lr,
                              beta1, beta2, eps, _stream()))


def kkm_mlp_train(params, m, v, Xtrain, Ktrain, batch_idx, t0=0, lr=1e-3, beta1=0.9,
                  beta2=0.999, eps=1e-8, h1=512, h2=512, out=256, ws=None):
    """Train for batch_idx.shape[0] steps (batch_idx: device int32 [steps, B]).
    Returns the per-step losses (device float64 [steps])."""
    _dev(Xtrain, torch.float32, "Xtrain", 2)
    _dev(Ktrain, torch.float32, "Ktrain", 2)
    _dev(batch_idx, torch.int32, "batch_idx", 2)
    mt, d, ldx = _rows(Xtrain, "Xtrain")
    _, _, ldk = _rows(Ktrain, "Ktrain")
    steps, B = batch_idx.shape
    if not batch_idx.is_contiguous():
        raise ValueError("batch_idx must be contiguous")
    losses = torch.empty(max(steps, 1), dtype=torch.float64, device=Xtrain.device)
    need = int(lib().kkm_mlp_train_workspace_bytes(B, d, h1, h2, out))
    if ws is None:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=Xtrain.device)
    _check(lib().kkm_mlp_train(_ptr(params), _ptr(m), _ptr(v), d, h1, h2, out, _ptr(Xtrain), mt,
                               ldx, _ptr(Ktrain), ldk, _ptr(batch_idx), B, steps, t0, lr, beta1,
                               beta2, eps, _ptr(losses), _ptr(ws), ws.numel(), _stream()))
    return losses[:steps]


def kkm_mlp_train_fresh(params, m, v, Xtrain, B, kernel=GAUSS, gamma=1.0, coef0=0.0, degree=1,
                        t0=0, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, h1=512, h2=512, out=256,
                        ws=None):
    """Train on consecutive batches of B rows of Xtrain (Xtrain.shape[0] // B steps),
    each batch's kernel values computed by the Gram kernel.  Returns the per-step
    losses (device float64)."""
    _dev(Xtrain, torch.float32, "Xtrain", 2)
    mt, d, ldx = _rows(Xtrain, "Xtrain")
    steps = mt // B
    losses = torch.empty(max(steps, 1), dtype=torch.float64, device=Xtrain.device)
    need = int(lib().kkm_mlp_train_fresh_workspace_bytes(B, d, h1, h2, out))
    if ws is None:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=Xtrain.device)
    _check(lib().kkm_mlp_train_fresh(_ptr(params), _ptr(m), _ptr(v), d, h1, h2, out, _ptr(Xtrain),
                                     ldx, B, steps, t0, kernel, gamma, coef0, degree, lr, beta1,
                                     beta2, eps, _ptr(losses), _ptr(ws), ws.numel(), _stream()))
    return losses[:steps]


def kkm_feature_lloyd(F, k, labels0, max_iter=100, labels_out=None, ws=None,
                      return_objective=False):
    """Lloyd on feature rows.  Returns (labels_out, iters, changed_trace), plus the
    feature-space objective of the last step when return_objective is set."""
    import numpy as np
    _dev(F, torch.float32, "F", 2)
    _dev(labels0, torch.int32, "labels0", 1)
    n, f, ldf = _rows(F, "F")
    if labels_out is None:
        labels_out = torch.empty(n, dtype=torch.int32, device=F.device)
    need = int(lib().kkm_feature_lloyd_workspace_bytes(n, f, k))
    if ws is None:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=F.device)
    it = _i32()
    obj = _d()
    tr = np.zeros(max(max_iter, 1), dtype=np.int64)
    _check(lib().kkm_feature_lloyd(_ptr(F), n, f, ldf, k, _ptr(labels0), max_iter, _ptr(labels_out),
                                   ctypes.byref(it), tr.ctypes.data_as(_vp), ctypes.byref(obj),
                                   _ptr(ws), ws.numel(), _stream()))
    if return_objective:
        return labels_out, int(it.value), tr[:int(it.value)], obj.value
    return labels_out, int(it.value), tr[:int(it.value)]


def kkm_feature_kmeanspp(F, k, uniforms, seeds=None, labels_out=None, ws=None):
    """K-means++ seeds on feature rows (uniforms: k host floats in [0,1)).
    Returns (seeds, labels_out): device int32 [k] and [n]."""
    import numpy as np
    _dev(F, torch.float32, "F", 2)
    n, f, ldf = _rows(F, "F")
    u = np.ascontiguousarray(uniforms, dtype=np.float64)
    if u.shape != (k,):
        raise ValueError("need k uniforms")
    if seeds is None:
        seeds = torch.empty(k, dtype=torch.int32, device=F.device)
    if labels_out is None:
        labels_out = torch.empty(n, dtype=torch.int32, device=F.device)
    need = int(lib().kkm_feature_kmeanspp_workspace_bytes(n, f, k))
    if ws is None:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=F.device)
    _check(lib().kkm_feature_kmeanspp(_ptr(F), n, f, ldf, k, u.ctypes.data_as(_vp), _ptr(seeds),
                                      _ptr(labels_out), _ptr(ws), ws.numel(), _stream()))
    return seeds, labels_out


def kkm_warm_start(params, X, k, uniforms, max_iter=60, streams=4, h1=512, h2=512, out=256,
                   labels_out=None, ws=None):
    """The learned warm start: phi_theta(X), len(uniforms) k-means++ seedings with
    Lloyd in feature space, the lowest feature-space objective kept.  uniforms:
    host float64 [restarts, k] in [0, 1).  Returns a dict with labels (device
    int32 [n]), objective, cheap_iters (summed over restarts) and best (restart)."""
    import numpy as np
    _dev(params, torch.float32, "params", 1)
    _dev(X, torch.float32, "X", 2)
    n, d, ldx = _rows(X, "X")
    if params.numel() != mlp_param_count(d, h1, h2, out):
        raise ValueError("params has %d entries, expected %d" % (params.numel(),
                                                                 mlp_param_count(d, h1, h2, out)))
    u = np.ascontiguousarray(uniforms, dtype=np.float64)
    if u.ndim != 2 or u.shape[1] != k:
        raise ValueError("uniforms must be [restarts, k]")
    if labels_out is None:
        labels_out = torch.empty(n, dtype=torch.int32, device=X.device)
    _dev(labels_out, torch.int32, "labels_out", 1)
    need = int(lib().kkm_warm_start_workspace_bytes(n, d, h1, h2, out, k, streams))
    if ws is None:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=X.device)
    obj, it, best = _d(), _i32(), _i32()
    _check(lib().kkm_warm_start(_ptr(params), d, h1, h2, out, _ptr(X), n, ldx, k, u.shape[0],
                                u.ctypes.data_as(_vp), max_iter, streams, _ptr(labels_out),
                                ctypes.byref(obj), ctypes.byref(it), ctypes.byref(best), _ptr(ws),
                                ws.numel(), _stream()))
    return dict(labels=labels_out, objective=obj.value, cheap_iters=int(it.value),
                best=int(best.value))
