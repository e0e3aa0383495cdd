"""Kernel K-means on MI355X (gfx950): Gram matrix, SpMM row sweep, centroid
norms and fused distance/argmin, behind the C ABI of libkkm.so.

The functions below are a thin binding of that C ABI (see include/kkm.h);
torch supplies device memory and the HIP stream.  Nothing here falls back to
a CPU path: without the built library every call raises.
"""
from ._binding import (BF16, EMPTY_INF, EMPTY_ZERO_CENTROID, EXPORTS, F32, FP8_ROWSCALED, GAUSS,
                       LINEAR, MAX_K, POLY, KKMError, alloc_kernel_matrix, gram_workspace_bytes,
                       iterate_workspace_bytes, kkm_fit, kkm_fit_ex, kkm_gram, kkm_iterate,
                       kkm_iterate_noalloc, iterate_noalloc_max_bytes, kkm_iterate_matfree,
                       kkm_fit_matfree, matfree_workspace_bytes, kkm_gram_packed,
                       kkm_iterate_packed, kkm_fit_packed, packed_elements, alloc_packed_kernel_matrix,
                       packed_workspace_bytes,
                       kkm_timing_enable, kkm_timing_read, kkm_timing_spans, lib, mlp_param_count, kkm_mlp_forward,
                       kkm_mlp_loss_grad, kkm_mlp_adam, kkm_mlp_train, kkm_feature_lloyd,
                       kkm_feature_kmeanspp, kkm_mlp_train_fresh, kkm_fit_batched,
                       kkm_fit_batched_workspace_bytes, KkmInstance, kkm_kernel_kmeanspp, kkm_refine, kkm_warm_start, kkm_mlp_forward_layers,
                       GRAM_TRIANGLE, GRAM_FULL, GRAM_TRIANGLE_128, GRAM_TRIANGLE_256)

__all__ = ["kkm_gram", "kkm_iterate", "kkm_iterate_noalloc", "iterate_noalloc_max_bytes", "kkm_iterate_matfree",
           "kkm_fit_matfree", "matfree_workspace_bytes", "kkm_gram_packed",
           "kkm_iterate_packed", "kkm_fit_packed", "packed_elements", "alloc_packed_kernel_matrix",
           "packed_workspace_bytes", "kkm_fit", "kkm_fit_ex", "kkm_timing_enable",
           "kkm_timing_read", "kkm_timing_spans", "mlp_param_count", "kkm_mlp_forward", "kkm_mlp_loss_grad",
           "kkm_mlp_adam", "kkm_mlp_train", "kkm_feature_lloyd", "alloc_kernel_matrix",
           "gram_workspace_bytes", "iterate_workspace_bytes", "KKMError", "lib", "EXPORTS",
           "LINEAR", "POLY", "GAUSS", "F32", "BF16", "FP8_ROWSCALED", "EMPTY_INF",
           "EMPTY_ZERO_CENTROID", "MAX_K", "kkm_fit_batched", "kkm_fit_batched_workspace_bytes",
           "KkmInstance", "kkm_feature_kmeanspp", "kkm_mlp_train_fresh", "kkm_kernel_kmeanspp", "kkm_refine", "kkm_warm_start", "kkm_mlp_forward_layers",
           "GRAM_TRIANGLE", "GRAM_FULL", "GRAM_TRIANGLE_128", "GRAM_TRIANGLE_256"]
