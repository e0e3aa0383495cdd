// One reassignment step for a set of independent clustering problems.
// Internal to the library.
#pragma once

#include "kkm_common.h"

namespace kkm {

// One clustering problem as the step kernels see it: its kernel matrix, its
// workspace (V in CSR form, partial sums) and where its outputs go.
struct Inst {
    int64_t n;          // points
    int32_t k;          // clusters
    int32_t empty_policy;
    int64_t L;          // CSR positions per sweep chunk
    int64_t nblk;       // 256-point label blocks
    int64_t ldp;        // row stride of the segment partials
    int64_t nstrip;     // sweep column strips (256 lanes x 16 bytes each)
    int64_t nws;        // 64-lane wave strips of columns
    const void *K;      // [n, ldk] FP32 or bfloat16
    int64_t ldk;
    const float *diag;  // [n]
    int64_t lab_off;    // first label of this problem in the label arrays
    // workspace
    int32_t *perm, *offsets, *counts, *blk_hist, *blk_bad, *err;
    float *P, *Zp, *ctilde;
    double *Jpart;
    // outputs of the step
    int32_t *counts_out;
    int64_t *n_changed;
    double *J_in;
    float *D_out, *ctilde_out;  // nullable
};

// A set of problems: `one` passed by value (table == nullptr), or a device
// table of up to `count` live problems whose label blocks / clusters / sweep
// items are laid end to end.  The prefix arrays have count + 1 entries; the
// entries past the last live problem all hold the live total, so a table can
// shrink between launches of a captured graph of fixed grid sizes.
struct InstSet {
    const Inst *table;
    const int64_t *blk_start, *cl_start, *item_start;
    int32_t count;
    Inst one;
};

struct InstGeom {
    int64_t n;
    int32_t k;
    int64_t L, nblk, nchunk, slots, ldp, nws_max;
};

// Reads of data that every lane of a workgroup takes from the same address and
// that no kernel of the step writes, through the constant address space, so
// they are scalar loads and the values stay in scalar registers.
template <typename T>
__device__ __forceinline__ T uniform_load(const T *p) {
#if defined(__HIP_DEVICE_COMPILE__)
    return *(const __attribute__((address_space(4))) T *)(p);
#else
    return *p;  // the host pass only parses device functions
#endif
}

__device__ __forceinline__ int32_t find_inst(const int64_t *start, int32_t count, int64_t g) {
    int32_t lo = 0, hi = count - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (uniform_load(start + mid) <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Geometry of a problem; L = 0 picks the default chunk length.
InstGeom inst_geometry(int64_t n, int32_t k, int64_t L);
size_t inst_workspace_bytes(const InstGeom &g);
// Carves a problem's workspace from `base` and fills its geometry and
// workspace fields in `in` (when non-null); `bytes` receives the size.
void inst_carve(void *base, const InstGeom &g, Inst *in, size_t *bytes);
int64_t inst_sweep_items(const InstGeom &g, int32_t k_store);
// Sets the strip counts that depend on the element type of K.
void inst_set_store(Inst *in, int32_t k_store);

// The seven kernels of one step over the whole set.  total_blocks,
// total_clusters and sweep_grid are grid sizes: label blocks, clusters and
// sweep items summed over every problem the set can hold; max_k sizes the
// dynamic LDS; vec: every K row is 16-byte aligned.
kkm_status step_launch(const InstSet &s, int64_t total_blocks, int64_t total_clusters,
                       int64_t sweep_grid, int32_t max_k, int32_t k_store, bool vec,
                       const int32_t *labels_in, int32_t *labels_out, hipStream_t stream);

// One step of a single problem with the sweep replaced by `sweep` (which must
// fill in.P and in.Zp as the stored-K sweep does), between the CSR build of V
// and the centroid norms.
kkm_status step_launch_custom(const Inst &in, const int32_t *labels_in, int32_t *labels_out,
                              const std::function<kkm_status(hipStream_t)> &sweep,
                              hipStream_t stream);

kkm_status vcsr_build(const int32_t *labels, int64_t n, int32_t k, int32_t *blk_hist,
                      int32_t *blk_bad, int32_t *err, int32_t *counts, int32_t *perm,
                      int32_t *offsets, int32_t *counts_out, int64_t *n_changed,
                      hipStream_t stream);

}  // namespace kkm
