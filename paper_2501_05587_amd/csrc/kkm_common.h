// Internal definitions shared by the library's translation units (not part of
// the C ABI).  Device helpers for gfx950 wave64 and the error plumbing.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>

#include "../../include/kkm.h"

namespace kkm {

constexpr int kWave = 64;

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// ---------------------------------------------------------------- errors

void set_error(const char *fmt, ...);
kkm_status hip_fail(hipError_t e, const char *what);

#define KKM_HIP(call)                                                  \
    do {                                                               \
        hipError_t e_ = (call);                                        \
        if (e_ != hipSuccess) return ::kkm::hip_fail(e_, #call);       \
    } while (0)

#define KKM_TRY(call)                                                  \
    do {                                                               \
        kkm_status s_ = (call);                                        \
        if (s_ != KKM_OK) return s_;                                   \
    } while (0)

// ---------------------------------------------------------------- launch timing
// When enabled (kkm_timing_enable), HIP events bracket the Gram and sweep
// launches on their stream; kkm_timing_read turns them into totals.

enum TimedKernel { TK_GRAM = 0, TK_SWEEP = 1, TK_ITERATE = 2, TK_FOLD = 3, TK_COUNT = 4 };

struct TimedSpan {
    hipEvent_t start = nullptr, stop = nullptr;
    int cls = -1;
};
TimedSpan timing_begin(int cls, hipStream_t stream);
void timing_end(const TimedSpan &span, hipStream_t stream);

// ---------------------------------------------------------------- argument checks

kkm_status check_kernel(int32_t kernel_type, double gamma, double coef0, int32_t degree);
kkm_status check_dtypes(int32_t gram_prec, int32_t k_store);
size_t elem_bytes(int32_t k_store);

// ---------------------------------------------------------------- shared launchers

// flag = 1 if any of v[0..n) is not finite, else 0 (clears flag first).
void flag_nonfinite(const float *v, int64_t n, int32_t *flag, hipStream_t stream);
// p[0..n) = v by a kernel (graph-safe, unlike a memset node).
void fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t stream);

size_t gram_workspace_bytes(int64_t n, int64_t d, int32_t gram_prec);
// shape: KKM_GRAM_TRIANGLE (upper-triangle tiles, mirrored stores) or
// KKM_GRAM_FULL (every tile, each storing its own block).  packed: K in the
// strip-packed upper layout (packed_row_offset; ldk unused), triangle only.
kkm_status gram_launch(const float *X, int64_t n, int64_t d, int64_t ldx, int32_t kernel,
                       double gamma, double coef0, int32_t degree, int32_t gram_prec,
                       int32_t k_store, void *K, int64_t ldk, float *diagK, void *ws,
                       size_t ws_bytes, hipStream_t stream, int32_t shape = KKM_GRAM_TRIANGLE,
                       bool packed = false);

// The loop of Algorithm 2 around a step function: steps from labels0 until
// no label changes (check_convergence != 0) or max_iter steps, then the
// objective of the final labels; synchronises `s` before returning.  `step`
// performs one reassignment step (labels in, labels out, cluster sizes,
// changed count and J of the input labels, all device pointers) on a
// workspace of step_ws bytes.  times_ms (host double[2], nullable): {all
// steps, final objective pass}.
using StepFn = std::function<kkm_status(const int32_t *labels_in, int32_t *labels_out,
                                        int32_t *counts, int64_t *n_changed, double *J_in,
                                        void *ws, size_t ws_bytes, hipStream_t s)>;
kkm_status run_steps(const StepFn &step, size_t step_ws, int64_t n, int32_t k,
                     const int32_t *labels0, int32_t max_iter, int32_t check_convergence,
                     int32_t *labels_out, double *objective, int32_t *iters, double *J_trace,
                     int64_t *changed_trace, double *times_ms, const char *who, hipStream_t s);

// ---------------------------------------------------------------- strip-packed symmetric K
// The upper triangle of K in strips of W columns (W a power of two): row i,
// in strip s_i = i / W, stores the columns [s_i W, ns W) of its row, so the
// diagonal W x W block of every strip is stored whole (both triangles) and
// every block above it once.  Rows follow each other; element (i, j) with
// j >= s_i W sits at packed_row_offset(i) + (j - s_i W).  ns W elements per
// row of strip 0, (ns - s) W per row of strip s: W^2 ns (ns + 1) / 2 in all.
__host__ __device__ inline int64_t packed_row_offset(int64_t i, int lgw, int64_t ns) {
    const int64_t W = int64_t(1) << lgw;
    const int64_t s = i >> lgw;
    return W * W * (s * ns - s * (s - 1) / 2) + (i - s * W) * (ns - s) * W;
}
inline int64_t packed_strips(int64_t n, int lgw) { return (n + (int64_t(1) << lgw) - 1) >> lgw; }
inline int64_t packed_elements(int64_t n, int lgw) {
    const int64_t W = int64_t(1) << lgw, ns = packed_strips(n, lgw);
    return W * W * ns * (ns + 1) / 2;
}
// Strip width of the packed layout: 1024 columns for K stored FP32 or bfloat16.
inline int packed_lgw(int32_t k_store) {
    (void)k_store;
    return 10;
}

// ---------------------------------------------------------------- workspace carving

struct Carver {
    char *base;
    size_t off = 0;
    explicit Carver(void *p) : base(static_cast<char *>(p)) {}
    template <typename T>
    T *take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
    size_t bytes() const { return (off + 255) & ~size_t(255); }
};

// ---------------------------------------------------------------- device helpers

// Error-free transformation of a sum (Knuth's TwoSum): s + e == a + b exactly.
__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e) {
    s = a + b;
    float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ __forceinline__ long long wave_sum(long long v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Compensated pair (sum, error) reduction across a wave: deterministic tree.
__device__ __forceinline__ void wave_sum2(float &s, float &c) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        float s2 = __shfl_xor(s, off, kWave);
        float c2 = __shfl_xor(c, off, kWave);
        float t, e;
        two_sum(s, s2, t, e);
        s = t;
        c = c + c2 + e;
    }
}

}  // namespace kkm
