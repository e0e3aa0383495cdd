// C-ABI entry points: argument checks, workspace handling and the iteration
// loop of the paper's Algorithm 2 around the gfx950 kernels.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "kkm_common.h"

namespace kkm {

static thread_local char g_err[512];

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

kkm_status hip_fail(hipError_t e, const char *what) {
    set_error("HIP error %d (%s) in %s", (int)e, hipGetErrorString(e), what);
    return (e == hipErrorOutOfMemory) ? KKM_ERR_NOMEM : KKM_ERR_HIP;
}

size_t iterate_workspace_bytes(int64_t n, int32_t k);
kkm_status iterate_launch(const void *K, int32_t k_store, int64_t ldk, const float *diagK,
                          int64_t n, int32_t k, const int32_t *labels_in, int32_t empty_policy,
                          int32_t *labels_out, int32_t *counts_out, int64_t *n_changed,
                          double *J_in, float *D_out, float *ctilde_out, void *ws,
                          size_t ws_bytes, hipStream_t stream);

// ---------------------------------------------------------------- launch timing

namespace {
struct TimingState {
    bool on = false;
    std::vector<TimedSpan> spans;           // recorded, not yet read
    std::vector<double> done[TK_COUNT];     // durations read, in launch order
};
TimingState &timing() {
    static TimingState st;
    return st;
}
std::mutex g_timing_mu;
}  // namespace

TimedSpan timing_begin(int cls, hipStream_t stream) {
    TimedSpan sp;
    std::lock_guard<std::mutex> g(g_timing_mu);
    if (!timing().on) return sp;
    // launches being captured into a graph run later: they are not timed
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone)
        return sp;
    if (hipEventCreate(&sp.start) != hipSuccess || hipEventCreate(&sp.stop) != hipSuccess) return sp;
    sp.cls = cls;
    (void)hipEventRecord(sp.start, stream);
    return sp;
}

void timing_end(const TimedSpan &sp, hipStream_t stream) {
    if (sp.cls < 0) return;
    (void)hipEventRecord(sp.stop, stream);
    std::lock_guard<std::mutex> g(g_timing_mu);
    timing().spans.push_back(sp);
}

kkm_status check_kernel(int32_t kernel_type, double gamma, double coef0, int32_t degree) {
    if (kernel_type != KKM_LINEAR && kernel_type != KKM_POLY && kernel_type != KKM_GAUSS) {
        set_error("unknown kernel type %d", kernel_type);
        return KKM_ERR_ARG;
    }
    if (!isfinite(gamma) || !isfinite(coef0)) {
        set_error("kernel parameters must be finite");
        return KKM_ERR_ARG;
    }
    if (kernel_type == KKM_GAUSS && !(gamma > 0.0)) {
        set_error("Gaussian kernel needs gamma > 0 (got %g)", gamma);
        return KKM_ERR_ARG;
    }
    if (kernel_type == KKM_POLY && (degree < 1 || degree > 64)) {
        set_error("polynomial degree must lie in [1, 64] (got %d)", degree);
        return KKM_ERR_ARG;
    }
    return KKM_OK;
}

kkm_status check_dtypes(int32_t gram_prec, int32_t k_store) {
    if (gram_prec < KKM_F32 || gram_prec > KKM_FP8_ROWSCALED || k_store < KKM_F32 ||
        k_store > KKM_BF16) {
        set_error("invalid precision pair gram_prec=%d k_store=%d", gram_prec, k_store);
        return KKM_ERR_ARG;
    }
    return KKM_OK;
}

size_t elem_bytes(int32_t k_store) { return k_store == KKM_BF16 ? 2 : 4; }

__global__ void flag_nonfinite_kernel(const float *v, int64_t n, int32_t *flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && !isfinite(v[i])) atomicOr(flag, 1);
}

__global__ void fill_i32_kernel(int32_t *p, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

void flag_nonfinite(const float *v, int64_t n, int32_t *flag, hipStream_t stream) {
    hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(1), 0, stream, flag, (int64_t)1, 0);
    if (n > 0)
        hipLaunchKernelGGL(flag_nonfinite_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                           stream, v, n, flag);
}

void fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t stream) {
    if (n > 0)
        hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream,
                           p, n, v);
}

namespace {

// Device buffers owned by one kkm_fit call.
struct FitBuffers {
    void *block = nullptr;
    void *K_own = nullptr;
    double *host = nullptr;
    ~FitBuffers() {
        if (block) (void)hipFree(block);
        if (K_own) (void)hipFree(K_own);
        if (host) (void)hipHostFree(host);
    }
};

}  // namespace
}  // namespace kkm

using namespace kkm;

extern "C" const char *kkm_last_error(void) { return g_err; }

namespace kkm {
namespace {
// Turns every recorded span into a duration (waits for its events).
kkm_status timing_drain(TimingState &st) {
    for (auto &sp : st.spans) {
        float ms = 0.f;
        KKM_HIP(hipEventSynchronize(sp.stop));
        KKM_HIP(hipEventElapsedTime(&ms, sp.start, sp.stop));
        st.done[sp.cls].push_back(ms);
        (void)hipEventDestroy(sp.start);
        (void)hipEventDestroy(sp.stop);
    }
    st.spans.clear();
    return KKM_OK;
}
}  // namespace
}  // namespace kkm

extern "C" kkm_status kkm_timing_enable(int32_t on) {
    std::lock_guard<std::mutex> g(g_timing_mu);
    TimingState &st = timing();
    for (auto &sp : st.spans) {
        (void)hipEventDestroy(sp.start);
        (void)hipEventDestroy(sp.stop);
    }
    st.spans.clear();
    for (int c = 0; c < TK_COUNT; ++c) st.done[c].clear();
    st.on = on != 0;
    return KKM_OK;
}

extern "C" kkm_status kkm_timing_read(double *total_ms, int64_t *launches) {
    if (!total_ms || !launches) {
        set_error("kkm_timing_read: NULL output");
        return KKM_ERR_ARG;
    }
    std::lock_guard<std::mutex> g(g_timing_mu);
    TimingState &st = timing();
    KKM_TRY(timing_drain(st));
    for (int c = 0; c < TK_COUNT; ++c) {
        double t = 0.0;
        for (double v : st.done[c]) t += v;
        total_ms[c] = t;
        launches[c] = (int64_t)st.done[c].size();
    }
    return KKM_OK;
}

extern "C" kkm_status kkm_timing_spans(int32_t cls, double *ms, int64_t cap, int64_t *count) {
    if (cls < 0 || cls >= TK_COUNT || !count || (cap > 0 && !ms) || cap < 0) {
        set_error("kkm_timing_spans: bad class, capacity or NULL output");
        return KKM_ERR_ARG;
    }
    std::lock_guard<std::mutex> g(g_timing_mu);
    TimingState &st = timing();
    KKM_TRY(timing_drain(st));
    const std::vector<double> &v = st.done[cls];
    *count = (int64_t)v.size();
    for (int64_t i = 0; i < cap && i < (int64_t)v.size(); ++i) ms[i] = v[(size_t)i];
    return KKM_OK;
}

extern "C" size_t kkm_gram_workspace_bytes(int64_t n, int64_t d, int32_t gram_prec) {
    if (n < 1 || d < 1) return 0;
    return gram_workspace_bytes(n, d, gram_prec);
}

extern "C" size_t kkm_iterate_workspace_bytes(int64_t n, int32_t k) {
    if (n < 1 || k < 1) return 0;
    return iterate_workspace_bytes(n, k);
}

extern "C" kkm_status kkm_gram_ex(const float *X, int64_t n, int64_t d, int64_t ldx,
                                  int32_t kernel_type, double gamma, double coef0,
                                  int32_t degree, int32_t gram_prec, int32_t k_store,
                                  int32_t shape, void *K, int64_t ldk, float *diagK, void *ws,
                                  size_t ws_bytes, void *stream) {
    g_err[0] = 0;
    if (n < 1 || d < 1 || ldx < d || ldk < n || !X || !K || !diagK) {
        set_error("kkm_gram: bad sizes or NULL pointer (n=%lld d=%lld ldx=%lld ldk=%lld)",
                  (long long)n, (long long)d, (long long)ldx, (long long)ldk);
        return KKM_ERR_ARG;
    }
    if (shape != KKM_GRAM_TRIANGLE && shape != KKM_GRAM_FULL && shape != KKM_GRAM_TRIANGLE_128 &&
        shape != KKM_GRAM_TRIANGLE_256) {
        set_error("kkm_gram: unknown shape %d", shape);
        return KKM_ERR_ARG;
    }
    KKM_TRY(check_kernel(kernel_type, gamma, coef0, degree));
    KKM_TRY(check_dtypes(gram_prec, k_store));
    return gram_launch(X, n, d, ldx, kernel_type, gamma, coef0, degree, gram_prec, k_store, K,
                       ldk, diagK, ws, ws_bytes, (hipStream_t)stream, shape);
}

extern "C" kkm_status kkm_gram(const float *X, int64_t n, int64_t d, int64_t ldx,
                               int32_t kernel_type, double gamma, double coef0, int32_t degree,
                               int32_t gram_prec, int32_t k_store, void *K, int64_t ldk,
                               float *diagK, void *ws, size_t ws_bytes, void *stream) {
    return kkm_gram_ex(X, n, d, ldx, kernel_type, gamma, coef0, degree, gram_prec, k_store,
                       KKM_GRAM_TRIANGLE, K, ldk, diagK, ws, ws_bytes, stream);
}

extern "C" kkm_status kkm_iterate(const void *K, int32_t k_store, int64_t ldk,
                                  const float *diagK, int64_t n, int32_t k,
                                  const int32_t *labels_in, int32_t empty_policy,
                                  int32_t *labels_out, int32_t *counts_out, int64_t *n_changed,
                                  double *J_in, float *D_out, float *ctilde_out, void *ws,
                                  size_t ws_bytes, void *stream) {
    g_err[0] = 0;
    if (n < 1 || k < 1 || k > n || ldk < n || !K || !diagK || !labels_in || !labels_out ||
        !counts_out || !n_changed || !J_in) {
        set_error("kkm_iterate: bad sizes or NULL pointer (n=%lld k=%d ldk=%lld)", (long long)n,
                  k, (long long)ldk);
        return KKM_ERR_ARG;
    }
    if (labels_in == labels_out) {
        set_error("kkm_iterate: labels_out must not alias labels_in");
        return KKM_ERR_ARG;
    }
    if (k > KKM_MAX_K) {
        set_error("kkm_iterate: k=%d exceeds KKM_MAX_K=%d", k, KKM_MAX_K);
        return KKM_ERR_UNSUPPORTED;
    }
    if (empty_policy != KKM_EMPTY_INF && empty_policy != KKM_EMPTY_ZERO_CENTROID) {
        set_error("kkm_iterate: unknown empty-cluster policy %d", empty_policy);
        return KKM_ERR_ARG;
    }
    if (k_store != KKM_F32 && k_store != KKM_BF16) {
        set_error("kkm_iterate: invalid k_store %d", k_store);
        return KKM_ERR_ARG;
    }
    return iterate_launch(K, k_store, ldk, diagK, n, k, labels_in, empty_policy, labels_out,
                          counts_out, n_changed, J_in, D_out, ctilde_out, ws, ws_bytes,
                          (hipStream_t)stream);
}

namespace kkm {
// The loop of Algorithm 2: steps from labels0 until no label changes
// (check_convergence) or max_iter steps, then the objective of the final
// labels (free when the last step changed nothing).  Each step is one call of
// `step` (labels in, labels out, sizes, changed count and J of the input
// labels, all device; a workspace of step_ws bytes).  times_ms (host
// double[2], nullable): {all steps, final objective pass}.
kkm_status run_steps(const StepFn &step, size_t step_ws, int64_t n, int32_t k,
                     const int32_t *labels0, int32_t max_iter, int32_t check_convergence,
                     int32_t *labels_out, double *objective, int32_t *iters, double *J_trace,
                     int64_t *changed_trace, double *times_ms, const char *who, hipStream_t s) {
    const int32_t steps_cap = max_iter + 1;
    const size_t iws = step_ws;
    FitBuffers fb;
    Carver c(nullptr);
    c.take<char>(iws);
    c.take<int32_t>((size_t)n);           // labels A
    c.take<int32_t>((size_t)n);           // labels B
    c.take<int32_t>((size_t)k);           // counts
    c.take<int64_t>((size_t)steps_cap);   // changed per step
    c.take<double>((size_t)steps_cap);    // J per step
    KKM_HIP(hipMalloc(&fb.block, c.bytes()));
    Carver w(fb.block);
    void *iter_ws = w.take<char>(iws);
    int32_t *lab[2] = {w.take<int32_t>((size_t)n), w.take<int32_t>((size_t)n)};
    int32_t *counts = w.take<int32_t>((size_t)k);
    int64_t *changed_dev = w.take<int64_t>((size_t)steps_cap);
    double *J_dev = w.take<double>((size_t)steps_cap);
    KKM_HIP(hipHostMalloc((void **)&fb.host, sizeof(double) * 4, hipHostMallocDefault));

    hipEvent_t ev[3];
    for (auto &e : ev) KKM_HIP(hipEventCreate(&e));
    struct EvGuard {
        hipEvent_t *e;
        ~EvGuard() {
            for (int i = 0; i < 3; ++i) (void)hipEventDestroy(e[i]);
        }
    } evg{ev};

    KKM_HIP(hipMemcpyAsync(lab[0], labels0, (size_t)n * sizeof(int32_t),
                           hipMemcpyDeviceToDevice, s));
    KKM_HIP(hipEventRecord(ev[0], s));
    int cur = 0;
    int32_t t = 0;
    int64_t last_changed = -1;
    int64_t *hchanged = reinterpret_cast<int64_t *>(fb.host + 1);
    for (; t < max_iter; ++t) {
        KKM_TRY(step(lab[cur], lab[cur ^ 1], counts, changed_dev + t, J_dev + t, iter_ws, iws, s));
        if (check_convergence || t == 0) {
            KKM_HIP(hipMemcpyAsync(hchanged, changed_dev + t, sizeof(int64_t),
                                   hipMemcpyDeviceToHost, s));
            KKM_HIP(hipStreamSynchronize(s));
            if (*hchanged < 0) {
                set_error("%s: a label of labels0 lies outside [0, %d)", who, k);
                return KKM_ERR_LABEL;
            }
        }
        cur ^= 1;
        if (check_convergence && *hchanged == 0) {
            last_changed = 0;
            ++t;
            break;
        }
    }
    KKM_HIP(hipEventRecord(ev[1], s));
    // objective of the final labels: free after a step that changed nothing
    const bool need_final = !(t > 0 && last_changed == 0);
    if (need_final)
        KKM_TRY(step(lab[cur], lab[cur ^ 1], counts, changed_dev + t, J_dev + t, iter_ws, iws, s));
    KKM_HIP(hipEventRecord(ev[2], s));
    KKM_HIP(hipMemcpyAsync(labels_out, lab[cur], (size_t)n * sizeof(int32_t),
                           hipMemcpyDeviceToDevice, s));
    KKM_HIP(hipStreamSynchronize(s));

    // per-step records
    int64_t *hc = new int64_t[(size_t)steps_cap];
    double *hj = new double[(size_t)steps_cap];
    hipError_t e1 = hipMemcpy(hc, changed_dev, sizeof(int64_t) * (size_t)(t + 1),
                              hipMemcpyDeviceToHost);
    hipError_t e2 = hipMemcpy(hj, J_dev, sizeof(double) * (size_t)(t + 1), hipMemcpyDeviceToHost);
    if (e1 != hipSuccess || e2 != hipSuccess) {
        delete[] hc;
        delete[] hj;
        return hip_fail(e1 != hipSuccess ? e1 : e2, "hipMemcpy(step records)");
    }
    if (!need_final) hj[t] = hj[t - 1];  // the no-change step's input labels are the final ones
    kkm_status st = KKM_OK;
    if (hc[need_final ? t : 0] < 0) {
        set_error("%s: a label of labels0 lies outside [0, %d)", who, k);
        st = KKM_ERR_LABEL;
    } else {
        *objective = hj[t];
        *iters = t;
        if (J_trace)
            for (int32_t u = 0; u <= t; ++u) J_trace[u] = hj[u];
        if (changed_trace)
            for (int32_t u = 0; u < t; ++u) changed_trace[u] = hc[u];
        if (times_ms) {
            float a = 0.f, b = 0.f;
            (void)hipEventElapsedTime(&a, ev[0], ev[1]);
            (void)hipEventElapsedTime(&b, ev[1], ev[2]);
            times_ms[0] = a;
            times_ms[1] = b;
        }
    }
    delete[] hc;
    delete[] hj;
    return st;
}

namespace {

// run_steps with the stored-K step (kkm_iterate's kernels).
kkm_status run_loop(const void *K, int32_t k_store, int64_t ldk, const float *diag, int64_t n,
                    int32_t k, int32_t empty_policy, const int32_t *labels0, int32_t max_iter,
                    int32_t check_convergence, int32_t *labels_out, double *objective,
                    int32_t *iters, double *J_trace, int64_t *changed_trace, double *times_ms,
                    const char *who, hipStream_t s) {
    const StepFn step = [&](const int32_t *in, int32_t *out, int32_t *counts, int64_t *changed,
                            double *J, void *ws, size_t ws_bytes, hipStream_t st) {
        return iterate_launch(K, k_store, ldk, diag, n, k, in, empty_policy, out, counts, changed,
                              J, nullptr, nullptr, ws, ws_bytes, st);
    };
    return run_steps(step, iterate_workspace_bytes(n, k), n, k, labels0, max_iter,
                     check_convergence, labels_out, objective, iters, J_trace, changed_trace,
                     times_ms, who, s);
}

}  // namespace
}  // namespace kkm

extern "C" kkm_status kkm_fit_ex(const float *X, int64_t n, int64_t d, int64_t ldx, int32_t k,
                                 int32_t kernel_type, double gamma, double coef0,
                                 int32_t degree, int32_t gram_prec, int32_t k_store,
                                 int32_t empty_policy, const int32_t *labels0, int32_t max_iter,
                                 int32_t check_convergence, int32_t *labels_out,
                                 double *objective, int32_t *iters, void *K_ws, int64_t ldk,
                                 double *J_trace, int64_t *changed_trace, double *times_ms,
                                 void *stream) {
    g_err[0] = 0;
    if (n < 1 || d < 1 || ldx < d || k < 1 || k > n || max_iter < 0 || !X || !labels0 ||
        !labels_out || !objective || !iters) {
        set_error("kkm_fit: bad sizes or NULL pointer (n=%lld d=%lld k=%d max_iter=%d)",
                  (long long)n, (long long)d, k, max_iter);
        return KKM_ERR_ARG;
    }
    if (k > KKM_MAX_K) {
        set_error("kkm_fit: k=%d exceeds KKM_MAX_K=%d", k, KKM_MAX_K);
        return KKM_ERR_UNSUPPORTED;
    }
    if (K_ws && ldk < n) {
        set_error("kkm_fit: ldk=%lld < n=%lld", (long long)ldk, (long long)n);
        return KKM_ERR_ARG;
    }
    if (empty_policy != KKM_EMPTY_INF && empty_policy != KKM_EMPTY_ZERO_CENTROID) {
        set_error("kkm_fit: unknown empty-cluster policy %d", empty_policy);
        return KKM_ERR_ARG;
    }
    KKM_TRY(check_kernel(kernel_type, gamma, coef0, degree));
    KKM_TRY(check_dtypes(gram_prec, k_store));
    hipStream_t s = (hipStream_t)stream;

    FitBuffers fb;
    void *K = K_ws;
    if (!K) {
        ldk = (n + 127) & ~int64_t(127);  // rows 256-byte aligned in bfloat16 too
        const size_t kbytes = (size_t)n * (size_t)ldk * elem_bytes(k_store);
        hipError_t e = hipMalloc(&fb.K_own, kbytes);
        if (e != hipSuccess) {
            set_error("kkm_fit: cannot allocate %zu bytes for K (%s)", kbytes,
                      hipGetErrorString(e));
            return KKM_ERR_NOMEM;
        }
        K = fb.K_own;
    }
    const size_t gws = gram_workspace_bytes(n, d, gram_prec);
    Carver c(nullptr);
    c.take<char>(gws);
    c.take<float>((size_t)n);   // diag
    c.take<int32_t>(1);         // non-finite flag
    KKM_HIP(hipMalloc(&fb.block, c.bytes()));
    Carver w(fb.block);
    void *gram_ws = w.take<char>(gws);
    float *diag = w.take<float>((size_t)n);
    int32_t *flag = w.take<int32_t>(1);
    KKM_HIP(hipHostMalloc((void **)&fb.host, sizeof(double) * 2, hipHostMallocDefault));

    hipEvent_t ev[2];
    for (auto &e : ev) KKM_HIP(hipEventCreate(&e));
    struct EvGuard {
        hipEvent_t *e;
        ~EvGuard() {
            for (int i = 0; i < 2; ++i) (void)hipEventDestroy(e[i]);
        }
    } evg{ev};

    KKM_HIP(hipEventRecord(ev[0], s));
    KKM_TRY(gram_launch(X, n, d, ldx, kernel_type, gamma, coef0, degree, gram_prec, k_store, K,
                        ldk, diag, gram_ws, gws, s));
    flag_nonfinite(diag, n, flag, s);
    KKM_HIP(hipGetLastError());
    KKM_HIP(hipEventRecord(ev[1], s));
    int32_t *hflag = reinterpret_cast<int32_t *>(fb.host);
    KKM_HIP(hipMemcpyAsync(hflag, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    KKM_HIP(hipStreamSynchronize(s));
    if (*hflag != 0) {
        set_error("kkm_fit: diag(K) has a non-finite entry (NaN or infinity in X?)");
        return KKM_ERR_NONFINITE;
    }
    double loop_ms[2] = {0.0, 0.0};
    KKM_TRY(run_loop(K, k_store, ldk, diag, n, k, empty_policy, labels0, max_iter,
                     check_convergence, labels_out, objective, iters, J_trace, changed_trace,
                     loop_ms, "kkm_fit", s));
    if (times_ms) {
        float a = 0.f;
        (void)hipEventElapsedTime(&a, ev[0], ev[1]);
        times_ms[0] = a;
        times_ms[1] = loop_ms[0];
        times_ms[2] = loop_ms[1];
    }
    return KKM_OK;
}

extern "C" kkm_status kkm_refine(const void *K, int32_t k_store, int64_t ldk, const float *diagK,
                                 int64_t n, int32_t k, int32_t empty_policy,
                                 const int32_t *labels0, int32_t max_iter,
                                 int32_t check_convergence, int32_t *labels_out,
                                 double *objective, int32_t *iters, double *J_trace,
                                 int64_t *changed_trace, double *times_ms, void *stream) {
    g_err[0] = 0;
    if (n < 1 || k < 1 || k > n || ldk < n || max_iter < 0 || !K || !diagK || !labels0 ||
        !labels_out || !objective || !iters) {
        set_error("kkm_refine: bad sizes or NULL pointer (n=%lld k=%d ldk=%lld max_iter=%d)",
                  (long long)n, k, (long long)ldk, max_iter);
        return KKM_ERR_ARG;
    }
    if (k > KKM_MAX_K) {
        set_error("kkm_refine: k=%d exceeds KKM_MAX_K=%d", k, KKM_MAX_K);
        return KKM_ERR_UNSUPPORTED;
    }
    if (k_store != KKM_F32 && k_store != KKM_BF16) {
        set_error("kkm_refine: K must be stored as KKM_F32 or KKM_BF16");
        return KKM_ERR_ARG;
    }
    if (empty_policy != KKM_EMPTY_INF && empty_policy != KKM_EMPTY_ZERO_CENTROID) {
        set_error("kkm_refine: unknown empty-cluster policy %d", empty_policy);
        return KKM_ERR_ARG;
    }
    return run_loop(K, k_store, ldk, diagK, n, k, empty_policy, labels0, max_iter,
                    check_convergence, labels_out, objective, iters, J_trace, changed_trace,
                    times_ms, "kkm_refine", (hipStream_t)stream);
}

extern "C" kkm_status kkm_fit(const float *X, int64_t n, int64_t d, int64_t ldx, int32_t k,
                              int32_t kernel_type, double gamma, double coef0, int32_t degree,
                              const int32_t *labels0, int32_t max_iter,
                              int32_t check_convergence, int32_t *labels_out, double *objective,
                              int32_t *iters, void *K_ws, int64_t ldk, void *stream) {
    return kkm_fit_ex(X, n, d, ldx, k, kernel_type, gamma, coef0, degree, KKM_F32, KKM_F32,
                      KKM_EMPTY_INF, labels0, max_iter, check_convergence, labels_out, objective,
                      iters, K_ws, ldk, nullptr, nullptr, nullptr, stream);
}
