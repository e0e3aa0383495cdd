// The learned feature map phi_theta: R^d -> R^h1 -> R^h2 -> R^out (GELU after
// the first two layers, last layer linear), trained so that
// phi(x) . phi(y) approximates the kernel values kappa(x, y) the Gram kernel
// computes: loss (1/B^2) ||Phi Phi^T - K_B||_F^2 on batches of B points.
//
// Parameters: one FP32 master vector W1 [h1, d], b1 [h1], W2 [h2, h1], b2 [h2],
// W3 [out, h2], b3 [out] (row-major).  Matrix products take bfloat16 operands
// (weights and activations rounded to nearest even) with FP32 accumulation;
// the loss products (Phi Phi^T and its gradient) run in FP32.  Adam updates the
// FP32 master weights.
#include "gemm.h"

namespace kkm {

namespace {

struct Dims {
    int64_t d, h1, h2, out;
    int64_t oW1() const { return 0; }
    int64_t ob1() const { return h1 * d; }
    int64_t oW2() const { return ob1() + h1; }
    int64_t ob2() const { return oW2() + h2 * h1; }
    int64_t oW3() const { return ob2() + h2; }
    int64_t ob3() const { return oW3() + out * h2; }
    int64_t count() const { return ob3() + out; }
};

bool dims_ok(const Dims &m) { return m.d >= 1 && m.h1 >= 1 && m.h2 >= 1 && m.out >= 1; }

constexpr int64_t kFwdChunk = 32768;  // rows per forward pass through the workspace

GemmArgs gemm_args(const float *A, int64_t lda, const float *B, int64_t ldb, int64_t M, int64_t N,
                   int64_t K, float *C, int64_t ldc) {
    GemmArgs g{};
    g.A = A;
    g.lda = lda;
    g.B = B;
    g.ldb = ldb;
    g.M = M;
    g.N = N;
    g.K = K;
    g.alpha = 1.0f;
    g.C = C;
    g.ldc = ldc;
    return g;
}

// Forward of `rows` points: H1 = GELU(Z1), H2 = GELU(Z2), F = H2 W3^T + b3.
// Z1 / Z2 are stored only when non-null (training keeps them for GELU').
kkm_status forward_rows(const float *th, const Dims &m, const float *X, int64_t ldx, int64_t rows,
                        float *Z1, float *H1, float *Z2, float *H2, float *F, int64_t ldf,
                        hipStream_t s) {
    GemmArgs g = gemm_args(X, ldx, th + m.oW1(), m.d, rows, m.h1, m.d, Z1, m.h1);
    g.bias = th + m.ob1();
    g.C2 = H1;
    g.ldc2 = m.h1;
    KKM_TRY(gemm_launch(GEMM_BF16, true, true, EPI_BIAS_GELU, g, s));
    g = gemm_args(H1, m.h1, th + m.oW2(), m.h1, rows, m.h2, m.h1, Z2, m.h2);
    g.bias = th + m.ob2();
    g.C2 = H2;
    g.ldc2 = m.h2;
    KKM_TRY(gemm_launch(GEMM_BF16, true, true, EPI_BIAS_GELU, g, s));
    g = gemm_args(H2, m.h2, th + m.oW3(), m.h2, rows, m.out, m.h2, F, ldf);
    g.bias = th + m.ob3();
    return gemm_launch(GEMM_BF16, true, true, EPI_BIAS, g, s);
}

// Column sums of an [rows, cols] matrix (bias gradients), fixed order.
__global__ void column_sums(const float *A, int64_t rows, int64_t cols, int64_t lda, float *out) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    float s = 0.f;
    for (int64_t r = 0; r < rows; ++r) s += A[r * lda + c];
    out[c] = s;
}

__global__ void sum_partials(const double *part, int64_t np, double scale, double *out) {
    __shared__ double sh[256];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < np; i += 256) s += part[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0] * scale;
}

__global__ void gather_rows(const float *X, int64_t ldx, int64_t d, const int32_t *idx,
                            int64_t B, float *out) {
    const int64_t r = blockIdx.x;
    const int64_t src = idx[r];
    for (int64_t c = threadIdx.x; c < d; c += blockDim.x) out[r * d + c] = X[src * ldx + c];
}

__global__ void gather_block(const float *K, int64_t ldk, const int32_t *idx, int64_t B,
                             float *out) {
    const int64_t r = blockIdx.x;
    const int64_t src = idx[r];
    for (int64_t c = threadIdx.x; c < B; c += blockDim.x) out[r * B + c] = K[src * ldk + idx[c]];
}

// Adam (bias-corrected); omb1 = 1 - beta1 and omb2 = 1 - beta2 are formed in
// double on the host, c1 = 1 - beta1^t, c2 = 1 - beta2^t.
__global__ void adam_update(float *p, float *mo, float *ve, const float *g, int64_t n, float lr,
                            float b1, float b2, float omb1, float omb2, float eps, float c1,
                            float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float m = b1 * mo[i] + omb1 * gi;
    const float v = b2 * ve[i] + omb2 * gi * gi;
    mo[i] = m;
    ve[i] = v;
    p[i] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

__global__ void index_range_check(const int32_t *idx, int64_t count, int64_t m, int32_t *bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count && (idx[i] < 0 || idx[i] >= m)) atomicOr(bad, 1);
}

struct TrainWs {
    float *Z1, *H1, *Z2, *H2, *Phi, *G, *dPhi, *dZ2, *dZ1, *XB, *KB, *grad;
    double *part;
};

TrainWs carve_train(void *base, const Dims &m, int64_t B, size_t *bytes) {
    Carver c(base);
    TrainWs w;
    w.Z1 = c.take<float>((size_t)(B * m.h1));
    w.H1 = c.take<float>((size_t)(B * m.h1));
    w.Z2 = c.take<float>((size_t)(B * m.h2));
    w.H2 = c.take<float>((size_t)(B * m.h2));
    w.Phi = c.take<float>((size_t)(B * m.out));
    w.G = c.take<float>((size_t)(B * B));
    w.dPhi = c.take<float>((size_t)(B * m.out));
    w.dZ2 = c.take<float>((size_t)(B * m.h2));
    w.dZ1 = c.take<float>((size_t)(B * m.h1));
    w.XB = c.take<float>((size_t)(B * m.d));
    w.KB = c.take<float>((size_t)(B * B));
    w.grad = c.take<float>((size_t)m.count());
    w.part = c.take<double>((size_t)gemm_tiles(B, B));
    if (bytes) *bytes = c.bytes();
    return w;
}

// Loss and gradient for a batch already gathered into XB [B, ldx] / KB [B, ldkb].
kkm_status loss_grad(const float *th, const Dims &m, const float *XB, int64_t ldx,
                     const float *KB, int64_t ldkb, int64_t B, const TrainWs &w, float *grad,
                     double *loss, hipStream_t s) {
    KKM_TRY(forward_rows(th, m, XB, ldx, B, w.Z1, w.H1, w.Z2, w.H2, w.Phi, m.out, s));
    // G = Phi Phi^T - K_B and the sum of its squares
    GemmArgs g = gemm_args(w.Phi, m.out, w.Phi, m.out, B, B, m.out, w.G, B);
    g.Kb = KB;
    g.ldkb = ldkb;
    g.part = w.part;
    KKM_TRY(gemm_launch(GEMM_F32, true, true, EPI_LOSS, g, s));
    hipLaunchKernelGGL(sum_partials, dim3(1), dim3(256), 0, s, w.part, gemm_tiles(B, B),
                       1.0 / ((double)B * (double)B), loss);
    KKM_HIP(hipGetLastError());
    // dL/dPhi = (4/B^2) G Phi
    g = gemm_args(w.G, B, w.Phi, m.out, B, m.out, B, w.dPhi, m.out);
    g.alpha = (float)(4.0 / ((double)B * (double)B));
    KKM_TRY(gemm_launch(GEMM_F32, true, false, EPI_STORE, g, s));
    // layer 3: dW3 = dPhi^T H2, db3 = column sums, dZ2 = (dPhi W3) * GELU'(Z2)
    g = gemm_args(w.dPhi, m.out, w.H2, m.h2, m.out, m.h2, B, grad + m.oW3(), m.h2);
    KKM_TRY(gemm_launch(GEMM_BF16, false, false, EPI_STORE, g, s));
    hipLaunchKernelGGL(column_sums, dim3((unsigned)((m.out + 255) / 256)), dim3(256), 0, s, w.dPhi,
                       B, m.out, m.out, grad + m.ob3());
    g = gemm_args(w.dPhi, m.out, th + m.oW3(), m.h2, B, m.h2, m.out, w.dZ2, m.h2);
    g.Zp = w.Z2;
    g.ldz = m.h2;
    KKM_TRY(gemm_launch(GEMM_BF16, true, false, EPI_GELU_BWD, g, s));
    // layer 2
    g = gemm_args(w.dZ2, m.h2, w.H1, m.h1, m.h2, m.h1, B, grad + m.oW2(), m.h1);
    KKM_TRY(gemm_launch(GEMM_BF16, false, false, EPI_STORE, g, s));
    hipLaunchKernelGGL(column_sums, dim3((unsigned)((m.h2 + 255) / 256)), dim3(256), 0, s, w.dZ2,
                       B, m.h2, m.h2, grad + m.ob2());
    g = gemm_args(w.dZ2, m.h2, th + m.oW2(), m.h1, B, m.h1, m.h2, w.dZ1, m.h1);
    g.Zp = w.Z1;
    g.ldz = m.h1;
    KKM_TRY(gemm_launch(GEMM_BF16, true, false, EPI_GELU_BWD, g, s));
    // layer 1
    g = gemm_args(w.dZ1, m.h1, XB, ldx, m.h1, m.d, B, grad + m.oW1(), m.d);
    KKM_TRY(gemm_launch(GEMM_BF16, false, false, EPI_STORE, g, s));
    hipLaunchKernelGGL(column_sums, dim3((unsigned)((m.h1 + 255) / 256)), dim3(256), 0, s, w.dZ1,
                       B, m.h1, m.h1, grad + m.ob1());
    KKM_HIP(hipGetLastError());
    return KKM_OK;
}

kkm_status check_dims(const Dims &m) {
    if (!dims_ok(m)) {
        set_error("MLP dimensions must be positive (d=%lld h1=%lld h2=%lld out=%lld)",
                  (long long)m.d, (long long)m.h1, (long long)m.h2, (long long)m.out);
        return KKM_ERR_ARG;
    }
    return KKM_OK;
}

}  // namespace

}  // namespace kkm

using namespace kkm;

extern "C" int64_t kkm_mlp_param_count(int64_t d, int64_t h1, int64_t h2, int64_t out) {
    const Dims m{d, h1, h2, out};
    return dims_ok(m) ? m.count() : 0;
}

extern "C" size_t kkm_mlp_forward_workspace_bytes(int64_t n, int64_t d, int64_t h1, int64_t h2,
                                                  int64_t out) {
    (void)d;
    (void)out;
    const int64_t rows = n < kFwdChunk ? n : kFwdChunk;
    Carver c(nullptr);
    c.take<float>((size_t)(rows * h1));
    c.take<float>((size_t)(rows * h2));
    return c.bytes();
}

extern "C" kkm_status kkm_mlp_forward(const float *params, int64_t d, int64_t h1, int64_t h2,
                                      int64_t out, const float *X, int64_t n, int64_t ldx,
                                      float *F, int64_t ldf, void *ws, size_t ws_bytes,
                                      void *stream) {
    const Dims m{d, h1, h2, out};
    KKM_TRY(check_dims(m));
    if (n < 1 || ldx < d || ldf < out || !params || !X || !F) {
        set_error("kkm_mlp_forward: bad sizes or NULL pointer");
        return KKM_ERR_ARG;
    }
    const size_t need = kkm_mlp_forward_workspace_bytes(n, d, h1, h2, out);
    if (!ws || ws_bytes < need) {
        set_error("kkm_mlp_forward: workspace of %zu bytes is smaller than %zu", ws_bytes, need);
        return KKM_ERR_NOMEM;
    }
    hipStream_t s = (hipStream_t)stream;
    const int64_t rows = n < kFwdChunk ? n : kFwdChunk;
    Carver c(ws);
    float *H1 = c.take<float>((size_t)(rows * h1));
    float *H2 = c.take<float>((size_t)(rows * h2));
    for (int64_t r0 = 0; r0 < n; r0 += kFwdChunk) {
        const int64_t r = (n - r0) < kFwdChunk ? (n - r0) : kFwdChunk;
        KKM_TRY(forward_rows(params, m, X + r0 * ldx, ldx, r, nullptr, H1, nullptr, H2, F + r0 * ldf,
                             ldf, s));
    }
    return KKM_OK;
}

extern "C" kkm_status kkm_mlp_forward_layers(const float *params, int64_t d, int64_t h1,
                                             int64_t h2, int64_t out, const float *X, int64_t n,
                                             int64_t ldx, float *H1, float *H2, float *F,
                                             int64_t ldf, void *stream) {
    const Dims m{d, h1, h2, out};
    KKM_TRY(check_dims(m));
    if (n < 1 || ldx < d || ldf < out || !params || !X || !H1 || !H2 || !F) {
        set_error("kkm_mlp_forward_layers: bad sizes or NULL pointer");
        return KKM_ERR_ARG;
    }
    return forward_rows(params, m, X, ldx, n, nullptr, H1, nullptr, H2, F, ldf, (hipStream_t)stream);
}

extern "C" size_t kkm_mlp_train_workspace_bytes(int64_t B, int64_t d, int64_t h1, int64_t h2,
                                                int64_t out) {
    const Dims m{d, h1, h2, out};
    if (!dims_ok(m) || B < 1) return 0;
    size_t bytes = 0;
    carve_train(nullptr, m, B, &bytes);
    return bytes + 256;  // + index check flag
}

extern "C" kkm_status kkm_mlp_loss_grad(const float *params, int64_t d, int64_t h1, int64_t h2,
                                        int64_t out, const float *XB, int64_t B, int64_t ldx,
                                        const float *KB, int64_t ldkb, float *grad, double *loss,
                                        void *ws, size_t ws_bytes, void *stream) {
    const Dims m{d, h1, h2, out};
    KKM_TRY(check_dims(m));
    if (B < 1 || ldx < d || ldkb < B || !params || !XB || !KB || !grad || !loss) {
        set_error("kkm_mlp_loss_grad: bad sizes or NULL pointer");
        return KKM_ERR_ARG;
    }
    size_t need = 0;
    TrainWs w = carve_train(ws, m, B, &need);
    if (!ws || ws_bytes < need) {
        set_error("kkm_mlp_loss_grad: workspace of %zu bytes is smaller than %zu", ws_bytes, need);
        return KKM_ERR_NOMEM;
    }
    return loss_grad(params, m, XB, ldx, KB, ldkb, B, w, grad, loss, (hipStream_t)stream);
}

extern "C" kkm_status kkm_mlp_adam(float *params, float *adam_m, float *adam_v, const float *grad,
                                   int64_t count, int32_t t, double lr, double beta1,
                                   double beta2, double eps, void *stream) {
    if (count < 1 || t < 1 || !params || !adam_m || !adam_v || !grad || !(lr > 0) ||
        !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0)) {
        set_error("kkm_mlp_adam: bad arguments");
        return KKM_ERR_ARG;
    }
    const float c1 = (float)(1.0 - pow(beta1, (double)t));
    const float c2 = (float)(1.0 - pow(beta2, (double)t));
    hipLaunchKernelGGL(adam_update, dim3((unsigned)((count + 255) / 256)), dim3(256), 0,
                       (hipStream_t)stream, params, adam_m, adam_v, grad, count, (float)lr,
                       (float)beta1, (float)beta2, (float)(1.0 - beta1), (float)(1.0 - beta2),
                       (float)eps, c1, c2);
    KKM_HIP(hipGetLastError());
    return KKM_OK;
}

extern "C" kkm_status kkm_mlp_train(float *params, float *adam_m, float *adam_v, int64_t d,
                                    int64_t h1, int64_t h2, int64_t out, const float *Xtrain,
                                    int64_t mtrain, int64_t ldx, const float *Ktrain, int64_t ldk,
                                    const int32_t *batch_idx, int64_t B, int32_t steps,
                                    int32_t t0, double lr, double beta1, double beta2, double eps,
                                    double *loss_trace, void *ws, size_t ws_bytes,
                                    void *stream) {
    const Dims m{d, h1, h2, out};
    KKM_TRY(check_dims(m));
    if (B < 1 || steps < 0 || t0 < 0 || mtrain < 1 || ldx < d || ldk < mtrain || !params ||
        !adam_m || !adam_v || !Xtrain || !Ktrain || !batch_idx || !loss_trace) {
        set_error("kkm_mlp_train: bad sizes or NULL pointer");
        return KKM_ERR_ARG;
    }
    size_t need = 0;
    TrainWs w = carve_train(ws, m, B, &need);
    if (!ws || ws_bytes < need + 256) {
        set_error("kkm_mlp_train: workspace of %zu bytes is smaller than %zu", ws_bytes, need + 256);
        return KKM_ERR_NOMEM;
    }
    hipStream_t s = (hipStream_t)stream;
    int32_t *bad = reinterpret_cast<int32_t *>(static_cast<char *>(ws) + need);
    int32_t hbad = 0;
    KKM_HIP(hipMemcpyAsync(bad, &hbad, sizeof hbad, hipMemcpyHostToDevice, s));
    const int64_t nidx = (int64_t)steps * B;
    if (nidx > 0) {
        hipLaunchKernelGGL(index_range_check, dim3((unsigned)((nidx + 255) / 256)), dim3(256), 0, s,
                           batch_idx, nidx, mtrain, bad);
        KKM_HIP(hipGetLastError());
    }
    KKM_HIP(hipMemcpyAsync(&hbad, bad, sizeof hbad, hipMemcpyDeviceToHost, s));
    KKM_HIP(hipStreamSynchronize(s));
    if (hbad) {
        set_error("kkm_mlp_train: a batch index lies outside [0, %lld)", (long long)mtrain);
        return KKM_ERR_ARG;
    }
    for (int32_t st = 0; st < steps; ++st) {
        const int32_t *idx = batch_idx + (int64_t)st * B;
        hipLaunchKernelGGL(gather_rows, dim3((unsigned)B), dim3(256), 0, s, Xtrain, ldx, d, idx, B,
                           w.XB);
        hipLaunchKernelGGL(gather_block, dim3((unsigned)B), dim3(256), 0, s, Ktrain, ldk, idx, B,
                           w.KB);
        KKM_HIP(hipGetLastError());
        KKM_TRY(loss_grad(params, m, w.XB, d, w.KB, B, B, w, w.grad, loss_trace + st, s));
        KKM_TRY(kkm_mlp_adam(params, adam_m, adam_v, w.grad, m.count(), t0 + st + 1, lr, beta1,
                             beta2, eps, stream));
    }
    return KKM_OK;
}

extern "C" size_t kkm_mlp_train_fresh_workspace_bytes(int64_t B, int64_t d, int64_t h1,
                                                      int64_t h2, int64_t out) {
    const Dims m{d, h1, h2, out};
    if (!dims_ok(m) || B < 1) return 0;
    size_t bytes = 0;
    carve_train(nullptr, m, B, &bytes);
    return bytes + gram_workspace_bytes(B, d, KKM_F32);
}

extern "C" kkm_status kkm_mlp_train_fresh(float *params, float *adam_m, float *adam_v, int64_t d,
                                          int64_t h1, int64_t h2, int64_t out,
                                          const float *Xtrain, int64_t ldx, int64_t B,
                                          int32_t steps, int32_t t0, int32_t kernel_type,
                                          double gamma, double coef0, int32_t degree, double lr,
                                          double beta1, double beta2, double eps,
                                          double *loss_trace, void *ws, size_t ws_bytes,
                                          void *stream) {
    const Dims m{d, h1, h2, out};
    KKM_TRY(check_dims(m));
    if (B < 1 || steps < 0 || t0 < 0 || ldx < d || !params || !adam_m || !adam_v || !Xtrain ||
        !loss_trace) {
        set_error("kkm_mlp_train_fresh: bad sizes or NULL pointer");
        return KKM_ERR_ARG;
    }
    KKM_TRY(check_kernel(kernel_type, gamma, coef0, degree));
    size_t need = 0;
    TrainWs w = carve_train(ws, m, B, &need);
    const size_t gws = gram_workspace_bytes(B, d, KKM_F32);
    if (!ws || ws_bytes < need + gws) {
        set_error("kkm_mlp_train_fresh: workspace of %zu bytes is smaller than %zu", ws_bytes,
                  need + gws);
        return KKM_ERR_NOMEM;
    }
    void *gram_ws = static_cast<char *>(ws) + need;
    hipStream_t s = (hipStream_t)stream;
    for (int32_t st = 0; st < steps; ++st) {
        // step st trains on rows st*B .. st*B+B-1 and their kernel values, computed now
        const float *XB = Xtrain + (int64_t)st * B * ldx;
        KKM_TRY(gram_launch(XB, B, d, ldx, kernel_type, gamma, coef0, degree, KKM_F32, KKM_F32,
                            w.KB, B, w.Z1 /* diag(K), unused */, gram_ws, gws, s));
        KKM_TRY(loss_grad(params, m, XB, ldx, w.KB, B, B, w, w.grad, loss_trace + st, s));
        KKM_TRY(kkm_mlp_adam(params, adam_m, adam_v, w.grad, m.count(), t0 + st + 1, lr, beta1,
                             beta2, eps, stream));
    }
    return KKM_OK;
}
