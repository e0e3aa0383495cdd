/*
 * kkm.h — C ABI of the MI355X (gfx950) Kernel K-means library, libkkm.so.
 *
 * The method (paper: "Popcorn: Accelerating Kernel K-means on GPUs through
 * Sparse Linear Algebra", PPoPP'25):
 *
 *   K = kappa(P P^T) once (Sec. 3.2, Algorithm 2 first step), then per
 *   iteration (Algorithm 2 loop body, Eq. dist_sp_1 and Eq. cnorms_gemv)
 *     E = K V^T                 SpMM with the k x n selection matrix V
 *                               (Eq. v_init: V_ci = 1/|c| if a(i) = c)
 *     ||c_c||^2 = (V z)_c       SpMV with z_i = E_{i,a(i)}
 *     D_ic = K_ii - 2 E_ic + ||c_c||^2
 *     a'(i) = argmin_c D_ic
 *   until no label changes or maxiter steps ran (Algorithm 1).
 *
 * Conventions for every entry point
 *  - Array arguments are DEVICE pointers owned by the caller unless a comment
 *    says "host".  Matrices are row-major with an explicit leading dimension
 *    (in elements).  The library never frees caller memory.
 *  - `stream` is a hipStream_t (NULL = the default stream).  kkm_gram and
 *    kkm_iterate only enqueue work on it and return at once; their scalar
 *    results are written to device memory.  kkm_fit and kkm_fit_ex
 *    synchronise the stream before returning.
 *  - Calls return a kkm_status and never abort or throw.  On an error the
 *    outputs are unspecified and kkm_last_error() describes the cause
 *    (thread-local, valid until the next call on the same thread).
 *  - Labels are int32 cluster indices in [0, k).
 *  - Kernel functions (Sec. 3.2; sigma of the Gaussian is folded into gamma):
 *      KKM_LINEAR  kappa(x,y) = x.y
 *      KKM_POLY    kappa(x,y) = (gamma x.y + coef0)^degree,  degree >= 1
 *      KKM_GAUSS   kappa(x,y) = exp(-gamma ||x - y||^2),     gamma > 0
 *  - Empty clusters (|c| = 0, where V's row and the centroid are undefined):
 *      KKM_EMPTY_INF            D_ic = +inf, the cluster stays empty
 *      KKM_EMPTY_ZERO_CENTROID  D_ic = K_ii (V's row of zeros taken literally:
 *                               a centroid at the feature-space origin)
 *    argmin ties go to the lowest cluster index.
 */
#ifndef KKM_H
#define KKM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    KKM_OK = 0,
    KKM_ERR_ARG = -1,         /* a size, pointer or parameter is invalid        */
    KKM_ERR_LABEL = -2,       /* an input label lies outside [0, k)             */
    KKM_ERR_NOMEM = -3,       /* a device allocation or a workspace is too small */
    KKM_ERR_HIP = -4,         /* the HIP runtime reported an error               */
    KKM_ERR_UNSUPPORTED = -5, /* valid request the library does not implement   */
    KKM_ERR_NONFINITE = -6    /* the kernel matrix has a non-finite diagonal     */
} kkm_status;

typedef enum { KKM_LINEAR = 0, KKM_POLY = 1, KKM_GAUSS = 2 } kkm_kernel_type;

/* Element types: arithmetic of the Gram product / storage of K. */
typedef enum { KKM_F32 = 0, KKM_BF16 = 1, KKM_FP8_ROWSCALED = 2 } kkm_dtype;

typedef enum { KKM_EMPTY_INF = 0, KKM_EMPTY_ZERO_CENTROID = 1 } kkm_empty_policy;

/* Largest k supported by the per-iteration kernels (LDS histogram size). */
#define KKM_MAX_K 1024

/*
 * kkm_gram — kernel matrix K = kappa(P P^T) and its diagonal (Sec. 3.2 and
 * Sec. 4.2: B = P P^T by a dense product, the kernel function applied to each
 * entry, diag(K) extracted; here all three are one pass, with the product on
 * MFMA and the kernel function and diagonal in its epilogue).
 *
 *   X       [n, ldx] float32 points, row-major (d features used per row).
 *   n, d    number of points (>= 1) and features (>= 1); ldx >= d.
 *   kernel_type, gamma, coef0, degree   kernel function (see above).
 *   gram_prec  arithmetic of the product: KKM_F32 (FP32 MFMA), KKM_BF16
 *           (inputs rounded to bfloat16, FP32 accumulation) or
 *           KKM_FP8_ROWSCALED (each row scaled by max|x|/448 and rounded to
 *           OCP FP8 E4M3, FP32 accumulation).  Squared norms for the Gaussian
 *           are taken from the same rounded values the product uses.
 *   k_store element type of K: KKM_F32 or KKM_BF16.
 *   K       [n, ldk] output, ldk >= n; both triangles are written and K is
 *           exactly symmetric.  With KKM_F32 storage, ldk*4 bytes per row.
 *   diagK   [n] float32 output, K_ii (exactly 1 for the Gaussian).
 *   ws, ws_bytes  device workspace of at least
 *           kkm_gram_workspace_bytes(n, d, gram_prec) bytes (may be NULL
 *           when that is 0).
 * Errors: KKM_ERR_ARG for bad sizes/params/NULL outputs, KKM_ERR_NOMEM for a
 * small workspace, KKM_ERR_UNSUPPORTED for an unimplemented precision pair.
 */
kkm_status kkm_gram(const float *X, int64_t n, int64_t d, int64_t ldx,
                    int32_t kernel_type, double gamma, double coef0, int32_t degree,
                    int32_t gram_prec, int32_t k_store,
                    void *K, int64_t ldk, float *diagK,
                    void *ws, size_t ws_bytes, void *stream);

size_t kkm_gram_workspace_bytes(int64_t n, int64_t d, int32_t gram_prec);

/* Tile shapes of the product (Sec. 4.2 weighs GEMM against SYRK and switches at
 * a tuned n/d threshold): KKM_GRAM_TRIANGLE multiplies the tiles on and above
 * the diagonal only and stores each value at (i, j) and (j, i) (the SYRK
 * work); KKM_GRAM_FULL multiplies every tile of the square, each storing its
 * own block (the GEMM work, twice the flops, one store per value).  Both give
 * the same, exactly symmetric K.  The triangle uses 128 x 128 tiles
 * (KKM_GRAM_TRIANGLE, KKM_GRAM_TRIANGLE_128); KKM_GRAM_TRIANGLE_256 asks for
 * 256 x 256 tiles with a BF16 or FP8 product (half the operand traffic per
 * MFMA, one workgroup per CU; slower on MI355X in every case measured, kept
 * selectable).  Every shape gives the same K bit for bit. */
typedef enum {
    KKM_GRAM_TRIANGLE = 0,
    KKM_GRAM_FULL = 1,
    KKM_GRAM_TRIANGLE_128 = 2,
    KKM_GRAM_TRIANGLE_256 = 3
} kkm_gram_shape;

/* kkm_gram_ex — kkm_gram with the tile shape chosen (kkm_gram uses
 * KKM_GRAM_TRIANGLE).  KKM_ERR_ARG for an unknown shape. */
kkm_status kkm_gram_ex(const float *X, int64_t n, int64_t d, int64_t ldx, int32_t kernel_type,
                       double gamma, double coef0, int32_t degree, int32_t gram_prec,
                       int32_t k_store, int32_t shape, void *K, int64_t ldk, float *diagK,
                       void *ws, size_t ws_bytes, void *stream);

/*
 * kkm_iterate — one reassignment step (Algorithm 2 loop body) for labels_in:
 * builds V in CSR form from the labels (Sec. 4.1), E = K V^T by a row sweep of
 * K (Eq. dist_sp_1), the centroid norms diag(V K V^T) = V z (Eq. c_norm,
 * Eq. cnorms_gemv), D = K_ii - 2E + ||c||^2 and the argmin with the new
 * cluster sizes, all on the GPU.  Stateless: resume = call again.
 *
 *   K, k_store, ldk   kernel matrix from kkm_gram (n x n, row stride ldk).
 *   diagK      [n] float32, K_ii.
 *   n, k       points and clusters, 1 <= k <= min(n, KKM_MAX_K).
 *   labels_in  [n] int32 current labels (not modified).
 *   empty_policy  KKM_EMPTY_INF or KKM_EMPTY_ZERO_CENTROID.
 *   labels_out [n] int32 new labels (must not alias labels_in).
 *   counts_out [k] int32 cluster sizes of labels_out.
 *   n_changed  [1] int64 number of i with labels_out[i] != labels_in[i];
 *              -1 if a label of labels_in lies outside [0, k) (the step is
 *              then skipped and the other outputs are unspecified).
 *   J_in       [1] double objective of labels_in:
 *              sum_i ||phi(x_i) - mu_{a(i)}||^2 = sum_i D_{i, labels_in(i)}.
 *   D_out      [n, k] float32 distances, nullable (for checking).
 *   ctilde_out [k] float32 centroid norms ||c_c||^2, nullable (0 for empty).
 *   ws, ws_bytes  device workspace of at least kkm_iterate_workspace_bytes(n, k).
 * The result is deterministic: the same inputs give bitwise the same outputs.
 */
kkm_status kkm_iterate(const void *K, int32_t k_store, int64_t ldk, const float *diagK,
                       int64_t n, int32_t k, const int32_t *labels_in, int32_t empty_policy,
                       int32_t *labels_out, int32_t *counts_out, int64_t *n_changed,
                       double *J_in, float *D_out, float *ctilde_out,
                       void *ws, size_t ws_bytes, void *stream);

size_t kkm_iterate_workspace_bytes(int64_t n, int32_t k);

/*
 * kkm_iterate_noalloc — kkm_iterate for callers that cannot allocate device
 * memory (code under HIP stream capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same step, the same kernels and bitwise the same
 * outputs, with no workspace argument.  Its scratch is a file-scope device
 * array of KKM_NOALLOC_SCRATCH_BYTES (96 MiB: enough for n = 200000 at
 * k = 64) that each GPU the library runs on holds from the first call on that
 * device until the process ends; the call itself allocates nothing.
 *
 *   Arguments as kkm_iterate without ws / ws_bytes.  The stream (NULL for
 *   the default stream) must belong to the current device.
 *   KKM_ERR_UNSUPPORTED when kkm_iterate_workspace_bytes(n, k) exceeds
 *   KKM_NOALLOC_SCRATCH_BYTES (call kkm_iterate with a workspace instead).
 *   All calls on one GPU share its array, which keeps the last call's
 *   contents: calls that overlap on one GPU (two streams or host threads)
 *   race and must be serialised by the caller.
 */
#define KKM_NOALLOC_SCRATCH_BYTES ((size_t)96 << 20)
kkm_status kkm_iterate_noalloc(const void *K, int32_t k_store, int64_t ldk, const float *diagK,
                               int64_t n, int32_t k, const int32_t *labels_in,
                               int32_t empty_policy, int32_t *labels_out, int32_t *counts_out,
                               int64_t *n_changed, double *J_in, float *D_out, float *ctilde_out,
                               void *stream);
size_t kkm_iterate_noalloc_max_bytes(void);

/*
 * kkm_fit — the whole method (Algorithm 2): K once, then steps until no label
 * changes (check_convergence != 0) or max_iter steps ran.
 *
 *   X, n, d, ldx, kernel_type, gamma, coef0, degree   as kkm_gram.
 *   k          clusters, 1 <= k <= min(n, KKM_MAX_K).
 *   labels0    [n] int32 initial labels (the paper draws them uniformly at
 *              random; the caller supplies them).
 *   max_iter   >= 0; 0 returns labels0 and its objective.
 *   labels_out [n] int32 final labels (device).
 *   objective  host double: J of labels_out (FP64 reduction on the GPU).
 *   iters      host int32: steps executed, including a last step that
 *              changed nothing.
 *   K_ws       device buffer for K of at least n*ldk*4 bytes, or NULL to let
 *              the library allocate (and free) it.  ldk >= n is used with K_ws;
 *              it is ignored when K_ws is NULL.
 * Errors: as kkm_gram and kkm_iterate, plus KKM_ERR_LABEL for labels0 outside
 * [0, k) and KKM_ERR_NONFINITE when diag(K) has a NaN or infinity.
 */
kkm_status kkm_fit(const float *X, int64_t n, int64_t d, int64_t ldx, int32_t k,
                   int32_t kernel_type, double gamma, double coef0, int32_t degree,
                   const int32_t *labels0, int32_t max_iter, int32_t check_convergence,
                   int32_t *labels_out, double *objective, int32_t *iters,
                   void *K_ws, int64_t ldk, void *stream);

/*
 * kkm_fit_ex — kkm_fit with the precision forms and per-run records.
 *
 *   gram_prec, k_store, empty_policy   as kkm_gram / kkm_iterate.
 *   J_trace       host double [max_iter + 1], nullable: J of the labels
 *                 entering each executed step, then J(labels_out).
 *   changed_trace host int64 [max_iter], nullable: labels changed per step.
 *   times_ms      host double [3], nullable: {Gram, all steps, final objective}
 *                 wall time on the stream, in milliseconds.
 */
kkm_status kkm_fit_ex(const float *X, int64_t n, int64_t d, int64_t ldx, int32_t k,
                      int32_t kernel_type, double gamma, double coef0, int32_t degree,
                      int32_t gram_prec, int32_t k_store, int32_t empty_policy,
                      const int32_t *labels0, int32_t max_iter, int32_t check_convergence,
                      int32_t *labels_out, double *objective, int32_t *iters,
                      void *K_ws, int64_t ldk, double *J_trace, int64_t *changed_trace,
                      double *times_ms, void *stream);

/*
 * kkm_refine — the loop of kkm_fit_ex on a kernel matrix already in memory
 * (Algorithm 2 without its first step): for warm starts that need K before
 * the first step, such as kkm_kernel_kmeanspp.
 *
 *   K, k_store, ldk, diagK   as kkm_iterate (from kkm_gram).
 *   empty_policy, labels0, max_iter, check_convergence, labels_out,
 *   objective, iters, J_trace, changed_trace   as kkm_fit_ex.
 *   times_ms   host double [2], nullable: {all steps, final objective pass}.
 * Synchronises the stream before returning; the same labels0 give bitwise
 * the same results as the loop inside kkm_fit_ex on the same K.
 */
kkm_status kkm_refine(const void *K, int32_t k_store, int64_t ldk, const float *diagK, int64_t n,
                      int32_t k, int32_t empty_policy, const int32_t *labels0, int32_t max_iter,
                      int32_t check_convergence, int32_t *labels_out, double *objective,
                      int32_t *iters, double *J_trace, int64_t *changed_trace, double *times_ms,
                      void *stream);

/* ------------------------------------------------------------------------
 * Batched form: many independent clustering problems of uneven sizes, each
 * the computation of kkm_fit_ex (Algorithm 2 of the paper run once per
 * problem), sharing every launch.  One persistent Gram launch takes 128 x 128
 * tiles of all problems from a device queue, problems with the costliest
 * tiles first; then each iteration is one set of launches over the problems
 * still running, replayed from a captured HIP graph while a device-side
 * predicate retires converged problems.
 */

/* One problem of a batch (host struct; X is a device pointer). */
typedef struct {
    const float *X;      /* [n, ldx] float32 points, row-major              */
    int64_t n, d, ldx;   /* n >= 1, d >= 1, ldx >= d                        */
    int32_t k;           /* 1 <= k <= min(n, KKM_MAX_K)                     */
    int32_t kernel_type; /* kernel function, as kkm_gram                    */
    double gamma, coef0;
    int32_t degree;
    int32_t chunk_rows;  /* rows of K per sweep workgroup, in [1, 2^20];
                            0 = the single-problem default (results then
                            match kkm_fit_ex bit for bit)                   */
} kkm_instance;

/*
 * kkm_fit_batched_workspace_bytes — device workspace that kkm_fit_batched
 * needs for these problems: every K (n x roundup(n, 64) elements of k_store,
 * kept for the whole run), the rounded rows of the product, the per-problem
 * step buffers and the instance tables.  0 on invalid arguments.
 */
size_t kkm_fit_batched_workspace_bytes(const kkm_instance *inst, int32_t count,
                                       int32_t gram_prec, int32_t k_store);

/*
 * kkm_fit_batched — kkm_fit_ex for each of `count` problems.
 *
 *   inst          host kkm_instance [count].
 *   gram_prec, k_store, empty_policy   as kkm_fit_ex, for every problem.
 *   labels0       int32 [sum n]: the initial labels of problem 0, then of
 *                 problem 1, ... (problem b starts at n_0 + ... + n_{b-1}).
 *   max_iter, check_convergence   as kkm_fit_ex, for every problem.
 *   use_graph     1: the iteration is captured once into a HIP graph (one
 *                 per label-buffer parity) and replayed; 0: launched
 *                 directly.  The results are identical.
 *   labels_out    int32 [sum n], same layout as labels0.
 *   objective     host double [count]: J(labels_out) of each problem.
 *   iters         host int32 [count]: steps run per problem (as kkm_fit_ex).
 *   times_ms      host double [3], nullable: {Gram with its prologue, all
 *                 steps, final objective pass} on the stream.
 *   ws, ws_bytes  workspace of kkm_fit_batched_workspace_bytes bytes, or
 *                 NULL to let the call allocate (and free) it.
 * Synchronises the stream before returning.  KKM_ERR_LABEL names the first
 * problem whose labels0 holds a label outside [0, k); KKM_ERR_NONFINITE is
 * returned when any problem's diag(K) is not finite.
 */
kkm_status kkm_fit_batched(const kkm_instance *inst, int32_t count, int32_t gram_prec,
                           int32_t k_store, int32_t empty_policy, const int32_t *labels0,
                           int32_t max_iter, int32_t check_convergence, int32_t use_graph,
                           int32_t *labels_out, double *objective, int32_t *iters,
                           double *times_ms, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Learned warm start.  The paper draws the initial labels at random (Sec.
 * 3.4); these entry points produce a better start: a small network
 * phi_theta: R^d -> R^h1 -> R^h2 -> R^out (GELU after the first two layers,
 * last layer linear) is trained so that phi(x).phi(y) approximates the kernel
 * values kappa(x, y) that kkm_gram computes, and Lloyd's iterations with
 * explicit centroids (Sec. 2.1) on the rows of F = phi_theta(X) give labels
 * that kkm_fit then refines exactly.
 *
 * Parameter vector (FP32, device, `kkm_mlp_param_count` floats, row-major):
 *   W1 [h1, d], b1 [h1], W2 [h2, h1], b2 [h2], W3 [out, h2], b3 [out].
 * Matrix products take bfloat16 operands (weights and activations rounded to
 * nearest even) with FP32 accumulation; loss products and Adam are FP32.
 * ------------------------------------------------------------------------ */

int64_t kkm_mlp_param_count(int64_t d, int64_t h1, int64_t h2, int64_t out);

/* F [n, ldf] = phi_theta(X [n, ldx]).  Asynchronous.  Workspace: at least
 * kkm_mlp_forward_workspace_bytes(n, d, h1, h2, out). */
kkm_status kkm_mlp_forward(const float *params, int64_t d, int64_t h1, int64_t h2, int64_t out,
                           const float *X, int64_t n, int64_t ldx, float *F, int64_t ldf,
                           void *ws, size_t ws_bytes, void *stream);
size_t kkm_mlp_forward_workspace_bytes(int64_t n, int64_t d, int64_t h1, int64_t h2, int64_t out);

/* kkm_mlp_forward with every layer's output: H1 [n, h1] = GELU(X W1^T + b1),
 * H2 [n, h2] = GELU(H1 W2^T + b2) (row strides h1 and h2, FP32, device) and
 * F [n, ldf] = H2 W3^T + b3, the same values kkm_mlp_forward computes (each
 * product rounds its operands to bfloat16 and accumulates in FP32), for
 * checking the layers one at a time.  No workspace.  Asynchronous. */
kkm_status kkm_mlp_forward_layers(const float *params, int64_t d, int64_t h1, int64_t h2,
                                  int64_t out, const float *X, int64_t n, int64_t ldx, float *H1,
                                  float *H2, float *F, int64_t ldf, void *stream);

/* Loss L = (1/B^2) ||Phi Phi^T - KB||_F^2 of a batch XB [B, ldx] with kernel
 * values KB [B, ldkb] (symmetric), and dL/dparams into grad (param_count
 * floats, device).  *loss is a device double.  Asynchronous.  Workspace: at
 * least kkm_mlp_train_workspace_bytes(B, d, h1, h2, out). */
kkm_status kkm_mlp_loss_grad(const float *params, int64_t d, int64_t h1, int64_t h2, int64_t out,
                             const float *XB, int64_t B, int64_t ldx, const float *KB,
                             int64_t ldkb, float *grad, double *loss, void *ws, size_t ws_bytes,
                             void *stream);
size_t kkm_mlp_train_workspace_bytes(int64_t B, int64_t d, int64_t h1, int64_t h2, int64_t out);

/* One Adam step (bias-corrected, step number t >= 1) on `count` parameters:
 * params, first and second moments adam_m / adam_v updated in place. */
kkm_status kkm_mlp_adam(float *params, float *adam_m, float *adam_v, const float *grad,
                        int64_t count, int32_t t, double lr, double beta1, double beta2,
                        double eps, void *stream);

/* `steps` training steps.  Step s takes the B training points listed in
 * batch_idx[s*B .. s*B+B) (device int32, each in [0, mtrain); the caller draws
 * them), gathers their rows of Xtrain [mtrain, ldx] and their block of the
 * kernel matrix Ktrain [mtrain, ldk] (from kkm_gram), computes the loss and
 * gradient and applies Adam with step numbers t0+1 .. t0+steps.  loss_trace
 * (device double [steps]) receives each step's loss.  KKM_ERR_ARG when an
 * index is out of range (checked before any update).  Asynchronous apart from
 * that check. */
kkm_status kkm_mlp_train(float *params, float *adam_m, float *adam_v, int64_t d, int64_t h1,
                         int64_t h2, int64_t out, const float *Xtrain, int64_t mtrain,
                         int64_t ldx, const float *Ktrain, int64_t ldk, const int32_t *batch_idx,
                         int64_t B, int32_t steps, int32_t t0, double lr, double beta1,
                         double beta2, double eps, double *loss_trace, void *ws, size_t ws_bytes,
                         void *stream);

/* `steps` training steps on fresh batches: step s takes rows s*B .. s*B+B-1 of
 * Xtrain [steps*B, ldx], computes their B x B kernel values with the Gram
 * kernel (FP32; kernel_type/gamma/coef0/degree as kkm_gram), then the loss,
 * the gradient and an Adam step (step numbers t0+1 .. t0+steps).  Over all
 * steps the network sees steps * B(B-1)/2 distinct kernel-value pairs.
 * loss_trace: device double [steps].  Asynchronous.  Workspace: at least
 * kkm_mlp_train_fresh_workspace_bytes(B, d, h1, h2, out). */
kkm_status kkm_mlp_train_fresh(float *params, float *adam_m, float *adam_v, int64_t d, int64_t h1,
                               int64_t h2, int64_t out, const float *Xtrain, int64_t ldx,
                               int64_t B, int32_t steps, int32_t t0, int32_t kernel_type,
                               double gamma, double coef0, int32_t degree, double lr,
                               double beta1, double beta2, double eps, double *loss_trace,
                               void *ws, size_t ws_bytes, void *stream);
size_t kkm_mlp_train_fresh_workspace_bytes(int64_t B, int64_t d, int64_t h1, int64_t h2,
                                           int64_t out);

/* Lloyd's iterations with explicit centroids on feature rows F [n, ldf] (f
 * features), from labels0 (device int32 [n]), until no label changes or
 * max_iter steps: d_ic = ||f_i - mean_{j in c} f_j||^2, lowest index on ties,
 * empty clusters never chosen.  labels_out (device) must not alias labels0;
 * iters (host) = steps executed; changed_trace (host int64 [max_iter],
 * nullable) = labels changed per step; objective (host double, nullable) =
 * sum_i min_c d_ic of the last step, i.e. the feature-space objective of
 * labels_out when that step changed nothing (NaN if no step ran).
 * Synchronous.  KKM_ERR_LABEL when labels0 has a label outside [0, k). */
kkm_status kkm_feature_lloyd(const float *F, int64_t n, int64_t f, int64_t ldf, int32_t k,
                             const int32_t *labels0, int32_t max_iter, int32_t *labels_out,
                             int32_t *iters, int64_t *changed_trace, double *objective, void *ws,
                             size_t ws_bytes, void *stream);
size_t kkm_feature_lloyd_workspace_bytes(int64_t n, int64_t f, int32_t k);

/* K-means++ seeding (D^2 sampling, the K-means++ of Sec. 2.1) on feature rows
 * F [n, ldf]: seed 0 is row floor(u_0 n); seed t is the first row whose running
 * sum of squared distances to the nearest earlier seed exceeds u_t times their
 * total (sums in FP64, fixed order).  uniforms: host double [k] in [0, 1),
 * drawn by the caller.  seeds (device int32 [k]) receives the chosen rows and
 * labels_out (device int32 [n]) the index of each row's nearest seed (lowest
 * on ties).  Asynchronous. */
kkm_status kkm_feature_kmeanspp(const float *F, int64_t n, int64_t f, int64_t ldf, int32_t k,
                                const double *uniforms, int32_t *seeds, int32_t *labels_out,
                                void *ws, size_t ws_bytes, void *stream);
size_t kkm_feature_kmeanspp_workspace_bytes(int64_t n, int64_t f, int32_t k);

/* K-means++ seeding in the kernel's feature space, from the kernel matrix
 * itself (no learned features): the same D^2 sampling as
 * kkm_feature_kmeanspp with the squared distance of point i to seed s taken
 * as K_ii + K_ss - 2 K_si (Sec. 2.2's kernel trick on two points, clamped at
 * 0 against rounding; FP32).  Reads one row of K per seed and k rows for the
 * labels.  K [n, ldk] (KKM_F32 or KKM_BF16, k_store), diagK [n] as written by
 * kkm_gram; uniforms: host double [k] in [0, 1); seeds (device int32 [k]);
 * labels_out (device int32 [n]) = index of each point's nearest seed (lowest
 * on ties).  k <= KKM_MAX_K.  Asynchronous. */
kkm_status kkm_kernel_kmeanspp(const void *K, int32_t k_store, int64_t ldk, const float *diagK,
                               int64_t n, int32_t k, const double *uniforms, int32_t *seeds,
                               int32_t *labels_out, void *ws, size_t ws_bytes, void *stream);
size_t kkm_kernel_kmeanspp_workspace_bytes(int64_t n, int32_t k);

/* kkm_warm_start — the learned warm start in one call (replacing the random
 * initial labels of Sec. 3.4): F = phi_theta(X) as kkm_mlp_forward computes it,
 * then `restarts` independent k-means++ seedings (the D^2 sampling of Sec.
 * 2.1, as kkm_feature_kmeanspp) each followed by at most max_iter Lloyd steps
 * in feature space (as kkm_feature_lloyd, Sec. 2.1's three phases with
 * explicit centroids), and the labelling whose feature-space objective (the
 * `objective` of kkm_feature_lloyd) is lowest; ties, and restarts whose
 * objective is NaN, go to the lowest restart index.  kkm_fit_ex then refines
 * labels_out exactly.
 *
 *   params, d, h1, h2, out   the network, as kkm_mlp_forward.
 *   X [n, ldx]    float32 points (device).
 *   k             clusters, 1 <= k <= min(n, KKM_MAX_K).
 *   restarts      >= 1 seedings; restart r draws with uniforms[r*k .. r*k+k)
 *                 (host double, each in [0, 1)).
 *   max_iter      >= 0 Lloyd steps per restart.
 *   streams       >= 1: the restarts run on this many internal streams of
 *                 default priority, one host thread each; the result is the
 *                 same for every value.
 *   labels_out    [n] int32 (device) the chosen labelling.
 *   objective, cheap_iters, best_restart   host, nullable: the chosen
 *                 restart's feature-space objective, the Lloyd steps summed
 *                 over all restarts, and the chosen restart's index.
 *   ws, ws_bytes  at least kkm_warm_start_workspace_bytes(n, d, h1, h2, out,
 *                 k, streams) bytes of device workspace.
 * Synchronises `stream` before returning.  Errors: KKM_ERR_ARG (sizes, NULL
 * pointers, a uniform outside [0, 1)), KKM_ERR_NOMEM (small workspace),
 * KKM_ERR_UNSUPPORTED (k > KKM_MAX_K), or the error of a failing restart. */
kkm_status kkm_warm_start(const float *params, int64_t d, int64_t h1, int64_t h2, int64_t out,
                          const float *X, int64_t n, int64_t ldx, int32_t k, int32_t restarts,
                          const double *uniforms, int32_t max_iter, int32_t streams,
                          int32_t *labels_out, double *objective, int32_t *cheap_iters,
                          int32_t *best_restart, void *ws, size_t ws_bytes, void *stream);
size_t kkm_warm_start_workspace_bytes(int64_t n, int64_t d, int64_t h1, int64_t h2, int64_t out,
                                      int32_t k, int32_t streams);

/*
 * kkm_iterate_matfree — one reassignment step without a stored kernel matrix
 * (the paper computes K once, Sec. 3.2, and streams it every iteration,
 * Sec. 4.3; here every entry K_ij = kappa(x_i, x_j) is recomputed on the
 * MFMA inside the step and added into E = K V^T at once, Eq. dist_sp_1, so
 * no n x n buffer exists).  Worth it below the product's ridge point (small
 * d); the result is the stored-K step's up to summation order.
 *
 *   X, n, d, ldx, kernel_type, gamma, coef0, degree, gram_prec   as kkm_gram
 *              (the product in FP32, BF16 or FP8 per-row scaled; the kernel
 *              values summed are not rounded further, as k_store = KKM_F32).
 *   k, labels_in, empty_policy, labels_out, counts_out, n_changed, J_in,
 *   D_out, ctilde_out   as kkm_iterate.
 *   diagK_out  [n] float32, nullable: K_ii as the step used it.
 *   ws, ws_bytes  device workspace of at least
 *              kkm_iterate_matfree_workspace_bytes(n, d, k, gram_prec).
 * Asynchronous; deterministic.  Errors as kkm_gram and kkm_iterate.
 */
kkm_status kkm_iterate_matfree(const float *X, int64_t n, int64_t d, int64_t ldx,
                               int32_t kernel_type, double gamma, double coef0, int32_t degree,
                               int32_t gram_prec, int32_t k, const int32_t *labels_in,
                               int32_t empty_policy, int32_t *labels_out, int32_t *counts_out,
                               int64_t *n_changed, double *J_in, float *D_out, float *ctilde_out,
                               float *diagK_out, void *ws, size_t ws_bytes, void *stream);
size_t kkm_iterate_matfree_workspace_bytes(int64_t n, int64_t d, int32_t k, int32_t gram_prec);

/*
 * kkm_fit_matfree — Algorithm 2 end to end with the matrix-free step: the
 * product's inputs (rounded rows, squared norms) and diag(K) once, then
 * kkm_iterate_matfree steps until no label changes (check_convergence != 0)
 * or max_iter steps, then the objective of the final labels.  Arguments and
 * results as kkm_fit_ex without K (k_store is FP32 by construction);
 * times_ms (host double [3], nullable): {prologue, all steps, final
 * objective}.  Allocates its workspace (about (slots + d) n floats, no n^2
 * term) and synchronises the stream before returning.
 */
kkm_status kkm_fit_matfree(const float *X, int64_t n, int64_t d, int64_t ldx, int32_t k,
                           int32_t kernel_type, double gamma, double coef0, int32_t degree,
                           int32_t gram_prec, int32_t empty_policy, const int32_t *labels0,
                           int32_t max_iter, int32_t check_convergence, int32_t *labels_out,
                           double *objective, int32_t *iters, double *J_trace,
                           int64_t *changed_trace, double *times_ms, void *stream);

/*
 * The strip-packed symmetric K (Sec. 4.2 names packed triangular storage as
 * what a SYRK-built K needs; Sec. 4.3 streams K every iteration): the upper
 * triangle in strips of W = 1024 columns (FP32 or bfloat16).
 * Row i, in strip s_i = i / W, stores its columns [s_i W, ns W) contiguously,
 * ns = ceil(n / W): the diagonal W x W block of each strip whole, every block
 * right of it once, about n^2 / 2 entries.  Rows follow each other with no
 * stride argument; kkm_packed_elements(n, k_store) entries in all.
 *
 * kkm_gram_packed — kkm_gram writing K in this layout (the 128 x 128
 * triangle of tiles; K 16-byte aligned).  Arguments as kkm_gram without ldk.
 *
 * kkm_iterate_packed — kkm_iterate on a strip-packed K: each stored entry is
 * read once and feeds both S_{i,a(j)} and S_{j,a(i)}.  Arguments as
 * kkm_iterate without ldk; k <= 128 (else KKM_ERR_UNSUPPORTED); workspace of
 * at least kkm_iterate_packed_workspace_bytes(n, k, k_store) (about
 * k n^2 / (2 W) floats of per-row bins besides the step's partial sums).
 * Asynchronous; deterministic.
 *
 * kkm_fit_packed — kkm_fit_ex with K strip-packed: K_ws (nullable) holds
 * kkm_packed_elements(n, k_store) entries of k_store, else the library
 * allocates them.  Synchronous; results and traces as kkm_fit_ex.
 */
size_t kkm_packed_elements(int64_t n, int32_t k_store);
kkm_status kkm_gram_packed(const float *X, int64_t n, int64_t d, int64_t ldx, int32_t kernel_type,
                           double gamma, double coef0, int32_t degree, int32_t gram_prec,
                           int32_t k_store, void *K, float *diagK, void *ws, size_t ws_bytes,
                           void *stream);
kkm_status kkm_iterate_packed(const void *K, int32_t k_store, const float *diagK, int64_t n,
                              int32_t k, const int32_t *labels_in, int32_t empty_policy,
                              int32_t *labels_out, int32_t *counts_out, int64_t *n_changed,
                              double *J_in, float *D_out, float *ctilde_out, void *ws,
                              size_t ws_bytes, void *stream);
size_t kkm_iterate_packed_workspace_bytes(int64_t n, int32_t k, int32_t k_store);
kkm_status kkm_fit_packed(const float *X, int64_t n, int64_t d, int64_t ldx, int32_t k,
                          int32_t kernel_type, double gamma, double coef0, int32_t degree,
                          int32_t gram_prec, int32_t k_store, int32_t empty_policy,
                          const int32_t *labels0, int32_t max_iter, int32_t check_convergence,
                          int32_t *labels_out, double *objective, int32_t *iters, void *K_ws,
                          double *J_trace, int64_t *changed_trace, double *times_ms, void *stream);

/*
 * Launch timing for benchmarks (process-wide).  kkm_timing_enable(1) clears
 * the records and starts bracketing every Gram launch, every SpMM sweep launch
 * (for a strip-packed K the sweep kernel alone), every fold of the packed row
 * part and every whole kkm_iterate step with HIP events on the caller's
 * stream; kkm_timing_enable(0) clears and stops.  kkm_timing_read waits for
 * the recorded events and returns, per class {0: Gram, 1: sweep, 2: iterate
 * step, 3: packed fold}, the total milliseconds (host double[4]) and the
 * number of launches (host int64[4]) since timing was enabled.
 */
kkm_status kkm_timing_enable(int32_t on);
kkm_status kkm_timing_read(double *total_ms, int64_t *launches);

/* kkm_timing_spans — the individual durations (milliseconds, launch order) of
 * the launches of class cls (0: Gram, 1: sweep, 2: iterate step, 3: packed
 * fold) recorded since
 * timing was enabled: ms (host double [cap]) receives the first min(cap,
 * *count) of them and *count (host) their number.  Waits for the recorded
 * events.  KKM_ERR_ARG for an unknown class or a NULL output. */
kkm_status kkm_timing_spans(int32_t cls, double *ms, int64_t cap, int64_t *count);

/* Message for the last error on this thread ("" if none). */
const char *kkm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* KKM_H */
