// Kernel matrix K = kappa(P P^T) with diag(K), MFMA on gfx950.
//
// Sec. 3.2 of the paper builds B = P P^T with a dense product and then applies
// the kernel function to every entry (polynomial: pow(gamma B + c, r);
// Gaussian: Eq. gauss, exp(-gamma (B_ii + B_jj - 2 B_ij))); Sec. 3.3 reads
// ||phi(p_i)||^2 off diag(K).  Sec. 4.2 weighs GEMM (all of B) against SYRK
// (one triangle plus a copy into the other, because the sparse routines need
// K stored in full).
//
// Here the three steps are one kernel: only tiles on or above the diagonal are
// multiplied (the SYRK flop count), and the epilogue applies kappa and writes
// each value to both K[i][j] and K[j][i], so no copy pass exists and K is
// exactly symmetric.  B never reaches memory.
//
// Arithmetic of the product (gram_prec):
//   F32   FP32 inputs, v_mfma_f32_32x32x2_f32.
//   BF16  inputs rounded to bfloat16 (round to nearest even), FP32 accumulation,
//         v_mfma_f32_32x32x16_bf16.
//   FP8   each row scaled by s_i = max_l |x_il| / 448 and rounded to OCP FP8
//         E4M3 (round to nearest even, clamped to +-448), FP32 accumulation,
//         v_mfma_f32_32x32x16_fp8_fp8; B_ij = s_i s_j sum_l q_il q_jl.
// For BF16/FP8 the squared norms of the Gaussian are taken from the same
// rounded values.  K is stored as FP32 or bfloat16 (k_store).  The Gaussian is
// evaluated as 2^(-gamma log2(e) s) with the hardware base-2 exponential.
#include "gram_tile.h"

namespace kkm {

namespace {

using namespace gt;

// ---------------------------------------------------------------- prologues

// Squared row norms ||x_i||^2 for the Gaussian (FP32 product): one wave per row.
__global__ __launch_bounds__(256) void row_sqnorms(const float *X, int64_t n, int64_t d,
                                                   int64_t ldx, float *nrm) {
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    sqnorm_row(X + row * ldx, d, nrm + row, lane);
}

// One wave per row: rounds the row and records its squared norm (and scale).
template <int PREC>
__global__ __launch_bounds__(256) void quantize_rows(const float *X, int64_t n, int64_t d,
                                                     int64_t ldx, int64_t dpad,
                                                     unsigned char *Xq, float *nrm,
                                                     float *scale) {
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= n) return;
    const int64_t eb = (PREC == KKM_BF16) ? 2 : 1;
    quantize_row<PREC>(X + row * ldx, d, dpad, Xq + row * dpad * eb, nrm + row, scale + row,
                       threadIdx.x & 63);
}

// log2 of the tile group edge of the launch order: 8 x 8 groups, so the 64
// tiles an XCD holds at once (32 CUs x 2 workgroups) read 16 operand panels.
int group_log2(int64_t d, int32_t gram_prec) {
    (void)d;
    (void)gram_prec;
    return 3;
}

}  // namespace

size_t gram_workspace_bytes(int64_t n, int64_t d, int32_t gram_prec) {
    Carver c(nullptr);
    c.take<float>((size_t)n);  // squared norms
    if (gram_prec != KKM_F32) {
        c.take<float>((size_t)n);  // row scales
        const size_t eb = (gram_prec == KKM_BF16) ? 2 : 1;
        c.take<unsigned char>((size_t)n * (size_t)padded_d(d, gram_prec) * eb);
    }
    return c.bytes();
}

kkm_status gram_launch(const float *X, int64_t n, int64_t d, int64_t ldx, int32_t kernel,
                       double gamma, double coef0, int32_t degree, int32_t gram_prec,
                       int32_t k_store, void *K, int64_t ldk, float *diagK, void *ws,
                       size_t ws_bytes, hipStream_t stream, int32_t shape, bool packed) {
    const size_t need = gram_workspace_bytes(n, d, gram_prec);
    if (ws == nullptr || ws_bytes < need) {
        set_error("kkm_gram: workspace of %zu bytes is smaller than %zu", ws_bytes, need);
        return KKM_ERR_NOMEM;
    }
    if (gram_prec != KKM_F32 && !lowp_rows_fit(d, gram_prec)) {
        set_error("kkm_gram: d=%lld is too large for the BF16 / FP8 product's 32-bit row ranges",
                  (long long)d);
        return KKM_ERR_UNSUPPORTED;
    }
    Carver c(ws);
    float *nrm = c.take<float>((size_t)n);
    Epi e;
    e.n = n;
    e.ldk = ldk;
    e.kernel = kernel;
    e.gamma = epi_gamma(kernel, gamma);
    e.coef0 = (float)coef0;
    e.degree = degree;
    e.nrm = nrm;
    e.scale = nullptr;
    e.K = K;
    e.diag = diagK;
    const uintptr_t kaddr = reinterpret_cast<uintptr_t>(K);
    e.vec_k = (k_store == KKM_F32) ? (((ldk % 4) == 0) && ((kaddr & 15) == 0))
                                   : (((ldk % 4) == 0) && ((kaddr & 7) == 0));
    e.plgw = 0;
    e.pns = 0;
    if (packed) {
        // strip-packed rows start at multiples of the strip width
        e.plgw = packed_lgw(k_store);
        e.pns = packed_strips(n, e.plgw);
        e.vec_k = (k_store == KKM_F32) ? ((kaddr & 15) == 0) : ((kaddr & 7) == 0);
        if (shape != KKM_GRAM_TRIANGLE && shape != KKM_GRAM_TRIANGLE_128) {
            set_error("kkm_gram: a packed K is written by the 128 x 128 triangle only");
            return KKM_ERR_UNSUPPORTED;
        }
    }
    const bool full = (shape == KKM_GRAM_FULL);
    // 256 x 256 tiles only on request: measured slower on MI355X at every n and
    // d tried (one workgroup per CU leaves the epilogue and the operand-load
    // latency of a tile without another tile to hide behind)
    const bool big = gram_prec != KKM_F32 && shape == KKM_GRAM_TRIANGLE_256;
    const TileOrder order = tile_order(n, group_log2(d, gram_prec), full, big ? GB : GM);
    const int64_t grid = order.per_xcd * 8;
    if (grid > 0x7fffffff) {
        set_error("kkm_gram: n=%lld needs more than 2^31 tiles", (long long)n);
        return KKM_ERR_UNSUPPORTED;
    }
    const unsigned qgrid = (unsigned)((n + 3) / 4);

    if (gram_prec == KKM_F32) {
        if (kernel == KKM_GAUSS) {
            hipLaunchKernelGGL(row_sqnorms, dim3(qgrid), dim3(256), 0, stream, X, n, d, ldx, nrm);
            KKM_HIP(hipGetLastError());
        }
        F32Tile a;
        a.X = X;
        a.d = d;
        a.ldx = ldx;
        a.vec_x = ((ldx % 4) == 0) && ((reinterpret_cast<uintptr_t>(X) & 15) == 0);
        a.e = e;
        const TimedSpan span = timing_begin(TK_GRAM, stream);
        launch_gram_f32(k_store, full, dim3((unsigned)grid), a, order, stream);
        KKM_HIP(hipGetLastError());
        timing_end(span, stream);
        return KKM_OK;
    }

    float *scale = c.take<float>((size_t)n);
    const int64_t dpad = padded_d(d, gram_prec);
    const int64_t eb = (gram_prec == KKM_BF16) ? 2 : 1;
    unsigned char *Xq = c.take<unsigned char>((size_t)n * (size_t)dpad * (size_t)eb);
    if (gram_prec == KKM_BF16)
        hipLaunchKernelGGL(quantize_rows<KKM_BF16>, dim3(qgrid), dim3(256), 0, stream, X, n, d,
                           ldx, dpad, Xq, nrm, scale);
    else
        hipLaunchKernelGGL(quantize_rows<KKM_FP8_ROWSCALED>, dim3(qgrid), dim3(256), 0, stream,
                           X, n, d, ldx, dpad, Xq, nrm, scale);
    KKM_HIP(hipGetLastError());
    LowpTile a;
    a.Xq = Xq;
    a.ldq_bytes = dpad * eb;
    a.nslab = dpad * eb / SLAB;
    a.e = e;
    if (gram_prec == KKM_FP8_ROWSCALED) a.e.scale = scale;
    const TimedSpan span = timing_begin(TK_GRAM, stream);
    if (big)
        launch_gram_lowp256(gram_prec, k_store, dim3((unsigned)grid), a, order, stream);
    else
        launch_gram_lowp(gram_prec, k_store, full, dim3((unsigned)grid), a, order, stream);
    KKM_HIP(hipGetLastError());
    timing_end(span, stream);
    return KKM_OK;
}

}  // namespace kkm
