// Kernel matrix K = kappa(P P^T) with diag(K), FP32 MFMA on gfx950.
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
#include "kkm_common.h"

namespace kkm {

namespace {

constexpr int GM = 128;       // tile edge (rows = columns)
constexpr int GK = 32;        // k-slab staged in LDS per step
constexpr int GLD = GK + 4;   // padded LDS row stride in floats (conflict-free b128 reads)
constexpr int GTHREADS = 256; // 4 waves as 2 x 2, each owns a 64 x 64 sub-tile

struct GramArgs {
    const float *X;
    int64_t n, d, ldx;
    int kernel;
    float gamma, coef0;
    int degree;
    const float *nrm;  // squared row norms (Gaussian only)
    float *K;
    int64_t ldk;
    float *diag;
    int64_t nb;        // tile rows
    int64_t ntiles;    // nb (nb + 1) / 2
    int64_t per_xcd;   // ceil(ntiles / 8)
    int vec_x;         // X rows 16-byte aligned: float4 loads allowed
    int vec_k;         // K rows 16-byte aligned: float4 stores allowed
};

__device__ __forceinline__ float kappa_from_dot(float b, float ni, float nj, int kernel,
                                                float gamma, float coef0, int degree) {
    if (kernel == KKM_GAUSS) {
        float sq = fmaxf(ni + nj - 2.0f * b, 0.0f);
        return expf(-gamma * sq);
    }
    if (kernel == KKM_POLY) {
        float t = fmaf(gamma, b, coef0);
        float v = t;
        for (int r = 1; r < degree; ++r) v *= t;
        return v;
    }
    return b;
}

__device__ __forceinline__ f32x4 load_row4(const GramArgs &a, int64_t row, int64_t col) {
    f32x4 v = {0.f, 0.f, 0.f, 0.f};
    if (row < a.n) {
        const float *src = a.X + row * a.ldx + col;
        if (a.vec_x && col + 3 < a.d) {
            v = *reinterpret_cast<const f32x4 *>(src);
        } else {
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (col + u < a.d) v[u] = src[u];
        }
    }
    return v;
}

// Upper-triangle tile t -> (bi, bj), bi <= bj, column by column.
__device__ __forceinline__ void tile_coords(int64_t t, int64_t &bi, int64_t &bj) {
    int64_t j = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while (j * (j + 1) / 2 > t) --j;
    while ((j + 1) * (j + 2) / 2 <= t) ++j;
    bj = j;
    bi = t - j * (j + 1) / 2;
}

__global__ __launch_bounds__(GTHREADS, 2) void gram_f32_mfma(GramArgs a) {
    __shared__ __attribute__((aligned(16))) float lds[2][2][GM * GLD];

    // Workgroups are dealt to the 8 XCDs round-robin; give each XCD a contiguous
    // range of tiles so that the tiles sharing an operand panel share an L2.
    const int64_t pid = blockIdx.x;
    const int64_t t = (pid % 8) * a.per_xcd + pid / 8;
    if (t >= a.ntiles) return;
    int64_t bi, bj;
    tile_coords(t, bi, bj);
    const int64_t m0 = bi * GM, n0 = bj * GM;
    const bool diag_tile = (bi == bj);

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;

    // staging: 8 threads cover one 32-float row slice; 4 row groups of 32
    const int ld_row = tid >> 3;
    const int ld_col = (tid & 7) * 4;

    f32x4 ra[4], rb[4];
    auto gload = [&](int64_t k0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            ra[u] = load_row4(a, m0 + ld_row + 32 * u, k0 + ld_col);
            rb[u] = load_row4(a, n0 + ld_row + 32 * u, k0 + ld_col);
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            *reinterpret_cast<f32x4 *>(&lds[buf][0][(ld_row + 32 * u) * GLD + ld_col]) = ra[u];
            *reinterpret_cast<f32x4 *>(&lds[buf][1][(ld_row + 32 * u) * GLD + ld_col]) = rb[u];
        }
    };

    f32x16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    const int64_t nk = (a.d + GK - 1) / GK;
    gload(0);
    sstore(0);
    __syncthreads();

    // The 32x32x2 MFMA takes A[i][kk] from lane (kk*32 + i) and B[kk][j] from
    // lane (kk*32 + j).  Within a slab the k index is permuted the same way for
    // both operands (lane half h covers k = 16h .. 16h+15 across 16 MFMAs), so
    // each lane fetches 16 consecutive floats with four b128 LDS reads.
    const int half = lane >> 5;
    const int l32 = lane & 31;
    for (int64_t kt = 0; kt < nk; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < nk) gload((kt + 1) * GK);

        const float *As = lds[buf][0];
        const float *Bs = lds[buf][1];
        f32x4 av[2][4], bv[2][4];
#pragma unroll
        for (int mi = 0; mi < 2; ++mi) {
            const float *pa = As + (wr * 64 + mi * 32 + l32) * GLD + half * 16;
            const float *pb = Bs + (wc * 64 + mi * 32 + l32) * GLD + half * 16;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                av[mi][q] = *reinterpret_cast<const f32x4 *>(pa + 4 * q);
                bv[mi][q] = *reinterpret_cast<const f32x4 *>(pb + 4 * q);
            }
        }
#pragma unroll
        for (int s = 0; s < 16; ++s)
#pragma unroll
            for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                for (int ni = 0; ni < 2; ++ni)
                    acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x2f32(
                        av[mi][s >> 2][s & 3], bv[ni][s >> 2][s & 3], acc[mi][ni], 0, 0, 0);

        if (kt + 1 < nk) sstore(buf ^ 1);
        __syncthreads();
    }

    // Epilogue.  Accumulator register r of lane l holds output row
    // 8*(r/4) + 4*(l/32) + r%4 and column l%32 of each 32x32 block.
#pragma unroll
    for (int mi = 0; mi < 2; ++mi) {
#pragma unroll
        for (int ni = 0; ni < 2; ++ni) {
            const int64_t gj = n0 + wc * 64 + ni * 32 + l32;
            const float nrm_j = (a.kernel == KKM_GAUSS && gj < a.n) ? a.nrm[gj] : 0.f;
#pragma unroll
            for (int rg = 0; rg < 4; ++rg) {
                const int64_t gi0 = m0 + wr * 64 + mi * 32 + 8 * rg + 4 * half;
                float v[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t gi = gi0 + r;
                    const float nrm_i = (a.kernel == KKM_GAUSS && gi < a.n) ? a.nrm[gi] : 0.f;
                    v[r] = kappa_from_dot(acc[mi][ni][4 * rg + r], nrm_i, nrm_j, a.kernel,
                                          a.gamma, a.coef0, a.degree);
                }
                if (gj >= a.n) continue;
                if (!diag_tile) {
                    // K[gi][gj]: lanes of a half write 32 consecutive floats of one row
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (gi0 + r < a.n) a.K[(gi0 + r) * a.ldk + gj] = v[r];
                    // mirror K[gj][gi0..gi0+3]: four consecutive floats of row gj
                    float *dst = a.K + gj * a.ldk + gi0;
                    if (a.vec_k && gi0 + 3 < a.n) {
                        f32x4 w = {v[0], v[1], v[2], v[3]};
                        *reinterpret_cast<f32x4 *>(dst) = w;
                    } else {
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            if (gi0 + r < a.n) dst[r] = v[r];
                    }
                } else {
                    // diagonal tile: the upper triangle is the source of truth
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int64_t gi = gi0 + r;
                        if (gi >= a.n || gi > gj) continue;
                        if (gi == gj) {
                            // kappa(x, x) = exp(0) = 1 exactly; a non-finite row stays visible
                            const float b = acc[mi][ni][4 * rg + r];
                            const float dv = (a.kernel == KKM_GAUSS)
                                                 ? (isfinite(b) ? 1.0f : __builtin_nanf(""))
                                                 : v[r];
                            a.K[gi * a.ldk + gi] = dv;
                            a.diag[gi] = dv;
                        } else {
                            a.K[gi * a.ldk + gj] = v[r];
                            a.K[gj * a.ldk + gi] = v[r];
                        }
                    }
                }
            }
        }
    }
}

// Squared row norms ||x_i||^2 for the Gaussian: one wave per row, fixed order.
__global__ __launch_bounds__(256) void row_sqnorms(const float *X, int64_t n, int64_t d,
                                                   int64_t ldx, float *nrm) {
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    const float *x = X + row * ldx;
    float s = 0.f;
    for (int64_t l = lane; l < d; l += kWave) s = fmaf(x[l], x[l], s);
    s = wave_sum(s);
    if (lane == 0) nrm[row] = s;
}

}  // namespace

size_t gram_workspace_bytes(int64_t n, int64_t d, int32_t gram_prec) {
    (void)d;
    (void)gram_prec;
    Carver c(nullptr);
    c.take<float>((size_t)n);  // squared norms
    return c.bytes();
}

kkm_status gram_launch(const float *X, int64_t n, int64_t d, int64_t ldx, int32_t kernel,
                       double gamma, double coef0, int32_t degree, int32_t gram_prec,
                       int32_t k_store, void *K, int64_t ldk, float *diagK, void *ws,
                       size_t ws_bytes, hipStream_t stream) {
    if (gram_prec != KKM_F32 || k_store != KKM_F32) {
        set_error("kkm_gram: gram_prec=%d k_store=%d not available in this build", gram_prec,
                  k_store);
        return KKM_ERR_UNSUPPORTED;
    }
    if (ws_bytes < gram_workspace_bytes(n, d, gram_prec) || (ws == nullptr && n > 0)) {
        set_error("kkm_gram: workspace of %zu bytes is smaller than %zu", ws_bytes,
                  gram_workspace_bytes(n, d, gram_prec));
        return KKM_ERR_NOMEM;
    }
    Carver c(ws);
    float *nrm = c.take<float>((size_t)n);
    if (kernel == KKM_GAUSS) {
        hipLaunchKernelGGL(row_sqnorms, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, stream, X, n,
                           d, ldx, nrm);
        KKM_HIP(hipGetLastError());
    }
    GramArgs a;
    a.X = X;
    a.n = n;
    a.d = d;
    a.ldx = ldx;
    a.kernel = kernel;
    a.gamma = (float)gamma;
    a.coef0 = (float)coef0;
    a.degree = degree;
    a.nrm = nrm;
    a.K = static_cast<float *>(K);
    a.ldk = ldk;
    a.diag = diagK;
    a.nb = (n + GM - 1) / GM;
    a.ntiles = a.nb * (a.nb + 1) / 2;
    a.per_xcd = (a.ntiles + 7) / 8;
    a.vec_x = ((ldx % 4) == 0) && ((reinterpret_cast<uintptr_t>(X) & 15) == 0);
    a.vec_k = ((ldk % 4) == 0) && ((reinterpret_cast<uintptr_t>(K) & 15) == 0);
    const int64_t grid = a.per_xcd * 8;
    if (grid > 0x7fffffff) {
        set_error("kkm_gram: n=%lld needs more than 2^31 tiles", (long long)n);
        return KKM_ERR_UNSUPPORTED;
    }
    const TimedSpan span = timing_begin(TK_GRAM, stream);
    hipLaunchKernelGGL(gram_f32_mfma, dim3((unsigned)grid), dim3(GTHREADS), 0, stream, a);
    KKM_HIP(hipGetLastError());
    timing_end(span, stream);
    return KKM_OK;
}

}  // namespace kkm
