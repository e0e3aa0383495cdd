// MFMA products for the learned feature map: 64 x 64 output tile per 256-thread
// workgroup, 4 waves as 2 x 2, each one 32 x 32 MFMA block; k staged in LDS in
// slabs of 32 as FP32 and rounded to the operand type when the fragments are
// built (bfloat16: round to nearest even; FP32: unchanged).
#include "gemm.h"

namespace kkm {

namespace {

constexpr int TM = 64, TK = 32, TLD = TK + 1;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ __bf16 to_bf16(float f) {
    return (__bf16)f;  // round to nearest even (one hardware conversion on gfx950)
}

__device__ __forceinline__ float gelu(float z) {
    return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_grad(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) +
           z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// Stage a 64 x 32 operand slab (rows r0.., k k0..) into LDS as [row][k].
template <bool KCONTIG>
__device__ __forceinline__ void stage(const float *P, int64_t ld, int64_t rows, int64_t K,
                                      int64_t r0, int64_t k0, float (*S)[TLD]) {
    const int t = threadIdx.x;
    if (KCONTIG) {
        const int r = t >> 2, c = (t & 3) * 8;  // 8 consecutive k of one row
        const int64_t gr = r0 + r;
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            const int64_t gk = k0 + c + v;
            S[r][c + v] = (gr < rows && gk < K) ? P[gr * ld + gk] : 0.f;
        }
    } else {
        const int kk = t >> 3, c = (t & 7) * 8;  // 8 consecutive rows of one k
        const int64_t gk = k0 + kk;
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            const int64_t gr = r0 + c + v;
            S[c + v][kk] = (gr < rows && gk < K) ? P[gk * ld + gr] : 0.f;
        }
    }
}

template <int OP, bool AK, bool BK>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g, int epi) {
    __shared__ float As[TM][TLD], Bs[TM][TLD];
    __shared__ double red[4];
    const int64_t m0 = (int64_t)blockIdx.y * TM, n0 = (int64_t)blockIdx.x * TM;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int half = lane >> 5, l32 = lane & 31;

    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;

    for (int64_t k0 = 0; k0 < g.K; k0 += TK) {
        stage<AK>(g.A, g.lda, g.M, g.K, m0, k0, As);
        stage<BK>(g.B, g.ldb, g.N, g.K, n0, k0, Bs);
        __syncthreads();
        const float *ra = As[wm * 32 + l32];
        const float *rb = Bs[wn * 32 + l32];
        if (OP == GEMM_BF16) {
            // lane half h supplies k = 8h .. 8h+7 of each 16-wide step (same for A and B)
#pragma unroll
            for (int s = 0; s < TK / 16; ++s) {
                bf16x8 x, y;
#pragma unroll
                for (int v = 0; v < 8; ++v) {
                    x[v] = to_bf16(ra[16 * s + 8 * half + v]);
                    y[v] = to_bf16(rb[16 * s + 8 * half + v]);
                }
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x, y, acc, 0, 0, 0);
            }
        } else {
#pragma unroll
            for (int s = 0; s < TK / 2; ++s)
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(ra[2 * s + half], rb[2 * s + half], acc,
                                                           0, 0, 0);
        }
        __syncthreads();
    }

    // accumulator register r of lane l: row 8*(r/4) + 4*(l/32) + r%4, column l%32
    double sq = 0.0;
    const int64_t n = n0 + wn * 32 + l32;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int64_t m = m0 + wm * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
        if (m >= g.M || n >= g.N) continue;
        const float v = g.alpha * acc[r];
        switch (epi) {
        case EPI_STORE:
            g.C[m * g.ldc + n] = v;
            break;
        case EPI_BIAS:
            g.C[m * g.ldc + n] = v + g.bias[n];
            break;
        case EPI_BIAS_GELU: {
            const float z = v + g.bias[n];
            if (g.C) g.C[m * g.ldc + n] = z;
            g.C2[m * g.ldc2 + n] = gelu(z);
            break;
        }
        case EPI_GELU_BWD:
            g.C[m * g.ldc + n] = v * gelu_grad(g.Zp[m * g.ldz + n]);
            break;
        default: {  // EPI_LOSS
            const float e = v - g.Kb[m * g.ldkb + n];
            g.C[m * g.ldc + n] = e;
            sq += (double)e * (double)e;
        }
        }
    }
    if (epi == EPI_LOSS) {
        sq = wave_sum(sq);
        if (lane == 0) red[wave] = sq;
        __syncthreads();
        if (tid == 0)
            g.part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
    }
}

// ---------------------------------------------------------------- wide tiles
//
// Both operands k-contiguous (A(m,k) = A[m*lda+k], B(n,k) = B[n*ldb+k]) and
// large: a 64 x 256 output tile per workgroup, wave w owning columns
// 64w .. 64w+63 as 2 x 2 blocks of 32 x 32.  k-slabs of 32 floats per row are
// loaded with 16-byte reads (element reads at ragged edges), staged in LDS as
// FP32 and prefetched one slab ahead in registers.  Within a slab the k index
// is permuted the same way for both operands, so each lane builds its
// fragments from 16 consecutive floats of its row (four b128 LDS reads):
// FP32 MFMA s takes k = 16h + s from lane half h; BF16 MFMA s (s = 0, 1) takes
// k = 16h + 8s .. 16h + 8s + 7.

constexpr int WM = 64, WN = 256, WLD = TK + 4;

struct WideLds {
    float a[WM][WLD];
    float b[WN][WLD];
};

__device__ __forceinline__ f32x4 load4(const float *P, int64_t ld, int64_t rows, int64_t K,
                                       int64_t r, int64_t k, bool vec) {
    f32x4 v = {0.f, 0.f, 0.f, 0.f};
    if (r < rows) {
        const float *src = P + r * ld + k;
        if (vec && k + 3 < K) {
            v = *reinterpret_cast<const f32x4 *>(src);
        } else {
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (k + u < K) v[u] = src[u];
        }
    }
    return v;
}

template <int OP>
__global__ __launch_bounds__(256, 2) void gemm_wide(GemmArgs g, int epi, int vec_a, int vec_b) {
    __shared__ __attribute__((aligned(16))) WideLds lds;
    __shared__ double red[4];
    const int64_t m0 = (int64_t)blockIdx.y * WM, n0 = (int64_t)blockIdx.x * WN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int half = lane >> 5, l32 = lane & 31;
    const int lr = tid >> 3, lc = (tid & 7) * 4;  // 8 threads x 4 floats per 32-float row slice

    f32x4 ra[2], rb[8];
    auto gload = [&](int64_t k0) {
#pragma unroll
        for (int u = 0; u < 2; ++u)
            ra[u] = load4(g.A, g.lda, g.M, g.K, m0 + lr + 32 * u, k0 + lc, vec_a);
#pragma unroll
        for (int u = 0; u < 8; ++u)
            rb[u] = load4(g.B, g.ldb, g.N, g.K, n0 + lr + 32 * u, k0 + lc, vec_b);
    };
    auto sstore = [&]() {
#pragma unroll
        for (int u = 0; u < 2; ++u) *reinterpret_cast<f32x4 *>(&lds.a[lr + 32 * u][lc]) = ra[u];
#pragma unroll
        for (int u = 0; u < 8; ++u) *reinterpret_cast<f32x4 *>(&lds.b[lr + 32 * u][lc]) = rb[u];
    };

    f32x16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    gload(0);
    for (int64_t k0 = 0; k0 < g.K; k0 += TK) {
        sstore();
        __syncthreads();
        if (k0 + TK < g.K) gload(k0 + TK);
        f32x4 av[2][4], bv[2][4];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const float *pa = &lds.a[i * 32 + l32][16 * half];
            const float *pb = &lds.b[wave * 64 + i * 32 + l32][16 * half];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                av[i][q] = *reinterpret_cast<const f32x4 *>(pa + 4 * q);
                bv[i][q] = *reinterpret_cast<const f32x4 *>(pb + 4 * q);
            }
        }
        if constexpr (OP == GEMM_BF16) {
            bf16x8 x[2][2], y[2][2];  // [block][s], each operand element rounded once
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int s = 0; s < 2; ++s)
#pragma unroll
                    for (int v = 0; v < 8; ++v) {
                        x[i][s][v] = to_bf16(av[i][2 * s + v / 4][v % 4]);
                        y[i][s][v] = to_bf16(bv[i][2 * s + v / 4][v % 4]);
                    }
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                    for (int ni = 0; ni < 2; ++ni)
                        acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x[mi][s], y[ni][s],
                                                                               acc[mi][ni], 0, 0, 0);
        } else {
#pragma unroll
            for (int s = 0; s < 16; ++s)
#pragma unroll
                for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                    for (int ni = 0; ni < 2; ++ni)
                        acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x2f32(
                            av[mi][s >> 2][s & 3], bv[ni][s >> 2][s & 3], acc[mi][ni], 0, 0, 0);
        }
        __syncthreads();
    }

    // accumulator register r of lane l: row 8*(r/4) + 4*(l/32) + r%4, column l%32
    double sq = 0.0;
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni) {
            const int64_t n = n0 + wave * 64 + ni * 32 + l32;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t m = m0 + mi * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
                if (m >= g.M || n >= g.N) continue;
                const float v = g.alpha * acc[mi][ni][r];
                switch (epi) {
                case EPI_STORE:
                    g.C[m * g.ldc + n] = v;
                    break;
                case EPI_BIAS:
                    g.C[m * g.ldc + n] = v + g.bias[n];
                    break;
                case EPI_BIAS_GELU: {
                    const float z = v + g.bias[n];
                    if (g.C) g.C[m * g.ldc + n] = z;
                    g.C2[m * g.ldc2 + n] = gelu(z);
                    break;
                }
                case EPI_GELU_BWD:
                    g.C[m * g.ldc + n] = v * gelu_grad(g.Zp[m * g.ldz + n]);
                    break;
                default: {  // EPI_LOSS
                    const float e = v - g.Kb[m * g.ldkb + n];
                    g.C[m * g.ldc + n] = e;
                    sq += (double)e * (double)e;
                }
                }
            }
        }
    if (epi == EPI_LOSS) {
        sq = wave_sum(sq);
        if (lane == 0) red[wave] = sq;
        __syncthreads();
        if (tid == 0)
            g.part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
    }
}

// Products that take the wide tiles: both operands k-contiguous, no loss
// epilogue (its per-workgroup sums are laid out for 64 x 64 tiles), and large.
bool gemm_wide_fits(bool ak, bool bk, GemmEpi epi, const GemmArgs &g) {
    return ak && bk && epi != EPI_LOSS && g.M >= 32 && g.N >= 256 && g.M * g.N >= (1 << 20);
}

}  // namespace

kkm_status gemm_launch(GemmOp op, bool ak, bool bk, GemmEpi epi, const GemmArgs &g,
                       hipStream_t stream) {
    if (g.M <= 0 || g.N <= 0) return KKM_OK;
    if (gemm_wide_fits(ak, bk, epi, g)) {
        const dim3 grid((unsigned)((g.N + WN - 1) / WN), (unsigned)((g.M + WM - 1) / WM));
        const int va = ((g.lda & 3) == 0) && ((reinterpret_cast<uintptr_t>(g.A) & 15) == 0);
        const int vb = ((g.ldb & 3) == 0) && ((reinterpret_cast<uintptr_t>(g.B) & 15) == 0);
        if (op == GEMM_BF16)
            hipLaunchKernelGGL(gemm_wide<GEMM_BF16>, grid, dim3(256), 0, stream, g, (int)epi, va, vb);
        else
            hipLaunchKernelGGL(gemm_wide<GEMM_F32>, grid, dim3(256), 0, stream, g, (int)epi, va, vb);
        KKM_HIP(hipGetLastError());
        return KKM_OK;
    }
    const dim3 grid((unsigned)((g.N + TM - 1) / TM), (unsigned)((g.M + TM - 1) / TM));
    const dim3 blk(256);
    const int e = (int)epi;
#define KKM_GEMM(OPV, AKV, BKV) \
    hipLaunchKernelGGL((gemm_kernel<OPV, AKV, BKV>), grid, blk, 0, stream, g, e)
    if (op == GEMM_BF16) {
        if (ak && bk) KKM_GEMM(GEMM_BF16, true, true);
        else if (ak && !bk) KKM_GEMM(GEMM_BF16, true, false);
        else if (!ak && bk) KKM_GEMM(GEMM_BF16, false, true);
        else KKM_GEMM(GEMM_BF16, false, false);
    } else {
        if (ak && bk) KKM_GEMM(GEMM_F32, true, true);
        else if (ak && !bk) KKM_GEMM(GEMM_F32, true, false);
        else if (!ak && bk) KKM_GEMM(GEMM_F32, false, true);
        else KKM_GEMM(GEMM_F32, false, false);
    }
#undef KKM_GEMM
    KKM_HIP(hipGetLastError());
    return KKM_OK;
}

}  // namespace kkm
