// Dense products C[m][n] = alpha * sum_k A(m,k) B(n,k) on MFMA with FP32
// accumulation, used by the learned feature map and the feature-space Lloyd
// iterations.  Internal to the library.
#pragma once

#include "kkm_common.h"

namespace kkm {

enum GemmOp { GEMM_BF16 = 0, GEMM_F32 = 1 };
enum GemmEpi {
    EPI_STORE = 0,      // C = alpha * acc
    EPI_BIAS = 1,       // C = alpha * acc + bias[n]
    EPI_BIAS_GELU = 2,  // Z = alpha * acc + bias[n]; C = Z (if C), C2 = GELU(Z)
    EPI_GELU_BWD = 3,   // C = alpha * acc * GELU'(Zp[m][n])
    EPI_LOSS = 4        // C = alpha * acc - Kb[m][n]; per-workgroup sum of C^2 (FP64)
};

struct GemmArgs {
    const float *A;
    int64_t lda;
    const float *B;
    int64_t ldb;
    int64_t M, N, K;
    float alpha;
    float *C;
    int64_t ldc;
    const float *bias;
    float *C2;
    int64_t ldc2;
    const float *Zp;
    int64_t ldz;
    const float *Kb;
    int64_t ldkb;
    double *part;  // [gridDim.x * gridDim.y]
};

// a_kcontig: A(m,k) = A[m*lda + k], else A[k*lda + m]; likewise b_kcontig for B(n,k).
kkm_status gemm_launch(GemmOp op, bool a_kcontig, bool b_kcontig, GemmEpi epi, const GemmArgs &g,
                       hipStream_t stream);

inline int64_t gemm_tiles(int64_t M, int64_t N) { return ((M + 63) / 64) * ((N + 63) / 64); }

}  // namespace kkm
