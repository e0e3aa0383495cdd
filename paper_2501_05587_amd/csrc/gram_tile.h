// Device-side pieces of the kernel-matrix product shared by the single- and
// many-instance Gram kernels: the 128 x 128 tile of the FP32 and of the
// BF16 / FP8 MFMA product with its fused epilogue (kappa, diagonal, mirrored
// stores), the 256 x 256 BF16 / FP8 tile (selectable, not the default), the
// launch order of the tiles, and the row prologues (squared norm; rounding to
// the product's input type).  Internal to the library.
#pragma once

#include <type_traits>

#include "kkm_common.h"

namespace kkm {
namespace gt {

constexpr int GM = 128;       // tile edge (rows = columns)
constexpr int GTHREADS = 256; // 4 waves as 2 x 2, each owns a 64 x 64 sub-tile

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    // round to nearest even (one hardware conversion on gfx950); a NaN stays a NaN
    const __bf16 h = (__bf16)f;
    uint16_t u;
    __builtin_memcpy(&u, &h, 2);
    return u;
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ---------------------------------------------------------------- shared epilogue

struct Epi {
    int64_t n, ldk;
    int kernel;
    float gamma, coef0;  // Gaussian: gamma * log2(e), see epi_gamma
    int degree;
    const float *nrm;    // squared norms (Gaussian)
    const float *scale;  // per-row scales (FP8), else null
    void *K;
    float *diag;
    int vec_k;           // K rows aligned for 4-element stores
    int plgw;            // strip-packed layout: log2 of the strip width (0: rows of stride ldk)
    int64_t pns;         // strip-packed layout: strips
};

// Offset of K[i][j] (j at or right of the start of i's strip when packed).
__device__ __forceinline__ int64_t k_index(const Epi &e, int64_t i, int64_t j) {
    if (e.plgw == 0) return i * e.ldk + j;
    return packed_row_offset(i, e.plgw, e.pns) + (j - ((i >> e.plgw) << e.plgw));
}

// Whether the mirrored block K[j][i] of tile (rows m0.., columns n0..) is
// stored: always for rows of stride ldk, only inside a strip when packed.
__device__ __forceinline__ bool mirror_stored(const Epi &e, int64_t m0, int64_t n0) {
    return e.plgw == 0 || (m0 >> e.plgw) == (n0 >> e.plgw);
}

// The kernel's gamma as the epilogue takes it: for the Gaussian, gamma log2(e)
// (rounded once, from double), so that exp(-gamma s) = 2^(-gamma log2(e) s) is
// one multiply and the hardware base-2 exponential.
inline float epi_gamma(int kernel, double gamma) {
    return (float)(kernel == KKM_GAUSS ? gamma * 1.4426950408889634074 : gamma);
}

__device__ __forceinline__ float kappa_from_dot(float b, float ni, float nj, int kernel,
                                                float gamma, float coef0, int degree) {
    if (kernel == KKM_GAUSS) {
        float sq = fmaxf(ni + nj - 2.0f * b, 0.0f);
        return __builtin_amdgcn_exp2f(-gamma * sq);
    }
    if (kernel == KKM_POLY) {
        float t = fmaf(gamma, b, coef0);
        float v = t;
        for (int r = 1; r < degree; ++r) v *= t;
        return v;
    }
    return b;
}

// K leaves through non-temporal stores: it is written once and not read back
// by the kernel, so its lines should not displace the operand rows in the
// caches (measured 80 -> 75 ms for the BF16 product with bfloat16 K at
// n=200000, d=1024).
template <typename OUT> struct Store;
template <> struct Store<float> {
    static __device__ __forceinline__ float round(float v) { return v; }
    static __device__ __forceinline__ void one(void *K, int64_t idx, float v) {
        static_cast<float *>(K)[idx] = v;
    }
    static __device__ __forceinline__ void four(void *K, int64_t idx, const float v[4]) {
        f32x4 w = {v[0], v[1], v[2], v[3]};
        __builtin_nontemporal_store(w, reinterpret_cast<f32x4 *>(static_cast<float *>(K) + idx));
    }
};
template <> struct Store<uint16_t> {
    static __device__ __forceinline__ float round(float v) { return bf16_to_f32(f32_to_bf16(v)); }
    static __device__ __forceinline__ void one(void *K, int64_t idx, float v) {
        static_cast<uint16_t *>(K)[idx] = f32_to_bf16(v);
    }
    static __device__ __forceinline__ void four(void *K, int64_t idx, const float v[4]) {
        typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
        const f32x4 f = {v[0], v[1], v[2], v[3]};
        const bf16x4 b = __builtin_convertvector(f, bf16x4);
        __builtin_nontemporal_store(__builtin_bit_cast(uint64_t, b),
                                    reinterpret_cast<uint64_t *>(static_cast<uint16_t *>(K) + idx));
    }
};

// Row stride (floats) of the tile staged in LDS by the epilogue: the pad
// spreads the 16-byte accesses of lanes holding consecutive rows over all banks.
constexpr int TS = GM + 4;
// LDS the epilogue stages through: the whole tile, or half of it at a time
constexpr size_t epi_lds_bytes(int halves) { return sizeof(float) * (GM / halves) * TS; }

// Rows r = 0..ROWS-1 of the staged tile T to K[row0 + r][col0 .. col0 + 127],
// skipping rows and columns at or past n: each thread stores 4 columns of
// every eighth row, reading B rows from LDS before it waits (B = 4 when half
// a tile is staged: the half-tile epilogue keeps its accumulators live across
// the passes, and eight rows in flight made it spill registers to memory).
template <typename OUT, int ROWS = GM, int B = (ROWS == GM ? 8 : 4)>
__device__ __forceinline__ void store_rows(const Epi &e, const float *T, int64_t row0, int64_t col0) {
    const int tid = threadIdx.x;
    const int c4 = (tid & 31) * 4;
    const int64_t gj0 = col0 + c4;
    if (gj0 >= e.n) return;
    const bool vec = e.vec_k && gj0 + 3 < e.n;
#pragma unroll
    for (int h = 0; h < ROWS / (8 * B); ++h) {
        f32x4 w[B];
#pragma unroll
        for (int it = 0; it < B; ++it)
            w[it] = *reinterpret_cast<const f32x4 *>(T + ((tid >> 5) + 8 * (B * h + it)) * TS + c4);
#pragma unroll
        for (int it = 0; it < B; ++it) {
            const int64_t gi = row0 + (tid >> 5) + 8 * (B * h + it);
            if (gi >= e.n) continue;
            const float v[4] = {w[it][0], w[it][1], w[it][2], w[it][3]};
            const int64_t idx = k_index(e, gi, gj0);
            if (vec) {
                Store<OUT>::four(e.K, idx, v);
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (gj0 + r < e.n) Store<OUT>::one(e.K, idx + r, v[r]);
            }
        }
    }
}

// The whole tile staged as bfloat16 (bfloat16 K and the half-tile epilogue:
// it fits where half of it fits as FP32): row stride in elements, bytes.
constexpr int TS16 = GM + 8;
constexpr size_t epi_lds_bytes_bf16 = sizeof(uint16_t) * GM * TS16;

// The bfloat16 tile T16 to K[row0 + r][col0 .. col0 + 127], skipping rows and
// columns at or past n: each thread stores 8 columns (16 bytes) of every
// sixteenth row, reading 4 rows from LDS before it waits.
__device__ __forceinline__ void store_rows_bf16(const Epi &e, const uint16_t *T16, int64_t row0,
                                                int64_t col0) {
    const int tid = threadIdx.x;
    const int c8 = (tid & 15) * 8;
    const int64_t gj0 = col0 + c8;
    if (gj0 >= e.n) return;
    const bool full = gj0 + 7 < e.n;
    uint16_t *K16 = static_cast<uint16_t *>(e.K);
    constexpr int B = 4;
#pragma unroll
    for (int h = 0; h < GM / (16 * B); ++h) {
        uint4 w[B];
#pragma unroll
        for (int it = 0; it < B; ++it)
            w[it] = *reinterpret_cast<const uint4 *>(T16 + ((tid >> 4) + 16 * (B * h + it)) * TS16 + c8);
#pragma unroll
        for (int it = 0; it < B; ++it) {
            const int64_t gi = row0 + (tid >> 4) + 16 * (B * h + it);
            if (gi >= e.n) continue;
            uint16_t *dst = K16 + k_index(e, gi, gj0);
            if (full && (reinterpret_cast<uintptr_t>(dst) & 15) == 0) {
                typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
                const u32x4 v = {w[it].x, w[it].y, w[it].z, w[it].w};
                __builtin_nontemporal_store(v, reinterpret_cast<u32x4 *>(dst));
            } else {
                const uint32_t q[4] = {w[it].x, w[it].y, w[it].z, w[it].w};
#pragma unroll
                for (int r = 0; r < 8; ++r)
                    if (gj0 + r < e.n) dst[r] = (uint16_t)((r & 1) ? (q[r >> 1] >> 16) : (q[r >> 1] & 0xFFFFu));
            }
        }
    }
}

// The squared norms (and FP8 row scales) of a tile's 128 rows and 128
// columns, staged in LDS when the tile starts so that their loads overlap the
// product: [0, 128) rows m0.., [128, 256) rows n0...  Needs a barrier before
// the epilogue reads them (the main loop has several).
__device__ __forceinline__ void stage_norms(const Epi &e, int64_t m0, int64_t n0, float *rn,
                                            float *rs) {
    const int t = threadIdx.x;
    const int64_t g = (t < GM) ? m0 + t : n0 + (t - GM);
    const bool in = g < e.n;
    rn[t] = (e.kernel == KKM_GAUSS && in) ? e.nrm[g] : 0.f;
    rs[t] = (e.scale && in) ? e.scale[g] : 1.f;
}

// Writes the 128 x 128 tile held by the four waves (each a 64 x 64 sub-tile as
// 2 x 2 blocks of 32 x 32 accumulators).  Accumulator register r of lane l
// holds output row 8*(r/4) + 4*(l/32) + r%4 and column l%32 of its block.
//
// Off the diagonal kappa replaces the accumulators in place, then the tile
// goes through `T` twice, transposed for K[j][i] and as is for K[i][j], so
// that both leave as whole rows of 4-element vector stores; HALVES = 2 stages
// half of the tile at a time (64 columns of the transposed pass, 64 rows of
// the other, by the two waves that hold them).  `T` (epi_lds_bytes(HALVES))
// may alias the operand buffers: the caller's last barrier has retired every
// read of them.  The trailing barrier retires every read of `T`, `rn` and `rs`
// before the workgroup's next tile.
//
// FULL (every tile of the square is launched, the GEMM shape of the product):
// each tile writes only its own block K[i][j], through `T` as is; a diagonal
// tile also writes diag(K).  Tile (j, i) multiplies the same products in the
// same order as tile (i, j), so K is still exactly symmetric.
template <typename OUT, bool FULL, int HALVES = 1>
__device__ __forceinline__ void epilogue(const Epi &e, f32x16 (&acc)[2][2], int64_t m0,
                                         int64_t n0, bool diag_tile, int wr, int wc, int lane,
                                         float *T, const float *rn, const float *rs) {
    static_assert(HALVES == 1 || HALVES == 2, "whole tile or halves");
    constexpr int RH = GM / HALVES;  // rows of T staged at a time
    const int half = lane >> 5, l32 = lane & 31;
    if constexpr (HALVES == 1) {
        if constexpr (FULL) {
#pragma unroll
            for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                for (int ni = 0; ni < 2; ++ni) {
                    const int jj = wc * 64 + ni * 32 + l32;
                    const float nrm_j = rn[GM + jj], s_j = rs[GM + jj];
#pragma unroll
                    for (int rg = 0; rg < 4; ++rg) {
                        const int ii0 = wr * 64 + mi * 32 + 8 * rg + 4 * half;
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            float b = acc[mi][ni][4 * rg + r];
                            if (e.scale) b *= rs[ii0 + r] * s_j;
                            float v = kappa_from_dot(b, rn[ii0 + r], nrm_j, e.kernel, e.gamma,
                                                     e.coef0, e.degree);
                            if (diag_tile && ii0 + r == jj) {
                                // kappa(x, x) = exp(0) = 1 exactly; a non-finite row stays visible
                                v = (e.kernel == KKM_GAUSS) ? (isfinite(b) ? 1.0f : __builtin_nanf(""))
                                                            : Store<OUT>::round(v);
                                if (m0 + jj < e.n) e.diag[m0 + jj] = v;
                            }
                            T[(ii0 + r) * TS + jj] = v;
                        }
                    }
                }
            __syncthreads();
            store_rows<OUT>(e, T, m0, n0);  // rows and columns may pass n
            __syncthreads();
            return;
        }
        if (!diag_tile) {
#pragma unroll
            for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                for (int ni = 0; ni < 2; ++ni) {
                    const int jj = wc * 64 + ni * 32 + l32;
                    const float nrm_j = rn[GM + jj], s_j = rs[GM + jj];
#pragma unroll
                    for (int rg = 0; rg < 4; ++rg) {
                        const int ii0 = wr * 64 + mi * 32 + 8 * rg + 4 * half;
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            float b = acc[mi][ni][4 * rg + r];
                            if (e.scale) b *= rs[ii0 + r] * s_j;
                            acc[mi][ni][4 * rg + r] = kappa_from_dot(b, rn[ii0 + r], nrm_j, e.kernel,
                                                                     e.gamma, e.coef0, e.degree);
                        }
                        // transposed: T[jj][ii0 .. ii0+3]
                        const f32x4 w = {acc[mi][ni][4 * rg], acc[mi][ni][4 * rg + 1],
                                         acc[mi][ni][4 * rg + 2], acc[mi][ni][4 * rg + 3]};
                        *reinterpret_cast<f32x4 *>(T + jj * TS + ii0) = w;
                    }
                }
            __syncthreads();
            // K[n0 + jj][m0 ..]; off the diagonal m0 + 127 < n0
            if (mirror_stored(e, m0, n0)) store_rows<OUT>(e, T, n0, m0);
            __syncthreads();
            // as is: T[ii][jj]
#pragma unroll
            for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                for (int ni = 0; ni < 2; ++ni) {
                    const int jj = wc * 64 + ni * 32 + l32;
#pragma unroll
                    for (int rg = 0; rg < 4; ++rg) {
                        const int ii0 = wr * 64 + mi * 32 + 8 * rg + 4 * half;
#pragma unroll
                        for (int r = 0; r < 4; ++r) T[(ii0 + r) * TS + jj] = acc[mi][ni][4 * rg + r];
                    }
                }
            __syncthreads();
            store_rows<OUT>(e, T, m0, n0);  // K[m0 + ii][n0 ..]: every row exists; columns may pass n
            __syncthreads();
            return;
        }
    } else {
        if constexpr (FULL) {
            // as is, RH rows at a time (in halves: the waves with wr == h hold them)
#pragma unroll
            for (int h = 0; h < HALVES; ++h) {
                if (HALVES == 1 || wr == h) {
#pragma unroll
                    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                        for (int ni = 0; ni < 2; ++ni) {
                            const int jj = wc * 64 + ni * 32 + l32;
                            const float nrm_j = rn[GM + jj], s_j = rs[GM + jj];
#pragma unroll
                            for (int rg = 0; rg < 4; ++rg) {
                                const int ii0 = wr * 64 + mi * 32 + 8 * rg + 4 * half;
#pragma unroll
                                for (int r = 0; r < 4; ++r) {
                                    float b = acc[mi][ni][4 * rg + r];
                                    if (e.scale) b *= rs[ii0 + r] * s_j;
                                    float v = kappa_from_dot(b, rn[ii0 + r], nrm_j, e.kernel, e.gamma,
                                                             e.coef0, e.degree);
                                    if (diag_tile && ii0 + r == jj) {
                                        // kappa(x, x) = exp(0) = 1 exactly; a non-finite row stays visible
                                        v = (e.kernel == KKM_GAUSS)
                                                ? (isfinite(b) ? 1.0f : __builtin_nanf(""))
                                                : Store<OUT>::round(v);
                                        if (m0 + jj < e.n) e.diag[m0 + jj] = v;
                                    }
                                    T[(ii0 - RH * h + r) * TS + jj] = v;
                                }
                            }
                        }
                }
                __syncthreads();
                store_rows<OUT, RH>(e, T, m0 + RH * h, n0);  // rows and columns may pass n
                __syncthreads();
            }
            return;
        }
        if (!diag_tile) {
#pragma unroll
            for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                for (int ni = 0; ni < 2; ++ni) {
                    const int jj = wc * 64 + ni * 32 + l32;
                    const float nrm_j = rn[GM + jj], s_j = rs[GM + jj];
#pragma unroll
                    for (int rg = 0; rg < 4; ++rg) {
                        const int ii0 = wr * 64 + mi * 32 + 8 * rg + 4 * half;
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            float b = acc[mi][ni][4 * rg + r];
                            if (e.scale) b *= rs[ii0 + r] * s_j;
                            acc[mi][ni][4 * rg + r] = kappa_from_dot(b, rn[ii0 + r], nrm_j, e.kernel,
                                                                     e.gamma, e.coef0, e.degree);
                        }
                    }
                }
            // bfloat16 K: the values are rounded to bfloat16 here (the stores round
            // them anyway, and rounding an exact bfloat16 value again changes no bit)
            // and kept two per register through the passes below; with the FP32
            // accumulators live across them the kernel spilled registers to memory
            constexpr bool PACK = sizeof(OUT) == 2;
            uint32_t kb[2][2][PACK ? 8 : 1];
            if constexpr (PACK) {
                typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
                typedef float f32x2 __attribute__((ext_vector_type(2)));
#pragma unroll
                for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
                        for (int t = 0; t < 8; ++t) {
                            const f32x2 f = {acc[mi][ni][2 * t], acc[mi][ni][2 * t + 1]};
                            kb[mi][ni][t] = __builtin_bit_cast(uint32_t, __builtin_convertvector(f, bf16x2));
                        }
            }
            if constexpr (PACK && HALVES == 2) {
                // the whole tile staged as bfloat16: one round per pass, each
                // lane's four rows of a column leaving as one 8-byte LDS write
                // in the transposed pass
                uint16_t *T16 = reinterpret_cast<uint16_t *>(T);
                if (mirror_stored(e, m0, n0)) {  // uniform: a packed K outside a strip skips it
#pragma unroll
                    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                        for (int ni = 0; ni < 2; ++ni) {
                            const int jj = wc * 64 + ni * 32 + l32;
#pragma unroll
                            for (int rg = 0; rg < 4; ++rg) {
                                const int ii0 = wr * 64 + mi * 32 + 8 * rg + 4 * half;
                                *reinterpret_cast<uint2 *>(T16 + jj * TS16 + ii0) =
                                    make_uint2(kb[mi][ni][2 * rg], kb[mi][ni][2 * rg + 1]);
                            }
                        }
                    __syncthreads();
                    store_rows_bf16(e, T16, n0, m0);  // K[n0 + jj][m0 ..]; m0 + 127 < n0
                    __syncthreads();
                }
#pragma unroll
                for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                    for (int ni = 0; ni < 2; ++ni) {
                        const int jj = wc * 64 + ni * 32 + l32;
#pragma unroll
                        for (int rg = 0; rg < 4; ++rg) {
                            const int ii0 = wr * 64 + mi * 32 + 8 * rg + 4 * half;
#pragma unroll
                            for (int r = 0; r < 4; ++r) {
                                const uint32_t w = kb[mi][ni][(4 * rg + r) >> 1];
                                T16[(ii0 + r) * TS16 + jj] = (uint16_t)((r & 1) ? (w >> 16) : (w & 0xFFFFu));
                            }
                        }
                    }
                __syncthreads();
                store_rows_bf16(e, T16, m0, n0);  // every row exists; columns may pass n
                __syncthreads();
                return;
            }
            auto kept = [&](int mi, int ni, int idx) -> float {
                if constexpr (PACK) {
                    const uint32_t w = kb[mi][ni][idx >> 1];
                    return __uint_as_float((idx & 1) ? (w & 0xFFFF0000u) : (w << 16));
                } else {
                    return acc[mi][ni][idx];
                }
            };
            // transposed, RH columns at a time (in halves: the waves with wc == h
            // hold them): T[jj - RH h][ii], then rows K[n0 + jj][m0 ..]; off the
            // diagonal m0 + 127 < n0
#pragma unroll
            for (int h = 0; h < HALVES; ++h) {
                if (!mirror_stored(e, m0, n0)) break;  // uniform: a packed K outside a strip
                if (HALVES == 1 || wc == h) {
#pragma unroll
                    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                        for (int ni = 0; ni < 2; ++ni) {
                            const int jl = wc * 64 + ni * 32 + l32 - RH * h;
#pragma unroll
                            for (int rg = 0; rg < 4; ++rg) {
                                const int ii0 = wr * 64 + mi * 32 + 8 * rg + 4 * half;
                                const f32x4 w = {kept(mi, ni, 4 * rg), kept(mi, ni, 4 * rg + 1),
                                                 kept(mi, ni, 4 * rg + 2), kept(mi, ni, 4 * rg + 3)};
                                *reinterpret_cast<f32x4 *>(T + jl * TS + ii0) = w;
                            }
                        }
                }
                __syncthreads();
                store_rows<OUT, RH>(e, T, n0 + RH * h, m0);
                __syncthreads();
            }
            // as is, RH rows at a time: every row exists; columns may pass n
#pragma unroll
            for (int h = 0; h < HALVES; ++h) {
                if (HALVES == 1 || wr == h) {
#pragma unroll
                    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                        for (int ni = 0; ni < 2; ++ni) {
                            const int jj = wc * 64 + ni * 32 + l32;
#pragma unroll
                            for (int rg = 0; rg < 4; ++rg) {
                                const int il0 = wr * 64 + mi * 32 + 8 * rg + 4 * half - RH * h;
#pragma unroll
                                for (int r = 0; r < 4; ++r)
                                    T[(il0 + r) * TS + jj] = kept(mi, ni, 4 * rg + r);
                            }
                        }
                }
                __syncthreads();
                store_rows<OUT, RH>(e, T, m0 + RH * h, n0);
                __syncthreads();
            }
            return;
        }
    }
    // diagonal tile: the upper triangle is the source of truth
#pragma unroll
    for (int mi = 0; mi < 2; ++mi) {
#pragma unroll
        for (int ni = 0; ni < 2; ++ni) {
            const int jj = wc * 64 + ni * 32 + l32;
            const int64_t gj = n0 + jj;
            const float nrm_j = rn[GM + jj], s_j = rs[GM + jj];
#pragma unroll
            for (int rg = 0; rg < 4; ++rg) {
                const int ii0 = wr * 64 + mi * 32 + 8 * rg + 4 * half;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t gi = m0 + ii0 + r;
                    if (gj >= e.n || gi >= e.n || gi > gj) continue;
                    float b = acc[mi][ni][4 * rg + r];
                    if (e.scale) b *= rs[ii0 + r] * s_j;
                    const float v = kappa_from_dot(b, rn[ii0 + r], nrm_j, e.kernel, e.gamma,
                                                   e.coef0, e.degree);
                    if (gi == gj) {
                        // kappa(x, x) = exp(0) = 1 exactly; a non-finite row stays visible
                        const float dv = (e.kernel == KKM_GAUSS)
                                             ? (isfinite(b) ? 1.0f : __builtin_nanf(""))
                                             : Store<OUT>::round(v);
                        Store<OUT>::one(e.K, k_index(e, gi, gi), dv);
                        e.diag[gi] = dv;
                    } else {
                        Store<OUT>::one(e.K, k_index(e, gi, gj), v);
                        Store<OUT>::one(e.K, k_index(e, gj, gi), v);
                    }
                }
            }
        }
    }
    __syncthreads();
}

// The off-diagonal epilogue for tiles whose accumulators must stay where the
// product left them (the 256 x 256 tile holds all 256 accumulator registers
// of a lane): kappa is computed for the transposed pass and again, from the
// same accumulators with the same operations, for the pass as is.  Same
// stores as the off-diagonal branch of `epilogue`; a diagonal tile goes
// through `epilogue` (its diagonal branch only reads the accumulators).
template <typename OUT>
__device__ __forceinline__ void epilogue_keep(const Epi &e, f32x16 (&acc)[2][2], int64_t m0,
                                              int64_t n0, bool diag_tile, int wr, int wc,
                                              int lane, float *T, const float *rn,
                                              const float *rs) {
    if (diag_tile) {
        epilogue<OUT, false>(e, acc, m0, n0, true, wr, wc, lane, T, rn, rs);
        return;
    }
    const int half = lane >> 5, l32 = lane & 31;
    auto kap = [&](int mi, int ni, int rg, int r, float nrm_j, float s_j) {
        const int ii = wr * 64 + mi * 32 + 8 * rg + 4 * half + r;
        float b = acc[mi][ni][4 * rg + r];
        if (e.scale) b *= rs[ii] * s_j;
        return kappa_from_dot(b, rn[ii], nrm_j, e.kernel, e.gamma, e.coef0, e.degree);
    };
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni) {
            const int jj = wc * 64 + ni * 32 + l32;
            const float nrm_j = rn[GM + jj], s_j = rs[GM + jj];
#pragma unroll
            for (int rg = 0; rg < 4; ++rg) {
                const int ii0 = wr * 64 + mi * 32 + 8 * rg + 4 * half;
                const f32x4 w = {kap(mi, ni, rg, 0, nrm_j, s_j), kap(mi, ni, rg, 1, nrm_j, s_j),
                                 kap(mi, ni, rg, 2, nrm_j, s_j), kap(mi, ni, rg, 3, nrm_j, s_j)};
                *reinterpret_cast<f32x4 *>(T + jj * TS + ii0) = w;
            }
        }
    __syncthreads();
    // K[n0 + jj][m0 ..]; off the diagonal m0 + 127 < n0
    if (mirror_stored(e, m0, n0)) store_rows<OUT>(e, T, n0, m0);
    __syncthreads();
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni) {
            const int jj = wc * 64 + ni * 32 + l32;
            const float nrm_j = rn[GM + jj], s_j = rs[GM + jj];
#pragma unroll
            for (int rg = 0; rg < 4; ++rg) {
                const int ii0 = wr * 64 + mi * 32 + 8 * rg + 4 * half;
#pragma unroll
                for (int r = 0; r < 4; ++r) T[(ii0 + r) * TS + jj] = kap(mi, ni, rg, r, nrm_j, s_j);
            }
        }
    __syncthreads();
    store_rows<OUT>(e, T, m0, n0);  // K[m0 + ii][n0 ..]: every row exists; columns may pass n
    __syncthreads();
}

// Upper-triangle tile t -> (bi, bj), bi <= bj, column by column.
__device__ __forceinline__ void tile_coords(int64_t t, int64_t &bi, int64_t &bj) {
    int64_t j = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while (j * (j + 1) / 2 > t) --j;
    while ((j + 1) * (j + 2) / 2 <= t) ++j;
    bj = j;
    bi = t - j * (j + 1) / 2;
}

// Launch order of the tiles.  Positions walk g x g groups of tiles (g a power
// of two): the upper triangle of groups column by column, each group column
// by column.  A position whose tile lies below the diagonal or past the edge
// has no tile.  Workgroups are dealt to the 8 XCDs round-robin; each XCD gets
// a contiguous range of positions, so the tiles one XCD runs together share
// 2g operand panels in its L2 instead of one panel per tile.
struct TileOrder {
    int64_t nb;        // tiles per side
    int64_t G;         // groups per side, ceil(nb / g)
    int64_t npos;      // positions: G (G + 1) / 2 * g^2 (triangle) or G^2 g^2 (full)
    int64_t per_xcd;   // positions per XCD
    int lg;            // log2 g
    int full;          // every tile of the square (else the upper triangle)
};

inline TileOrder tile_order(int64_t n, int lg, bool full = false, int tile = GM) {
    TileOrder o;
    o.nb = (n + tile - 1) / tile;
    o.lg = lg;
    o.full = full;
    o.G = (o.nb + (int64_t(1) << lg) - 1) >> lg;
    o.npos = (full ? o.G * o.G : o.G * (o.G + 1) / 2) << (2 * lg);
    o.per_xcd = (o.npos + 7) / 8;
    return o;
}

__device__ __forceinline__ bool tile_of_block(const TileOrder &o, int64_t &bi, int64_t &bj) {
    const int64_t pid = blockIdx.x;
    const int64_t t = (pid % 8) * o.per_xcd + pid / 8;
    if (t >= o.npos) return false;
    int64_t I, J;
    if (o.full) {
        const int64_t sgrp = t >> (2 * o.lg);
        I = sgrp % o.G;
        J = sgrp / o.G;
        const int64_t w = t & ((int64_t(1) << (2 * o.lg)) - 1);
        bi = (I << o.lg) + (w & ((int64_t(1) << o.lg) - 1));
        bj = (J << o.lg) + (w >> o.lg);
        return bi < o.nb && bj < o.nb;
    }
    tile_coords(t >> (2 * o.lg), I, J);
    const int64_t w = t & ((int64_t(1) << (2 * o.lg)) - 1);
    const int64_t g1 = (int64_t(1) << o.lg) - 1;
    bi = (I << o.lg) + (w & g1);
    bj = (J << o.lg) + (w >> o.lg);
    return bi <= bj && bj < o.nb;
}

// ---------------------------------------------------------------- FP32 product

constexpr int GK = 32;        // k-slab staged in LDS per step (floats)
constexpr int GLD = GK + 4;   // padded LDS row stride in floats (conflict-free b128 reads)

struct F32Tile {
    const float *X;
    int64_t d, ldx;
    int vec_x;  // rows 16-byte aligned
    Epi e;
};

struct F32Lds {
    float op[2][2][GM * GLD];  // operand slabs, double-buffered
    float rn[2 * GM], rs[2 * GM];
};

__device__ __forceinline__ f32x4 load_row4(const F32Tile &a, int64_t row, int64_t col) {
    f32x4 v = {0.f, 0.f, 0.f, 0.f};
    if (row < a.e.n) {
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

// One 128 x 128 tile (bi, bj) of the FP32 product and its epilogue.
template <typename OUT, bool FULL = false>
__device__ __forceinline__ void f32_tile(const F32Tile &a, int64_t bi, int64_t bj, F32Lds &lds) {
    const int64_t m0 = bi * GM, n0 = bj * GM;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int ld_row = tid >> 3;        // 8 threads per 32-float row slice
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
            *reinterpret_cast<f32x4 *>(&lds.op[buf][0][(ld_row + 32 * u) * GLD + ld_col]) = ra[u];
            *reinterpret_cast<f32x4 *>(&lds.op[buf][1][(ld_row + 32 * u) * GLD + ld_col]) = rb[u];
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
    stage_norms(a.e, m0, n0, lds.rn, lds.rs);
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
        const float *As = lds.op[buf][0];
        const float *Bs = lds.op[buf][1];
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
    static_assert(sizeof(lds.op) >= epi_lds_bytes(1), "epilogue tile does not fit");
    epilogue<OUT, FULL>(a.e, acc, m0, n0, bi == bj, wr, wc, lane, &lds.op[0][0][0], lds.rn, lds.rs);
}

// Squared norm of one FP32 row (Gaussian, FP32 product), by one whole wave.
__device__ __forceinline__ void sqnorm_row(const float *x, int64_t d, float *nrm, int lane) {
    float s = 0.f;
    for (int64_t l = lane; l < d; l += kWave) s = fmaf(x[l], x[l], s);
    s = wave_sum(s);
    if (lane == 0) *nrm = s;
}

// ---------------------------------------------------------------- BF16 / FP8 product

// A slab is 128 bytes of every row (64 bf16 or 128 fp8), staged in LDS with a
// 16-byte pad.  The quantised matrix has its rows zero-padded to a whole
// number of slabs, so the loads need no column checks.
constexpr int SLAB = 128;
constexpr int SLD = SLAB + 16;

struct LowpTile {
    const unsigned char *Xq;  // [n][ldq_bytes]
    int64_t ldq_bytes;
    int64_t nslab;
    Epi e;
};

// DB: two sets of slabs (one barrier per slab; the epilogue stages the whole
// tile); else one set (the next slab waits in registers, two barriers per
// slab, the epilogue stages half a tile at a time): about half the LDS, so
// three workgroups fit on a CU.
template <bool DB>
struct LowpLds {
    unsigned char op[DB ? 2 : 1][2][GM * SLD];
    float rn[2 * GM], rs[2 * GM];
};

// Row length of the rounded matrix: d rounded up to whole slabs.
inline int64_t padded_d(int64_t d, int32_t gram_prec) {
    const int64_t per = (gram_prec == KKM_BF16) ? 64 : 128;
    return (d + per - 1) / per * per;
}

// Whether a tile's 128 rounded rows fit one 32-bit buffer range (the product
// reads its operand rows through such ranges).
inline bool lowp_rows_fit(int64_t d, int32_t gram_prec) {
    const int64_t eb = (gram_prec == KKM_BF16) ? 2 : 1;
    return (int64_t)GM * padded_d(d, gram_prec) * eb <= (int64_t)0x7fffffff;
}

// One 128 x 128 tile (bi, bj) of the product and its epilogue, by the 256
// threads of a workgroup, staging through `lds`.
template <int PREC, typename OUT, bool FULL = false, bool DB = true>
__device__ __forceinline__ void lowp_tile(const LowpTile &a, int64_t bi, int64_t bj, LowpLds<DB> &lds) {
    const int64_t m0 = bi * GM, n0 = bj * GM;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int ld_row = tid >> 3;          // 8 threads x 16 bytes per row slab
    const int ld_col = (tid & 7) * 16;

    // The tile's two row blocks as buffer ranges over their rows that exist
    // (a load past the range reads zeros, so rows at or past n need no
    // test): one 32-bit lane offset per row group, shared by both operands,
    // and the slab offset in a scalar register.
    const int64_t ra_rows = min((int64_t)GM, a.e.n - m0), rb_rows = min((int64_t)GM, a.e.n - n0);
    const __amdgpu_buffer_rsrc_t rsa = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<unsigned char *>(a.Xq + m0 * a.ldq_bytes), (short)0, (int)(ra_rows * a.ldq_bytes),
        0x00020000);
    const __amdgpu_buffer_rsrc_t rsb = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<unsigned char *>(a.Xq + n0 * a.ldq_bytes), (short)0, (int)(rb_rows * a.ldq_bytes),
        0x00020000);
    uint32_t voff[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) voff[u] = (uint32_t)((ld_row + 32 * u) * a.ldq_bytes + ld_col);
    uint4 ra[4], rb[4];
    auto gload = [&](int64_t slab) {
        const int soff = (int)(slab * SLAB);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const auto x = __builtin_amdgcn_raw_buffer_load_b128(rsa, voff[u], soff, 0);
            const auto y = __builtin_amdgcn_raw_buffer_load_b128(rsb, voff[u], soff, 0);
            ra[u] = make_uint4(x[0], x[1], x[2], x[3]);
            rb[u] = make_uint4(y[0], y[1], y[2], y[3]);
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            *reinterpret_cast<uint4 *>(&lds.op[buf][0][(ld_row + 32 * u) * SLD + ld_col]) = ra[u];
            *reinterpret_cast<uint4 *>(&lds.op[buf][1][(ld_row + 32 * u) * SLD + ld_col]) = rb[u];
        }
    };

    f32x16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    stage_norms(a.e, m0, n0, lds.rn, lds.rs);
    gload(0);
    sstore(0);
    __syncthreads();

    // Lane half h of a 32x32x16 MFMA supplies k = 8h .. 8h+7.  Within a slab the
    // same permutation is used for both operands: MFMA s takes, from half h,
    // the 8 (bf16) or 8 (fp8) elements starting at byte 64h + 16s (bf16) or
    // 64h + 8s (fp8), so each lane reads 64 consecutive bytes of its row.
    const int half = lane >> 5;
    const int l32 = lane & 31;
    for (int64_t kt = 0; kt < a.nslab; ++kt) {
        const int buf = DB ? (int)(kt & 1) : 0;
        if (kt + 1 < a.nslab) gload(kt + 1);
        const unsigned char *As = lds.op[buf][0];
        const unsigned char *Bs = lds.op[buf][1];
        uint4 av[2][4], bv[2][4];
#pragma unroll
        for (int mi = 0; mi < 2; ++mi) {
            const unsigned char *pa = As + (wr * 64 + mi * 32 + l32) * SLD + half * 64;
            const unsigned char *pb = Bs + (wc * 64 + mi * 32 + l32) * SLD + half * 64;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                av[mi][q] = *reinterpret_cast<const uint4 *>(pa + 16 * q);
                bv[mi][q] = *reinterpret_cast<const uint4 *>(pb + 16 * q);
            }
        }
        if constexpr (PREC == KKM_BF16) {
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                    for (int ni = 0; ni < 2; ++ni) {
                        bf16x8 x, y;
                        __builtin_memcpy(&x, &av[mi][s], 16);
                        __builtin_memcpy(&y, &bv[ni][s], 16);
                        acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x, y, acc[mi][ni], 0, 0, 0);
                    }
        } else {
#pragma unroll
            for (int s = 0; s < 8; ++s)
#pragma unroll
                for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                    for (int ni = 0; ni < 2; ++ni) {
                        const uint4 &p = av[mi][s >> 1];
                        const uint4 &q = bv[ni][s >> 1];
                        const long x = (s & 1) ? (long)(((uint64_t)p.w << 32) | p.z)
                                               : (long)(((uint64_t)p.y << 32) | p.x);
                        const long y = (s & 1) ? (long)(((uint64_t)q.w << 32) | q.z)
                                               : (long)(((uint64_t)q.y << 32) | q.x);
                        acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(x, y, acc[mi][ni], 0, 0, 0);
                    }
        }
        if constexpr (DB) {
            if (kt + 1 < a.nslab) sstore(buf ^ 1);
            __syncthreads();
        } else {
            __syncthreads();  // every read of the slab is done
            if (kt + 1 < a.nslab) {
                sstore(0);
                __syncthreads();
            }
        }
    }
    static_assert(sizeof(lds.op) >= epi_lds_bytes(DB ? 1 : 2), "epilogue tile does not fit");
    static_assert(DB || sizeof(OUT) != 2 || sizeof(lds.op) >= epi_lds_bytes_bf16,
                  "bfloat16 epilogue tile does not fit");
    epilogue<OUT, FULL, DB ? 1 : 2>(a.e, acc, m0, n0, bi == bj, wr, wc, lane,
                                    reinterpret_cast<float *>(&lds.op[0][0][0]), lds.rn, lds.rs);
}

// ---------------------------------------------------------------- BF16 / FP8 product, 256 x 256 tiles
//
// For large problems: a 256 x 256 tile per workgroup of 256 threads (one
// workgroup per CU).  Wave (wr, wc) holds, in each 128 x 128 quadrant (QR, QC)
// of the tile, the same 64 x 64 sub-block it holds in a 128 x 128 tile, so one
// k-step takes 4 A and 4 B fragments for 16 MFMAs (the 128 x 128 tile: 2 + 2
// for 4), halving the operand traffic per MFMA from LDS and from L2.  Every
// output element multiplies the same slabs in the same order as in the 128 x
// 128 tile, so K is the same bit for bit.  The quadrants leave one by one
// through the 128 x 128 epilogue; on a diagonal tile quadrant (1, 0) is the
// mirror of quadrant (0, 1) and is not written.
constexpr int GB = 2 * GM;

struct LowpLds256 {
    unsigned char op[2][2][GB * SLD];  // operand slabs, double-buffered
    float rn[2 * GB], rs[2 * GB];      // [0, 256) rows m0.., [256, 512) rows n0..
    float qn[2 * GM], qs[2 * GM];      // one quadrant's, in the epilogue's layout
};

template <int PREC, typename OUT>
__device__ __forceinline__ void lowp_tile256(const LowpTile &a, int64_t bi, int64_t bj,
                                             LowpLds256 &lds) {
    const int64_t m0 = bi * GB, n0 = bj * GB;
    const bool diag = (bi == bj);

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int ld_row = tid >> 3;  // 8 threads x 16 bytes per row slab
    const int ld_col = (tid & 7) * 16;

    uint4 ra[8], rb[8];
    auto gload = [&](int64_t slab) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t r1 = m0 + ld_row + 32 * u, r2 = n0 + ld_row + 32 * u;
            ra[u] = make_uint4(0, 0, 0, 0);
            rb[u] = make_uint4(0, 0, 0, 0);
            if (r1 < a.e.n)
                ra[u] = *reinterpret_cast<const uint4 *>(a.Xq + r1 * a.ldq_bytes + slab * SLAB + ld_col);
            if (r2 < a.e.n)
                rb[u] = *reinterpret_cast<const uint4 *>(a.Xq + r2 * a.ldq_bytes + slab * SLAB + ld_col);
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            *reinterpret_cast<uint4 *>(&lds.op[buf][0][(ld_row + 32 * u) * SLD + ld_col]) = ra[u];
            *reinterpret_cast<uint4 *>(&lds.op[buf][1][(ld_row + 32 * u) * SLD + ld_col]) = rb[u];
        }
    };

    f32x16 acc[2][2][2][2];  // [QR][QC][mi][ni]
#pragma unroll
    for (int q = 0; q < 16; ++q)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[q >> 3][(q >> 2) & 1][(q >> 1) & 1][q & 1][r] = 0.f;

#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int t = tid + 256 * h;
        const int64_t g = (t < GB) ? m0 + t : n0 + (t - GB);
        const bool in = g < a.e.n;
        lds.rn[t] = (a.e.kernel == KKM_GAUSS && in) ? a.e.nrm[g] : 0.f;
        lds.rs[t] = (a.e.scale && in) ? a.e.scale[g] : 1.f;
    }
    gload(0);
    sstore(0);
    __syncthreads();

    // the k permutation of the 128 x 128 tile: MFMA s takes from lane half h
    // the 16 bytes at 64h + 16s (bf16) or the 8 bytes at 64h + 8s (fp8)
    const int half = lane >> 5;
    const int l32 = lane & 31;
    for (int64_t kt = 0; kt < a.nslab; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < a.nslab) gload(kt + 1);
        const unsigned char *As = lds.op[buf][0] + (wr * 64 + l32) * SLD + half * 64;
        const unsigned char *Bs = lds.op[buf][1] + (wc * 64 + l32) * SLD + half * 64;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            uint4 av[2][2], bv[2][2];  // [Q][mi]
#pragma unroll
            for (int Q = 0; Q < 2; ++Q)
#pragma unroll
                for (int mi = 0; mi < 2; ++mi) {
                    av[Q][mi] = *reinterpret_cast<const uint4 *>(As + (Q * GM + mi * 32) * SLD + 16 * q);
                    bv[Q][mi] = *reinterpret_cast<const uint4 *>(Bs + (Q * GM + mi * 32) * SLD + 16 * q);
                }
            if constexpr (PREC == KKM_BF16) {
#pragma unroll
                for (int QR = 0; QR < 2; ++QR)
#pragma unroll
                    for (int QC = 0; QC < 2; ++QC)
#pragma unroll
                        for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                            for (int ni = 0; ni < 2; ++ni) {
                                bf16x8 x, y;
                                __builtin_memcpy(&x, &av[QR][mi], 16);
                                __builtin_memcpy(&y, &bv[QC][ni], 16);
                                acc[QR][QC][mi][ni] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                                    x, y, acc[QR][QC][mi][ni], 0, 0, 0);
                            }
            } else {
#pragma unroll
                for (int sub = 0; sub < 2; ++sub)
#pragma unroll
                    for (int QR = 0; QR < 2; ++QR)
#pragma unroll
                        for (int QC = 0; QC < 2; ++QC)
#pragma unroll
                            for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                                for (int ni = 0; ni < 2; ++ni) {
                                    const uint4 &p = av[QR][mi];
                                    const uint4 &r = bv[QC][ni];
                                    const long x = sub ? (long)(((uint64_t)p.w << 32) | p.z)
                                                       : (long)(((uint64_t)p.y << 32) | p.x);
                                    const long y = sub ? (long)(((uint64_t)r.w << 32) | r.z)
                                                       : (long)(((uint64_t)r.y << 32) | r.x);
                                    acc[QR][QC][mi][ni] = __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(
                                        x, y, acc[QR][QC][mi][ni], 0, 0, 0);
                                }
            }
        }
        if (kt + 1 < a.nslab) sstore(buf ^ 1);
        __syncthreads();
    }
    static_assert(sizeof(lds.op) >= epi_lds_bytes(1), "epilogue tile does not fit");
    float *T = reinterpret_cast<float *>(&lds.op[0][0][0]);
    // the quadrants one by one, with compile-time indices into acc (a loop
    // too large to unroll would index it at run time and force it into memory)
    auto quadrant = [&](auto qr, auto qc) {
        constexpr int QR = decltype(qr)::value, QC = decltype(qc)::value;
        const int64_t m0q = m0 + QR * GM, n0q = n0 + QC * GM;
        if ((diag && QR > QC) || m0q >= a.e.n || n0q >= a.e.n) return;
        lds.qn[tid] = (tid < GM) ? lds.rn[QR * GM + tid] : lds.rn[GB + QC * GM + (tid - GM)];
        lds.qs[tid] = (tid < GM) ? lds.rs[QR * GM + tid] : lds.rs[GB + QC * GM + (tid - GM)];
        __syncthreads();
        epilogue_keep<OUT>(a.e, acc[QR][QC], m0q, n0q, diag && QR == QC, wr, wc, lane, T, lds.qn,
                           lds.qs);
    };
    quadrant(std::integral_constant<int, 0>{}, std::integral_constant<int, 0>{});
    quadrant(std::integral_constant<int, 0>{}, std::integral_constant<int, 1>{});
    quadrant(std::integral_constant<int, 1>{}, std::integral_constant<int, 0>{});
    quadrant(std::integral_constant<int, 1>{}, std::integral_constant<int, 1>{});
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, kWave));
    return v;
}

// Rounds one row x (d features) to the product's input type into q (dpad
// elements, zero-padded) and returns through lane 0 the squared norm of the
// rounded row (and, for FP8, the row scale).  Called by one whole wave; lane l
// handles elements 4l .. 4l+3 of every 256-element group.
template <int PREC>
__device__ __forceinline__ void quantize_row(const float *x, int64_t d, int64_t dpad,
                                             unsigned char *q, float *nrm, float *scale,
                                             int lane) {
    float inv = 1.f, s = 1.f;
    if (PREC == KKM_FP8_ROWSCALED) {
        float m = 0.f;
        for (int64_t l = lane; l < d; l += kWave) m = fmaxf(m, fabsf(x[l]));
        m = wave_max(m);
        if (m > 0.f && isfinite(m)) {
            s = m / 448.0f;
            inv = 448.0f / m;
        } else if (!isfinite(m)) {
            s = m;  // propagate a non-finite row
        }
        if (lane == 0) *scale = s;
    }
    float acc = 0.f;
    for (int64_t l0 = 4 * lane; l0 < dpad; l0 += 4 * kWave) {
        float v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = (l0 + u < d) ? x[l0 + u] : 0.f;
        if (PREC == KKM_BF16) {
            uint16_t h[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                h[u] = f32_to_bf16(v[u]);
                const float r = bf16_to_f32(h[u]);
                acc = fmaf(r, r, acc);
            }
            uint2 w;
            w.x = (uint32_t)h[0] | ((uint32_t)h[1] << 16);
            w.y = (uint32_t)h[2] | ((uint32_t)h[3] << 16);
            *reinterpret_cast<uint2 *>(q + l0 * 2) = w;
        } else {
            float y[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) y[u] = fminf(fmaxf(v[u] * inv, -448.0f), 448.0f);
            int p = __builtin_amdgcn_cvt_pk_fp8_f32(y[0], y[1], 0, false);
            p = __builtin_amdgcn_cvt_pk_fp8_f32(y[2], y[3], p, true);
            const float q0 = __builtin_amdgcn_cvt_f32_fp8(p, 0);
            const float q1 = __builtin_amdgcn_cvt_f32_fp8(p, 1);
            const float q2 = __builtin_amdgcn_cvt_f32_fp8(p, 2);
            const float q3 = __builtin_amdgcn_cvt_f32_fp8(p, 3);
            acc = fmaf(q0, q0, acc);
            acc = fmaf(q1, q1, acc);
            acc = fmaf(q2, q2, acc);
            acc = fmaf(q3, q3, acc);
            *reinterpret_cast<int *>(q + l0) = p;
        }
    }
    acc = wave_sum(acc);
    if (lane == 0) *nrm = (PREC == KKM_FP8_ROWSCALED) ? s * s * acc : acc;
}

// Launchers of the product kernels, one translation unit each (gram_f32.hip,
// gram_lowp.hip, gram_lowp256.hip); g is the grid of the launch order.
void launch_gram_f32(int32_t k_store, bool full, dim3 g, const F32Tile &a, const TileOrder &order,
                     hipStream_t stream);
void launch_gram_lowp(int32_t gram_prec, int32_t k_store, bool full, dim3 g, const LowpTile &a,
                      const TileOrder &order, hipStream_t stream);
void launch_gram_lowp256(int32_t gram_prec, int32_t k_store, dim3 g, const LowpTile &a,
                         const TileOrder &order, hipStream_t stream);

}  // namespace gt
}  // namespace kkm
