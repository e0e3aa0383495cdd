// Matrix-free reassignment step: E = K V^T without a stored kernel matrix.
//
// The paper builds K once (Sec. 3.2) and then streams it every iteration
// (Sec. 4.3): n^2 elements of memory and n^2 s_K bytes of traffic per step.
// Below the product's ridge point (d of a few hundred for a BF16 product on
// this GPU) recomputing the entries costs less than reading them, and no n^2
// buffer is needed at all.  Each work item takes a strip of 128 points i and a
// chunk of L positions of V's CSR order (points grouped by cluster); it
// multiplies the strip's rows by the rows of the chunk's points, 128 positions
// at a time, on the MFMA (FP32, BF16 or FP8 per-row scaled, as kkm_gram),
// applies the kernel function to the accumulators in registers and adds them,
// per point i, into a running sum for the cluster the positions belong to.
// When a cluster (or the chunk) ends, the sums go to the same partial-sum
// slots the stored-K sweep writes (slot = chunk + cluster, one column per
// point), with the own-cluster sums per strip, so the centroid norms and the
// fused assignment of the stored-K step run unchanged.  Every entry K_ij is
// evaluated once per step (the GEMM count n^2 d, twice the SYRK count of the
// stored-K form's one Gram), and the sums are exact in their order: a step is
// bitwise repeatable.
#include <vector>

#include "gram_tile.h"
#include "iterate.h"

namespace kkm {
namespace {

using namespace gt;

constexpr int MF_N = 128;  // points i per work item (the columns of the partial sums)
constexpr int MF_M = 128;  // CSR positions per product tile

struct MfArgs {
    const float *X;            // FP32 product: the caller's rows
    int64_t ldx;
    int vec_x;
    const unsigned char *Xq;   // BF16 / FP8 product: rounded rows, padded to whole slabs
    int64_t ldq_bytes, nslab;
    int64_t d;
    int kernel;
    float gamma, coef0;        // Gaussian: gamma log2(e)
    int degree;
    const float *nrm;          // squared norms of the rows the product multiplies
    const float *scale;        // FP8 row scales, else null
    int64_t nstrip;            // strips of MF_N points
};

struct MfLds {
    alignas(16) unsigned char op[2][2][GM * SLD];  // operand slabs, double-buffered (FP32: GM * GLD floats)
    float rnA[MF_M], rsA[MF_M];        // norms / scales of the tile's positions
    float fs[MF_N], fc[MF_N];          // flush: sums and compensations of the second wave row
    float fz[2];
};
static_assert(sizeof(float) * 2 * 2 * GM * GLD <= sizeof(MfLds::op), "FP32 slabs do not fit");

__device__ __forceinline__ f32x4 load_f32x4(const MfArgs &a, int64_t row, int64_t col) {
    f32x4 v = {0.f, 0.f, 0.f, 0.f};
    if (row >= 0) {
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

// The 128 x 128 product tile: rows A = the points at 128 positions (arow,
// -1 past the chunk), columns B = the item's points (brow, -1 past n).  The
// four waves hold it as 2 x 2 sub-tiles of 64 x 64 (acc[mi][ni] as the Gram
// tile: register r of lane l is row 8(r/4) + 4(l/32) + r%4, column l%32).
template <int PREC>
__device__ __forceinline__ void mf_product(const MfArgs &a, const int64_t (&arow)[4],
                                           const int64_t (&brow)[4], MfLds &lds,
                                           f32x16 (&acc)[2][2]) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int half = lane >> 5, l32 = lane & 31;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    if constexpr (PREC == KKM_F32) {
        float(*op)[2][GM * GLD] = reinterpret_cast<float(*)[2][GM * GLD]>(&lds.op[0][0][0]);
        const int ld_row = tid >> 3, ld_col = (tid & 7) * 4;
        f32x4 ra[4], rb[4];
        auto gload = [&](int64_t k0) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                ra[u] = load_f32x4(a, arow[u], k0 + ld_col);
                rb[u] = load_f32x4(a, brow[u], k0 + ld_col);
            }
        };
        auto sstore = [&](int buf) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                *reinterpret_cast<f32x4 *>(&op[buf][0][(ld_row + 32 * u) * GLD + ld_col]) = ra[u];
                *reinterpret_cast<f32x4 *>(&op[buf][1][(ld_row + 32 * u) * GLD + ld_col]) = rb[u];
            }
        };
        const int64_t nk = (a.d + GK - 1) / GK;
        gload(0);
        sstore(0);
        __syncthreads();
        for (int64_t kt = 0; kt < nk; ++kt) {
            const int buf = kt & 1;
            if (kt + 1 < nk) gload((kt + 1) * GK);
            const float *As = op[buf][0];
            const float *Bs = op[buf][1];
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
    } else {
        const int ld_row = tid >> 3, ld_col = (tid & 7) * 16;
        uint4 ra[4], rb[4];
        auto gload = [&](int64_t slab) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                ra[u] = make_uint4(0, 0, 0, 0);
                rb[u] = make_uint4(0, 0, 0, 0);
                if (arow[u] >= 0)
                    ra[u] = *reinterpret_cast<const uint4 *>(a.Xq + arow[u] * a.ldq_bytes +
                                                             slab * SLAB + ld_col);
                if (brow[u] >= 0)
                    rb[u] = *reinterpret_cast<const uint4 *>(a.Xq + brow[u] * a.ldq_bytes +
                                                             slab * SLAB + ld_col);
            }
        };
        auto sstore = [&](int buf) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                *reinterpret_cast<uint4 *>(&lds.op[buf][0][(ld_row + 32 * u) * SLD + ld_col]) = ra[u];
                *reinterpret_cast<uint4 *>(&lds.op[buf][1][(ld_row + 32 * u) * SLD + ld_col]) = rb[u];
            }
        };
        gload(0);
        sstore(0);
        __syncthreads();
        for (int64_t kt = 0; kt < a.nslab; ++kt) {
            const int buf = kt & 1;
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
                            acc[mi][ni] =
                                __builtin_amdgcn_mfma_f32_32x32x16_bf16(x, y, acc[mi][ni], 0, 0, 0);
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
                            acc[mi][ni] =
                                __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(x, y, acc[mi][ni], 0, 0, 0);
                        }
            }
            if (kt + 1 < a.nslab) sstore(buf ^ 1);
            __syncthreads();
        }
    }
}

// One work item = (strip of MF_N points, chunk q of L CSR positions).  For
// every cluster c with positions in the chunk it writes
//   P[(q + c) ldp + i] = sum over those positions p of K(x_i, x_perm[p])
// for the strip's points i < n, and Zp[(q + c) nws + strip] = the sum of those
// values over the strip's points whose label is c: the outputs of the
// stored-K sweep for the same chunk length, in another summation order.
template <int PREC>
__global__ __launch_bounds__(256) void matfree_sweep(MfArgs a, Inst in, const int32_t *labels) {
    __shared__ MfLds lds;
    if (*in.err != 0) return;
    const int64_t n = in.n;
    const int32_t k = in.k;
    const int64_t item = blockIdx.x;
    const int64_t strip = item % a.nstrip;
    const int64_t q = item / a.nstrip;
    const int64_t n0 = strip * MF_N;
    const int64_t p_begin = q * in.L;
    const int64_t p_end = min(n, p_begin + in.L);
    const int32_t *__restrict__ perm = in.perm;
    const int32_t *__restrict__ offsets = in.offsets;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int half = lane >> 5, l32 = lane & 31;
    const int ld_row = tid >> 3;

    int64_t brow[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t i = n0 + ld_row + 32 * u;
        brow[u] = (i < n) ? i : -1;
    }
    // this lane's points (per ni), their labels (for the own-cluster sums),
    // squared norms and scales
    int64_t my_i[2];
    int32_t my_lab[2];
    float nB[2], sB[2];
#pragma unroll
    for (int ni = 0; ni < 2; ++ni) {
        my_i[ni] = n0 + wc * 64 + ni * 32 + l32;
        const bool in_n = my_i[ni] < n;
        my_lab[ni] = in_n ? labels[my_i[ni]] : -1;
        nB[ni] = in_n ? a.nrm[my_i[ni]] : 0.f;
        sB[ni] = (a.scale && in_n) ? a.scale[my_i[ni]] : 1.f;
    }

    // cluster holding position p_begin: last c with offsets[c] <= p_begin
    int32_t lo = 0, hi = k - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (offsets[mid] <= p_begin) lo = mid;
        else hi = mid - 1;
    }
    int32_t c = lo;

    float run[2] = {0.f, 0.f}, comp[2] = {0.f, 0.f};
    auto flush = [&](int32_t cl) {
        // lanes l and l + 32 hold the same point: fold the upper half in
        float s2[2], c2[2];
#pragma unroll
        for (int ni = 0; ni < 2; ++ni) {
            const float os = __shfl_xor(run[ni], 32, kWave);
            const float oc = __shfl_xor(comp[ni], 32, kWave);
            float t, e;
            two_sum(run[ni], os, t, e);
            s2[ni] = t;
            c2[ni] = comp[ni] + oc + e;
        }
        if (wr == 1 && half == 0) {
#pragma unroll
            for (int ni = 0; ni < 2; ++ni) {
                lds.fs[wc * 64 + ni * 32 + l32] = s2[ni];
                lds.fc[wc * 64 + ni * 32 + l32] = c2[ni];
            }
        }
        __syncthreads();
        if (wr == 0) {
            float z = 0.f;
            if (half == 0) {
#pragma unroll
                for (int ni = 0; ni < 2; ++ni) {
                    const int li = wc * 64 + ni * 32 + l32;
                    float t, e;
                    two_sum(s2[ni], lds.fs[li], t, e);
                    const float tot = t + (c2[ni] + lds.fc[li] + e);
                    if (my_i[ni] < n) in.P[(q + cl) * in.ldp + my_i[ni]] = tot;
                    if (my_lab[ni] == cl) z += tot;
                }
            }
            z = wave_sum(z);
            if (lane == 0) lds.fz[wc] = z;
        }
        __syncthreads();
        if (tid == 0) in.Zp[(q + cl) * in.nws + strip] = lds.fz[0] + lds.fz[1];
#pragma unroll
        for (int ni = 0; ni < 2; ++ni) run[ni] = comp[ni] = 0.f;
    };

    for (int64_t p0 = p_begin; p0 < p_end; p0 += MF_M) {
        int64_t arow[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t p = p0 + ld_row + 32 * u;
            arow[u] = (p < p_end) ? (int64_t)perm[p] : -1;
        }
        if (tid < MF_M) {
            const int64_t p = p0 + tid;
            const int64_t j = (p < p_end) ? (int64_t)perm[p] : -1;
            lds.rnA[tid] = (j >= 0) ? a.nrm[j] : 0.f;
            lds.rsA[tid] = (a.scale && j >= 0) ? a.scale[j] : 1.f;
        }
        f32x16 acc[2][2];
        mf_product<PREC>(a, arow, brow, lds, acc);  // ends with a barrier
        // kernel values of the positions [lo_m, hi_m) of the tile (all of them
        // when `all`), summed per point in a fixed order: register r of lane l
        // holds position wr 64 + mi 32 + 8 (r/4) + 4 (l/32) + r%4 of the tile
        auto tile_sums = [&](int lo_m, int hi_m, bool all, float (&part)[2]) {
            part[0] = part[1] = 0.f;
#pragma unroll
            for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                for (int rg = 0; rg < 4; ++rg) {
                    const int m0 = wr * 64 + mi * 32 + 8 * rg + 4 * half;
                    const f32x4 na = *reinterpret_cast<const f32x4 *>(&lds.rnA[m0]);
                    f32x4 sa = {1.f, 1.f, 1.f, 1.f};
                    if (a.scale) sa = *reinterpret_cast<const f32x4 *>(&lds.rsA[m0]);
#pragma unroll
                    for (int r4 = 0; r4 < 4; ++r4) {
                        if (!all && (m0 + r4 < lo_m || m0 + r4 >= hi_m)) continue;
#pragma unroll
                        for (int ni = 0; ni < 2; ++ni) {
                            float b = acc[mi][ni][4 * rg + r4];
                            if (a.scale) b *= sa[r4] * sB[ni];
                            part[ni] += kappa_from_dot(b, na[r4], nB[ni], a.kernel, a.gamma,
                                                       a.coef0, a.degree);
                        }
                    }
                }
        };
        // the tile's positions, cluster by cluster (workgroup-uniform)
        const int64_t pt = min(p0 + (int64_t)MF_M, p_end);
        int64_t p = p0;
        while (p < pt) {
            while (offsets[c + 1] <= p) ++c;  // skip empty clusters
            const int64_t seg_hi = min(pt, (int64_t)offsets[c + 1]);
            float part[2];
            if (p == p0 && seg_hi == p0 + MF_M)
                tile_sums(0, MF_M, true, part);  // the whole tile lies in one cluster
            else
                tile_sums((int)(p - p0), (int)(seg_hi - p0), false, part);
#pragma unroll
            for (int ni = 0; ni < 2; ++ni) {
                float t, e;
                two_sum(run[ni], part[ni], t, e);
                run[ni] = t;
                comp[ni] += e;
            }
            if (seg_hi == (int64_t)offsets[c + 1] || seg_hi == p_end) flush(c);
            p = seg_hi;
        }
        __syncthreads();  // every read of rnA / rsA is done before the next tile stages them
    }
}

// Squared norm of each FP32 row (one wave per row).
__global__ __launch_bounds__(256) void mf_sqnorms(const float *X, int64_t n, int64_t d, int64_t ldx,
                                                  float *nrm) {
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= n) return;
    sqnorm_row(X + row * ldx, d, nrm + row, threadIdx.x & 63);
}

// Rows rounded to the product's input type, with their squared norms (and FP8 scales).
template <int PREC>
__global__ __launch_bounds__(256) void mf_quantize(const float *X, int64_t n, int64_t d,
                                                   int64_t ldx, int64_t dpad, unsigned char *Xq,
                                                   float *nrm, float *scale) {
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= n) return;
    const int64_t eb = (PREC == KKM_BF16) ? 2 : 1;
    quantize_row<PREC>(X + row * ldx, d, dpad, Xq + row * dpad * eb, nrm + row, scale + row,
                       threadIdx.x & 63);
}

// diag(K) from the squared norms: kappa(x_i, x_i) (exactly 1 for the Gaussian;
// NaN for a row with a non-finite entry).
__global__ void mf_diag(const float *nrm, int64_t n, int kernel, float gamma, float coef0,
                        int degree, float *diag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float v = nrm[i];
    float dv;
    if (kernel == KKM_GAUSS) {
        dv = isfinite(v) ? 1.0f : __builtin_nanf("");
    } else {
        dv = kappa_from_dot(v, v, v, kernel, gamma, coef0, degree);
    }
    diag[i] = dv;
}

// CSR positions per work item: a multiple of the tile (128), the largest power
// of two up to 4096 that still gives about 8192 items.
int64_t mf_chunk(int64_t n) {
    const int64_t nstrip = (n + MF_N - 1) / MF_N;
    int64_t L = 4096;
    while (L > MF_M && ((n + L - 1) / L) * nstrip < 8192) L >>= 1;
    return L;
}

struct MfLayout {
    InstGeom g;
    int64_t nstrip, dpad;
    size_t inst_bytes, zp_floats, xq_bytes;
};

MfLayout mf_layout(int64_t n, int64_t d, int32_t k, int32_t gram_prec) {
    MfLayout m;
    m.g = inst_geometry(n, k, mf_chunk(n));
    m.nstrip = (n + MF_N - 1) / MF_N;
    m.dpad = (gram_prec == KKM_F32) ? d : padded_d(d, gram_prec);
    m.inst_bytes = inst_workspace_bytes(m.g);
    m.zp_floats = (size_t)m.g.slots * (size_t)m.nstrip;
    m.xq_bytes = (gram_prec == KKM_F32) ? 0
                 : (size_t)n * (size_t)m.dpad * ((gram_prec == KKM_BF16) ? 2 : 1);
    return m;
}

struct MfWs {
    float *nrm, *scale, *diag, *Zp;
    unsigned char *Xq;
    void *inst;
};

size_t mf_carve(void *base, const MfLayout &m, int64_t n, MfWs *w) {
    Carver c(base);
    float *nrm = c.take<float>((size_t)n);
    float *scale = c.take<float>((size_t)n);
    float *diag = c.take<float>((size_t)n);
    float *Zp = c.take<float>(m.zp_floats);
    unsigned char *Xq = c.take<unsigned char>(m.xq_bytes);
    void *inst = c.take<char>(m.inst_bytes);
    if (w) *w = MfWs{nrm, scale, diag, Zp, Xq, inst};
    return c.bytes();
}

// The product's inputs (rounded rows, norms, scales) and diag(K), once per fit.
kkm_status mf_prologue(const float *X, int64_t n, int64_t d, int64_t ldx, int32_t kernel,
                       double gamma, double coef0, int32_t degree, int32_t gram_prec,
                       const MfLayout &m, const MfWs &w, MfArgs *a, hipStream_t s) {
    const unsigned qgrid = (unsigned)((n + 3) / 4);
    MfArgs r{};
    r.X = X;
    r.ldx = ldx;
    r.vec_x = ((ldx % 4) == 0) && ((reinterpret_cast<uintptr_t>(X) & 15) == 0);
    r.d = d;
    r.kernel = kernel;
    r.gamma = epi_gamma(kernel, gamma);
    r.coef0 = (float)coef0;
    r.degree = degree;
    r.nrm = w.nrm;
    r.scale = nullptr;
    r.nstrip = m.nstrip;
    if (gram_prec == KKM_F32) {
        hipLaunchKernelGGL(mf_sqnorms, dim3(qgrid), dim3(256), 0, s, X, n, d, ldx, w.nrm);
    } else {
        const int64_t eb = (gram_prec == KKM_BF16) ? 2 : 1;
        if (gram_prec == KKM_BF16)
            hipLaunchKernelGGL(mf_quantize<KKM_BF16>, dim3(qgrid), dim3(256), 0, s, X, n, d, ldx,
                               m.dpad, w.Xq, w.nrm, w.scale);
        else
            hipLaunchKernelGGL(mf_quantize<KKM_FP8_ROWSCALED>, dim3(qgrid), dim3(256), 0, s, X, n,
                               d, ldx, m.dpad, w.Xq, w.nrm, w.scale);
        r.Xq = w.Xq;
        r.ldq_bytes = m.dpad * eb;
        r.nslab = m.dpad * eb / SLAB;
        if (gram_prec == KKM_FP8_ROWSCALED) r.scale = w.scale;
    }
    KKM_HIP(hipGetLastError());
    // the diagonal: for the FP8 product the norm already carries the scale
    hipLaunchKernelGGL(mf_diag, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, w.nrm, n,
                       kernel, r.gamma, r.coef0, degree, w.diag);
    KKM_HIP(hipGetLastError());
    *a = r;
    return KKM_OK;
}

kkm_status mf_step(const MfArgs &a, int32_t gram_prec, const MfLayout &m, const MfWs &w,
                   int64_t n, int32_t k, int32_t empty_policy, const int32_t *labels_in,
                   int32_t *labels_out, int32_t *counts_out, int64_t *n_changed, double *J_in,
                   float *D_out, float *ctilde_out, hipStream_t s) {
    Inst in{};
    inst_carve(w.inst, m.g, &in, nullptr);
    in.K = nullptr;
    in.ldk = 0;
    in.diag = w.diag;
    in.lab_off = 0;
    in.empty_policy = empty_policy;
    in.counts_out = counts_out;
    in.n_changed = n_changed;
    in.J_in = J_in;
    in.D_out = D_out;
    in.ctilde_out = ctilde_out;
    in.nstrip = m.nstrip;
    in.nws = m.nstrip;
    in.Zp = w.Zp;
    const int64_t items = m.nstrip * m.g.nchunk;
    if (items > 0x7fffffff) {
        set_error("kkm_iterate_matfree: n=%lld needs more than 2^31 work items", (long long)n);
        return KKM_ERR_UNSUPPORTED;
    }
    auto sweep = [&](hipStream_t st) -> kkm_status {
        const dim3 grid((unsigned)items), blk(256);
        const TimedSpan span = timing_begin(TK_SWEEP, st);
        if (gram_prec == KKM_F32)
            hipLaunchKernelGGL(matfree_sweep<KKM_F32>, grid, blk, 0, st, a, in, labels_in);
        else if (gram_prec == KKM_BF16)
            hipLaunchKernelGGL(matfree_sweep<KKM_BF16>, grid, blk, 0, st, a, in, labels_in);
        else
            hipLaunchKernelGGL(matfree_sweep<KKM_FP8_ROWSCALED>, grid, blk, 0, st, a, in, labels_in);
        KKM_HIP(hipGetLastError());
        timing_end(span, st);
        return KKM_OK;
    };
    (void)k;
    return step_launch_custom(in, labels_in, labels_out, sweep, s);
}

kkm_status mf_check(const char *who, const float *X, int64_t n, int64_t d, int64_t ldx, int32_t k,
                    int32_t kernel_type, double gamma, double coef0, int32_t degree,
                    int32_t gram_prec, int32_t empty_policy) {
    if (n < 1 || d < 1 || ldx < d || k < 1 || k > n || !X) {
        set_error("%s: bad sizes or NULL pointer (n=%lld d=%lld ldx=%lld k=%d)", who,
                  (long long)n, (long long)d, (long long)ldx, k);
        return KKM_ERR_ARG;
    }
    if (k > KKM_MAX_K) {
        set_error("%s: k=%d exceeds KKM_MAX_K=%d", who, k, KKM_MAX_K);
        return KKM_ERR_UNSUPPORTED;
    }
    if (empty_policy != KKM_EMPTY_INF && empty_policy != KKM_EMPTY_ZERO_CENTROID) {
        set_error("%s: unknown empty-cluster policy %d", who, empty_policy);
        return KKM_ERR_ARG;
    }
    KKM_TRY(check_kernel(kernel_type, gamma, coef0, degree));
    return check_dtypes(gram_prec, KKM_F32);
}

}  // namespace
}  // namespace kkm

using namespace kkm;

extern "C" size_t kkm_iterate_matfree_workspace_bytes(int64_t n, int64_t d, int32_t k,
                                                      int32_t gram_prec) {
    if (n < 1 || d < 1 || k < 1 || gram_prec < KKM_F32 || gram_prec > KKM_FP8_ROWSCALED) return 0;
    return mf_carve(nullptr, mf_layout(n, d, k, gram_prec), n, nullptr);
}

extern "C" kkm_status kkm_iterate_matfree(const float *X, int64_t n, int64_t d, int64_t ldx,
                                          int32_t kernel_type, double gamma, double coef0,
                                          int32_t degree, int32_t gram_prec, int32_t k,
                                          const int32_t *labels_in, int32_t empty_policy,
                                          int32_t *labels_out, int32_t *counts_out,
                                          int64_t *n_changed, double *J_in, float *D_out,
                                          float *ctilde_out, float *diagK_out, void *ws,
                                          size_t ws_bytes, void *stream) {
    KKM_TRY(mf_check("kkm_iterate_matfree", X, n, d, ldx, k, kernel_type, gamma, coef0, degree,
                     gram_prec, empty_policy));
    if (!labels_in || !labels_out || !counts_out || !n_changed || !J_in) {
        set_error("kkm_iterate_matfree: NULL output or label pointer");
        return KKM_ERR_ARG;
    }
    if (labels_in == labels_out) {
        set_error("kkm_iterate_matfree: labels_out must not alias labels_in");
        return KKM_ERR_ARG;
    }
    const MfLayout m = mf_layout(n, d, k, gram_prec);
    const size_t need = mf_carve(nullptr, m, n, nullptr);
    if (!ws || ws_bytes < need) {
        set_error("kkm_iterate_matfree: workspace of %zu bytes is smaller than %zu", ws_bytes, need);
        return KKM_ERR_NOMEM;
    }
    MfWs w;
    mf_carve(ws, m, n, &w);
    hipStream_t s = (hipStream_t)stream;
    MfArgs a;
    KKM_TRY(mf_prologue(X, n, d, ldx, kernel_type, gamma, coef0, degree, gram_prec, m, w, &a, s));
    KKM_TRY(mf_step(a, gram_prec, m, w, n, k, empty_policy, labels_in, labels_out, counts_out,
                    n_changed, J_in, D_out, ctilde_out, s));
    if (diagK_out)
        KKM_HIP(hipMemcpyAsync(diagK_out, w.diag, (size_t)n * sizeof(float),
                               hipMemcpyDeviceToDevice, s));
    return KKM_OK;
}

extern "C" kkm_status kkm_fit_matfree(const float *X, int64_t n, int64_t d, int64_t ldx, int32_t k,
                                      int32_t kernel_type, double gamma, double coef0,
                                      int32_t degree, int32_t gram_prec, int32_t empty_policy,
                                      const int32_t *labels0, int32_t max_iter,
                                      int32_t check_convergence, int32_t *labels_out,
                                      double *objective, int32_t *iters, double *J_trace,
                                      int64_t *changed_trace, double *times_ms, void *stream) {
    KKM_TRY(mf_check("kkm_fit_matfree", X, n, d, ldx, k, kernel_type, gamma, coef0, degree,
                     gram_prec, empty_policy));
    if (max_iter < 0 || !labels0 || !labels_out || !objective || !iters) {
        set_error("kkm_fit_matfree: bad max_iter or NULL pointer");
        return KKM_ERR_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    const MfLayout m = mf_layout(n, d, k, gram_prec);
    const size_t need = mf_carve(nullptr, m, n, nullptr);
    void *block = nullptr;
    int32_t *hflag = nullptr;
    struct Guard {
        void **b;
        int32_t **h;
        ~Guard() {
            if (*b) (void)hipFree(*b);
            if (*h) (void)hipHostFree(*h);
        }
    } guard{&block, &hflag};
    KKM_HIP(hipMalloc(&block, need + 256));
    KKM_HIP(hipHostMalloc((void **)&hflag, sizeof(int32_t), hipHostMallocDefault));
    MfWs w;
    mf_carve(block, m, n, &w);
    int32_t *flag = reinterpret_cast<int32_t *>(static_cast<char *>(block) + need);
    MfArgs a;
    hipEvent_t ev[2] = {nullptr, nullptr};
    struct EvGuard {
        hipEvent_t *e;
        ~EvGuard() {
            for (int i = 0; i < 2; ++i)
                if (e[i]) (void)hipEventDestroy(e[i]);
        }
    } evg{ev};
    for (auto &e : ev) KKM_HIP(hipEventCreate(&e));
    KKM_HIP(hipEventRecord(ev[0], s));
    KKM_TRY(mf_prologue(X, n, d, ldx, kernel_type, gamma, coef0, degree, gram_prec, m, w, &a, s));
    flag_nonfinite(w.diag, n, flag, s);
    KKM_HIP(hipGetLastError());
    KKM_HIP(hipEventRecord(ev[1], s));
    KKM_HIP(hipMemcpyAsync(hflag, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    KKM_HIP(hipStreamSynchronize(s));
    if (*hflag != 0) {
        set_error("kkm_fit_matfree: diag(K) has a non-finite entry (NaN or infinity in X?)");
        return KKM_ERR_NONFINITE;
    }
    const StepFn step = [&](const int32_t *in, int32_t *out, int32_t *counts, int64_t *changed,
                            double *J, void *, size_t, hipStream_t st) {
        return mf_step(a, gram_prec, m, w, n, k, empty_policy, in, out, counts, changed, J, nullptr,
                       nullptr, st);
    };
    double loop_ms[2] = {0.0, 0.0};
    KKM_TRY(run_steps(step, 0, n, k, labels0, max_iter, check_convergence, labels_out, objective,
                      iters, J_trace, changed_trace, loop_ms, "kkm_fit_matfree", s));
    if (times_ms) {
        float t0 = 0.f;
        (void)hipEventElapsedTime(&t0, ev[0], ev[1]);
        times_ms[0] = t0;
        times_ms[1] = loop_ms[0];
        times_ms[2] = loop_ms[1];
    }
    return KKM_OK;
}
