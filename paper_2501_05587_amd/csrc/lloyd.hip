// Cheap iterations of the learned warm start: Lloyd's algorithm (the three
// phases of the paper's Sec. 2.1) with explicit centroids on the feature rows
// F = phi_theta(X) (n x f).  One step costs O(n f k) instead of the O(n^2) of
// an exact step.  Per step:
//   1. V in CSR form from the labels (shared with the exact step);
//   2. centroid sums: chunks of CSR positions, running per-feature sums flushed
//      at cluster boundaries (slot chunk + cluster), then a fixed-order reduce
//      that also forms ||c_c||^2;
//   3. G = F C^T on MFMA (FP32);
//   4. d_ic = ||f_i||^2 - 2 G_ic + ||c_c||^2, argmin (lowest index on ties, an
//      empty cluster at +inf), changed count.
#include "gemm.h"

namespace kkm {

kkm_status vcsr_build(const int32_t *labels, int64_t n, int32_t k, int32_t *blk_hist,
                      int32_t *blk_bad, int32_t *err, int32_t *counts, int32_t *perm,
                      int32_t *offsets, int32_t *counts_out, int64_t *n_changed,
                      hipStream_t stream);

namespace {

constexpr int64_t kRows = 64;  // CSR positions per centroid-sum chunk

struct LloydWs {
    int32_t *blk_hist, *blk_bad, *err, *counts, *perm, *offsets, *counts_out;
    int64_t *changed;
    float *fn, *Cp, *C, *cn, *G;
    int32_t *lab[2];
    double *part, *obj;
};

LloydWs carve_lloyd(void *base, int64_t n, int64_t f, int32_t k, size_t *bytes) {
    const int64_t nblk = (n + 255) / 256;
    const int64_t slots = (n + kRows - 1) / kRows + k;
    Carver c(base);
    LloydWs w;
    w.blk_hist = c.take<int32_t>((size_t)(k * nblk));
    w.blk_bad = c.take<int32_t>((size_t)nblk);
    w.err = c.take<int32_t>(1);
    w.counts = c.take<int32_t>((size_t)k);
    w.perm = c.take<int32_t>((size_t)n);
    w.offsets = c.take<int32_t>((size_t)k + 1);
    w.counts_out = c.take<int32_t>((size_t)k);
    w.changed = c.take<int64_t>(1);
    w.fn = c.take<float>((size_t)n);
    w.Cp = c.take<float>((size_t)(slots * f));
    w.C = c.take<float>((size_t)(k * f));
    w.cn = c.take<float>((size_t)k);
    w.G = c.take<float>((size_t)(n * k));
    w.lab[0] = c.take<int32_t>((size_t)n);
    w.lab[1] = c.take<int32_t>((size_t)n);
    w.part = c.take<double>((size_t)((n + 255) / 256));
    w.obj = c.take<double>(1);
    if (bytes) *bytes = c.bytes();
    return w;
}

__global__ void feature_sqnorms(const float *F, int64_t n, int64_t f, int64_t ldf, float *fn) {
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    float s = 0.f;
    for (int64_t t = lane; t < f; t += kWave) s = fmaf(F[row * ldf + t], F[row * ldf + t], s);
    s = wave_sum(s);
    if (lane == 0) fn[row] = s;
}

// One wave per (chunk of kRows CSR positions, block of 256 features): lane l
// owns features 4l .. 4l+3 of the block; rows are read eight at a time and
// summed per cluster segment, flushed to slot chunk + cluster.
__global__ __launch_bounds__(256) void centroid_partials(const float *F, int64_t n, int64_t f,
                                                         int64_t ldf, int32_t k, int64_t nchunk,
                                                         const int32_t *perm,
                                                         const int32_t *offsets, float *Cp) {
    const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (q >= nchunk) return;
    const int64_t t0 = (int64_t)blockIdx.y * 256 + (threadIdx.x & 63) * 4;
    const bool vec = ((ldf & 3) == 0) && ((reinterpret_cast<uintptr_t>(F) & 15) == 0) && (t0 + 3 < f);
    const int64_t p0 = q * kRows, p1 = min(n, p0 + kRows);
    int32_t lo = 0, hi = k - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (offsets[mid] <= p0) lo = mid;
        else hi = mid - 1;
    }
    int32_t c = lo;
    int64_t p = p0;
    auto row = [&](int64_t j, float (&v)[4]) {
        const float *x = F + j * ldf + t0;
        if (vec) {
            const f32x4 w = *reinterpret_cast<const f32x4 *>(x);
            v[0] = w[0], v[1] = w[1], v[2] = w[2], v[3] = w[3];
        } else {
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = (t0 + u < f) ? x[u] : 0.f;
        }
    };
    while (p < p1) {
        while (offsets[c + 1] <= p) ++c;
        const int64_t e = min(p1, (int64_t)offsets[c + 1]);
        float s[4] = {0.f, 0.f, 0.f, 0.f};
        for (; p + 8 <= e; p += 8) {
            float v[8][4];
#pragma unroll
            for (int r = 0; r < 8; ++r) row(__builtin_amdgcn_readfirstlane(perm[p + r]), v[r]);
#pragma unroll
            for (int r = 0; r < 8; ++r)
#pragma unroll
                for (int u = 0; u < 4; ++u) s[u] += v[r][u];
        }
        for (; p < e; ++p) {
            float v[4];
            row(__builtin_amdgcn_readfirstlane(perm[p]), v);
#pragma unroll
            for (int u = 0; u < 4; ++u) s[u] += v[u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (t0 + u < f) Cp[(q + c) * f + t0 + u] = s[u];
    }
}

// One workgroup per cluster: centroid = sum of its chunk partials / |c|, and
// ||c||^2.  Thread t takes features 4 (t % 64) .. + 3 of each 256-feature
// block and chunks t / 64, t / 64 + 4, ...; the four chunk lanes are then
// added pairwise in a fixed order.
__global__ __launch_bounds__(256) void centroid_finalize(const float *Cp, int64_t f, int32_t k,
                                                         const int32_t *offsets, float *C,
                                                         float *cn) {
    __shared__ f32x4 part[4][64];
    __shared__ float sh[256];
    const int c = blockIdx.x;
    const int tid = threadIdx.x, fq = tid & 63, cl = tid >> 6;
    const int64_t a = offsets[c], b = offsets[c + 1];
    const int64_t q0 = (b > a) ? a / kRows : 0, q1 = (b > a) ? (b - 1) / kRows : -1;
    const bool vec = (f & 3) == 0 && (reinterpret_cast<uintptr_t>(Cp) & 15) == 0;
    float sq = 0.f;
    for (int64_t f0 = 0; f0 < f; f0 += 256) {
        const int64_t t0 = f0 + 4 * fq;
        f32x4 s = {0.f, 0.f, 0.f, 0.f};
        for (int64_t q = q0 + cl; q <= q1; q += 4) {
            const float *src = Cp + (q + c) * f + t0;
            if (vec && t0 + 3 < f) {
                const f32x4 v = *reinterpret_cast<const f32x4 *>(src);
                s += v;
            } else {
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (t0 + u < f) s[u] += src[u];
            }
        }
        part[cl][fq] = s;
        __syncthreads();
        if (cl == 0) {
            const f32x4 tot = (part[0][fq] + part[1][fq]) + (part[2][fq] + part[3][fq]);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (t0 + u >= f) break;
                // sum / |c| (an empty cluster keeps a zero centroid)
                const float v = (b > a) ? tot[u] / (float)(b - a) : 0.f;
                C[(int64_t)c * f + t0 + u] = v;
                sq = fmaf(v, v, sq);
            }
        }
        __syncthreads();
    }
    sh[tid] = sq;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (tid < h) sh[tid] += sh[tid + h];
        __syncthreads();
    }
    if (tid == 0) cn[c] = sh[0];
}

// Gt = C F^T ([k][n]: consecutive threads read consecutive entries).
// Also writes, per block, the sum of the chosen (smallest) distances in FP64
// (part, nullable): summed over blocks it is sum_i min_c d_ic, which equals the
// objective of the new labels once no label changes.
__global__ __launch_bounds__(256) void feature_assign(const float *Gt, const float *fn,
                                                      const float *cn, const int32_t *offsets,
                                                      int64_t n, int32_t k,
                                                      const int32_t *labels_in,
                                                      int32_t *labels_out, int64_t *changed,
                                                      double *part) {
    __shared__ long long wc[4];
    __shared__ double wd[4];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    long long ch = 0;
    double dmin = 0.0;
    if (i < n) {
        float best = __builtin_inff();
        int32_t arg = labels_in[i];
        for (int32_t c = 0; c < k; ++c) {
            if (offsets[c + 1] == offsets[c]) continue;
            const float d = fmaf(-2.0f, Gt[(int64_t)c * n + i], fn[i]) + cn[c];
            if (d < best) {
                best = d;
                arg = c;
            }
        }
        labels_out[i] = arg;
        ch = (arg != labels_in[i]);
        dmin = (double)fmaxf(best, 0.0f);
    }
    ch = wave_sum(ch);
    dmin = wave_sum(dmin);
    if ((threadIdx.x & 63) == 0) {
        wc[threadIdx.x >> 6] = ch;
        wd[threadIdx.x >> 6] = dmin;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const long long t = wc[0] + wc[1] + wc[2] + wc[3];
        if (t) atomicAdd((unsigned long long *)changed, (unsigned long long)t);
        if (part) part[blockIdx.x] = (wd[0] + wd[1]) + (wd[2] + wd[3]);
    }
}

__global__ __launch_bounds__(256) void sum_blocks(const double *part, int64_t np, double *out) {
    __shared__ double sh[256];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < np; i += 256) s += part[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

// ---------------------------------------------------------------- k-means++ seeding
//
// Seeding by D^2 sampling (Arthur and Vassilvitskii, 2007; the K-means++ the
// paper's Sec. 2.1 mentions): the first seed is row floor(u_0 n); seed t+1 is
// the first row i whose running sum of dmin exceeds u_{t+1} * sum(dmin), where
// dmin_i is the squared distance of row i to its nearest seed so far.  The
// uniforms u_t come from the caller.  Sums run in FP64 in a fixed order.

// The running sum is kept in three levels of FP64 sums: blocks of kKppRows
// rows, groups of kKppGroup rows (one update workgroup), and the total.  The
// update kernel writes the first two; a one-workgroup select kernel then
// locates the crossing level by level with block scans: ranges of groups,
// then groups, then blocks, then rows.  Each level takes the first element
// whose inclusive running sum passes the target, or its last element if
// rounding leaves the target at its very end.

constexpr int kKppRows = 4;
constexpr int kKppGroup = 256;
constexpr int kKppPerGroup = kKppGroup / kKppRows;  // block sums per group

struct KppSums {
    double *bsum;  // [ceil(n / kKppRows)]
    double *gsum;  // [ceil(n / kKppGroup)]
};

// Scan of one value per thread over a 256-thread workgroup (fixed order):
// returns the inclusive sum, with the exclusive sum in *excl and the total in
// *total.  The exclusive sum of thread i is bit for bit the inclusive sum of
// thread i-1, and the total that of thread 255, so "the first thread whose
// running sum passes a target" is well defined and consistent with the total.
__device__ double block_scan256(double v, double *sh, double *excl, double *total) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const double o = __shfl_up(v, off, kWave);
        if (lane >= off) v += o;
    }
    const double prev = __shfl_up(v, 1, kWave);
    if (lane == kWave - 1) sh[w] = v;
    __syncthreads();
    double base = 0.0;
    for (int q = 0; q < w; ++q) base += sh[q];
    double t = 0.0;
    for (int q = 0; q < 4; ++q) t += sh[q];
    *total = t;
    *excl = (lane == 0) ? base : base + prev;
    __syncthreads();
    return base + v;
}

// Smallest thread index of the workgroup whose pred is true, or -1.
__device__ int first_true256(bool pred, int *shi) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const unsigned long long m = __ballot(pred);
    if (lane == 0) shi[w] = m ? w * kWave + __ffsll((long long)m) - 1 : -1;
    __syncthreads();
    int r = -1;
    for (int q = 3; q >= 0; --q)
        if (shi[q] >= 0) r = shi[q];
    __syncthreads();
    return r;
}

// Index in [lo, hi) of the first element whose inclusive running sum, added
// to *run, passes target (the last one if none does), with *run advanced to
// the exclusive running sum before it.  hi - lo may exceed 256 (chunks of 256).
__device__ int64_t kpp_locate(const double *vals, int64_t lo, int64_t hi, double target, double *run,
                              double *sh, int *shi) {
    const int tid = threadIdx.x;
    double base = *run;
    for (int64_t c0 = lo; c0 < hi; c0 += 256) {
        const int64_t i = c0 + tid;
        const double v = (i < hi) ? vals[i] : 0.0;
        double excl, tot;
        const double incl = block_scan256(v, sh, &excl, &tot);
        const int f = first_true256(i < hi && base + incl > target, shi);
        if (f >= 0) {
            if (tid == f) sh[4] = base + excl;
            __syncthreads();
            *run = sh[4];
            __syncthreads();
            return c0 + f;
        }
        base += tot;
    }
    // rounding left the target at the very end
    *run = base - vals[hi - 1];
    return hi - 1;
}

// Seed t+1 from the sums: one workgroup of 256 threads.
__global__ __launch_bounds__(256) void kpp_select(KppSums q, const float *dmin, int64_t n, double u,
                                                  int32_t *seed_out) {
    __shared__ double sh[8];
    __shared__ int shi[4];
    const int64_t nb = (n + kKppRows - 1) / kKppRows, ng = (n + kKppGroup - 1) / kKppGroup;
    const int tid = threadIdx.x;
    // ranges of groups, one per thread
    const int64_t per = (ng + 255) / 256;
    const int64_t g0 = min(ng, (int64_t)tid * per), g1 = min(ng, g0 + per);
    double s = 0.0;
    for (int64_t g = g0; g < g1; ++g) s += q.gsum[g];
    double excl, total;
    const double incl = block_scan256(s, sh, &excl, &total);
    if (!(total > 0.0)) {
        if (tid == 0) *seed_out = (int32_t)min((int64_t)(u * (double)n), n - 1);
        return;  // every row coincides with a seed
    }
    const double target = u * total;
    int r = first_true256(g0 < g1 && incl > target, shi);
    if (r < 0) r = (int)((ng - 1) / per);  // the last non-empty range
    if (tid == r) sh[4] = excl;
    __syncthreads();
    double run = sh[4];
    __syncthreads();
    const int64_t rg0 = (int64_t)r * per, rg1 = min(ng, rg0 + per);
    const int64_t g = kpp_locate(q.gsum, rg0, rg1, target, &run, sh, shi);
    const int64_t b = kpp_locate(q.bsum, g * kKppPerGroup, min(nb, (g + 1) * kKppPerGroup), target,
                                 &run, sh, shi);
    if (tid == 0) {
        const int64_t r1 = min(n, (b + 1) * kKppRows);
        int64_t row = r1 - 1;
        for (int64_t i = b * kKppRows; i < r1; ++i) {
            run += (double)dmin[i];
            if (run > target) {
                row = i;
                break;
            }
        }
        *seed_out = (int32_t)row;
    }
}

// Block and group sums of the calling workgroup (thread i holds the updated
// dmin of row blockIdx.x * kKppGroup + i, 0 past n).
__device__ void kpp_sums(double v, int64_t n, const KppSums &q) {
    __shared__ double sh[4];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t row = (int64_t)blockIdx.x * kKppGroup + tid;
    const int g = lane & ~(kKppRows - 1);
    const double v0 = __shfl(v, g, kWave), v1 = __shfl(v, g + 1, kWave);
    const double v2 = __shfl(v, g + 2, kWave), v3 = __shfl(v, g + 3, kWave);
    const double bs = (v0 + v1) + (v2 + v3);
    const bool head = (lane & (kKppRows - 1)) == 0;
    if (head && row < n) q.bsum[row / kKppRows] = bs;
    const double ws = wave_sum(head ? bs : 0.0);
    if (lane == 0) sh[w] = ws;
    __syncthreads();
    if (tid == 0) q.gsum[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// dmin_i = min over seeds 0..t of |F_i - F_seed|^2.  Wave w of a workgroup
// takes rows 64w .. 64w+63 of its group, kKppPass at a time (all their loads
// issued together), each row's squared distance summed over 16-byte slices
// (lane l: columns 4l + 256j ..) and then across the wave.
constexpr int kKppPass = 16;

__global__ __launch_bounds__(256) void kpp_update(const float *F, int64_t n, int64_t f, int64_t ldf,
                                                  int vec, const int32_t *seeds, int t, float *dmin,
                                                  KppSums q) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * kKppGroup + 64 * w;
    const float *c = F + (int64_t)seeds[t] * ldf;
    float mine = 0.f;
    for (int p = 0; p < kWave / kKppPass; ++p) {
        float d[kKppPass];
#pragma unroll
        for (int j = 0; j < kKppPass; ++j) d[j] = 0.f;
        for (int64_t c0 = 0; c0 < f; c0 += 4 * kWave) {
            const int64_t col = c0 + 4 * lane;
            f32x4 cv = {0.f, 0.f, 0.f, 0.f};
            const bool full = vec && col + 3 < f;
            if (full) {
                cv = *reinterpret_cast<const f32x4 *>(c + col);
            } else {
                for (int e = 0; e < 4; ++e)
                    if (col + e < f) cv[e] = c[col + e];
            }
            f32x4 xv[kKppPass];
#pragma unroll
            for (int j = 0; j < kKppPass; ++j) {
                const int64_t row = r0 + kKppPass * p + j;
                xv[j] = f32x4{0.f, 0.f, 0.f, 0.f};
                if (row >= n) continue;
                const float *x = F + row * ldf + col;
                if (full) {
                    xv[j] = *reinterpret_cast<const f32x4 *>(x);
                } else {
                    for (int e = 0; e < 4; ++e)
                        if (col + e < f) xv[j][e] = x[e];
                }
            }
#pragma unroll
            for (int j = 0; j < kKppPass; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const float df = xv[j][e] - cv[e];
                    d[j] = fmaf(df, df, d[j]);
                }
        }
#pragma unroll
        for (int j = 0; j < kKppPass; ++j) {
            const float sj = wave_sum(d[j]);
            if (lane == kKppPass * p + j) mine = sj;
        }
    }
    const int64_t row = r0 + lane;
    double v = 0.0;
    if (row < n) {
        const float m = (t == 0) ? mine : fminf(dmin[row], mine);
        dmin[row] = m;
        v = (double)m;
    }
    kpp_sums(v, n, q);
}

// ---------------------------------------------------------------- seeding on K
//
// The same D^2 sampling in the kernel's feature space, with no features: the
// squared distance of point i to seed s is K_ii + K_ss - 2 K_si (row s of K,
// read along the row), clamped at 0.  O(n) per seed, O(nk) for the labels.

__device__ __forceinline__ float kentry(const float *K, int64_t idx) { return K[idx]; }
__device__ __forceinline__ float kentry(const uint16_t *K, int64_t idx) {
    return __uint_as_float((uint32_t)K[idx] << 16);
}

// dmin_i = min over seeds 0..t of the distance, one thread per row; the sums
// as for the feature rows.
template <typename T>
__global__ __launch_bounds__(256) void kkpp_update(const T *K, int64_t ldk, const float *diag,
                                                   int64_t n, const int32_t *seeds, int t,
                                                   float *dmin, KppSums q) {
    const int64_t i = (int64_t)blockIdx.x * kKppGroup + threadIdx.x;
    const int64_t sd = seeds[t];
    double v = 0.0;
    if (i < n) {
        const float d = fmaxf(diag[i] + diag[sd] - 2.0f * kentry(K, sd * ldk + i), 0.0f);
        const float m = (t == 0) ? d : fminf(dmin[i], d);
        dmin[i] = m;
        v = (double)m;
    }
    kpp_sums(v, n, q);
}

// label_i = index of the nearest seed (lowest on ties)
template <typename T>
__global__ __launch_bounds__(256) void kkpp_assign(const T *K, int64_t ldk, const float *diag,
                                                   int64_t n, int32_t k, const int32_t *seeds,
                                                   int32_t *labels) {
    extern __shared__ int32_t ss[];
    for (int t = threadIdx.x; t < k; t += 256) ss[t] = seeds[t];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float di = diag[i];
    float best = __builtin_inff();
    int32_t arg = 0;
    for (int32_t t = 0; t < k; ++t) {
        const int64_t sd = ss[t];
        const float d = fmaxf(di + diag[sd] - 2.0f * kentry(K, sd * ldk + i), 0.0f);
        if (d < best) {
            best = d;
            arg = t;
        }
    }
    labels[i] = arg;
}

__global__ void gather_seed_rows(const float *F, int64_t ldf, int64_t f, const int32_t *seeds,
                                 float *C) {
    const int64_t c = blockIdx.x;
    const int64_t src = seeds[c];
    for (int64_t t = threadIdx.x; t < f; t += blockDim.x) C[c * f + t] = F[src * ldf + t];
}

__global__ void row_sqnorms_small(const float *C, int64_t k, int64_t f, float *cn) {
    const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (c >= k) return;
    float s = 0.f;
    for (int64_t t = lane; t < f; t += kWave) s = fmaf(C[c * f + t], C[c * f + t], s);
    s = wave_sum(s);
    if (lane == 0) cn[c] = s;
}

__global__ void iota_i32(int32_t *p, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = (int32_t)i;
}

__global__ void fill_one_i32(int32_t *p, int32_t v) { *p = v; }

}  // namespace

}  // namespace kkm

using namespace kkm;

extern "C" size_t kkm_feature_kmeanspp_workspace_bytes(int64_t n, int64_t f, int32_t k) {
    if (n < 1 || f < 1 || k < 1) return 0;
    Carver c(nullptr);
    c.take<float>((size_t)n);                                  // dmin
    c.take<double>((size_t)((n + kKppRows - 1) / kKppRows));   // block sums
    c.take<double>((size_t)((n + kKppGroup - 1) / kKppGroup)); // group sums
    c.take<float>((size_t)(k * f));                            // seed rows
    c.take<float>((size_t)k);                                  // their norms
    c.take<float>((size_t)n);                                  // row norms
    c.take<float>((size_t)(n * k));                            // S F^T
    c.take<int32_t>((size_t)k + 1);                            // offsets 0..k
    c.take<int32_t>((size_t)n);                                // placeholder input labels
    c.take<int64_t>(1);                                        // changed count
    return c.bytes();
}

extern "C" kkm_status kkm_feature_kmeanspp(const float *F, int64_t n, int64_t f, int64_t ldf,
                                           int32_t k, const double *uniforms, int32_t *seeds,
                                           int32_t *labels_out, void *ws, size_t ws_bytes,
                                           void *stream) {
    if (n < 1 || f < 1 || ldf < f || k < 1 || k > n || !F || !uniforms || !seeds || !labels_out) {
        set_error("kkm_feature_kmeanspp: bad sizes or NULL pointer");
        return KKM_ERR_ARG;
    }
    for (int32_t t = 0; t < k; ++t)
        if (!(uniforms[t] >= 0.0 && uniforms[t] < 1.0)) {
            set_error("kkm_feature_kmeanspp: uniforms must lie in [0, 1)");
            return KKM_ERR_ARG;
        }
    const size_t need = kkm_feature_kmeanspp_workspace_bytes(n, f, k);
    if (!ws || ws_bytes < need) {
        set_error("kkm_feature_kmeanspp: workspace of %zu bytes is smaller than %zu", ws_bytes, need);
        return KKM_ERR_NOMEM;
    }
    hipStream_t s = (hipStream_t)stream;
    Carver c(ws);
    float *dmin = c.take<float>((size_t)n);
    const int64_t ng = (n + kKppGroup - 1) / kKppGroup;
    KppSums q;
    q.bsum = c.take<double>((size_t)((n + kKppRows - 1) / kKppRows));
    q.gsum = c.take<double>((size_t)ng);
    float *C = c.take<float>((size_t)(k * f));
    float *cn = c.take<float>((size_t)k);
    float *fn = c.take<float>((size_t)n);
    float *G = c.take<float>((size_t)(n * k));
    int32_t *offs = c.take<int32_t>((size_t)k + 1);
    int32_t *lab_in = c.take<int32_t>((size_t)n);
    int64_t *changed = c.take<int64_t>(1);
    const int64_t first = (int64_t)(uniforms[0] * (double)n);
    hipLaunchKernelGGL(fill_one_i32, dim3(1), dim3(1), 0, s, seeds, (int32_t)(first < n ? first : n - 1));
    const int vec = ((ldf & 3) == 0) && ((reinterpret_cast<uintptr_t>(F) & 15) == 0);
    for (int32_t t = 0; t + 1 < k; ++t) {
        hipLaunchKernelGGL(kpp_update, dim3((unsigned)ng), dim3(256), 0, s, F, n, f, ldf, vec, seeds,
                           t, dmin, q);
        hipLaunchKernelGGL(kpp_select, dim3(1), dim3(256), 0, s, q, dmin, n, uniforms[t + 1],
                           seeds + t + 1);
        KKM_HIP(hipGetLastError());
    }
    // labels: nearest seed (lowest index on ties), via the Lloyd assignment
    hipLaunchKernelGGL(gather_seed_rows, dim3((unsigned)k), dim3(256), 0, s, F, ldf, f, seeds, C);
    hipLaunchKernelGGL(row_sqnorms_small, dim3((unsigned)((k + 3) / 4)), dim3(256), 0, s, C,
                       (int64_t)k, f, cn);
    hipLaunchKernelGGL(feature_sqnorms, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, F, n, f,
                       ldf, fn);
    hipLaunchKernelGGL(iota_i32, dim3((unsigned)((k + 1 + 255) / 256)), dim3(256), 0, s, offs,
                       (int64_t)k + 1);
    hipLaunchKernelGGL(iota_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, lab_in, n);
    KKM_HIP(hipGetLastError());
    GemmArgs g{};
    g.A = C;
    g.lda = f;
    g.B = F;
    g.ldb = ldf;
    g.M = k;
    g.N = n;
    g.K = f;
    g.alpha = 1.0f;
    g.C = G;
    g.ldc = n;
    KKM_TRY(gemm_launch(GEMM_F32, true, true, EPI_STORE, g, s));
    hipLaunchKernelGGL(feature_assign, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, G, fn,
                       cn, offs, n, k, lab_in, labels_out, changed, nullptr);
    KKM_HIP(hipGetLastError());
    return KKM_OK;
}

extern "C" size_t kkm_kernel_kmeanspp_workspace_bytes(int64_t n, int32_t k) {
    if (n < 1 || k < 1) return 0;
    Carver c(nullptr);
    c.take<float>((size_t)n);                                   // dmin
    c.take<double>((size_t)((n + kKppRows - 1) / kKppRows));    // block sums
    c.take<double>((size_t)((n + kKppGroup - 1) / kKppGroup));  // group sums
    return c.bytes();
}

extern "C" kkm_status kkm_kernel_kmeanspp(const void *K, int32_t k_store, int64_t ldk,
                                          const float *diagK, int64_t n, int32_t k,
                                          const double *uniforms, int32_t *seeds,
                                          int32_t *labels_out, void *ws, size_t ws_bytes,
                                          void *stream) {
    if (n < 1 || k < 1 || k > n || ldk < n || !K || !diagK || !uniforms || !seeds ||
        !labels_out) {
        set_error("kkm_kernel_kmeanspp: bad sizes or NULL pointer");
        return KKM_ERR_ARG;
    }
    if (k_store != KKM_F32 && k_store != KKM_BF16) {
        set_error("kkm_kernel_kmeanspp: K must be stored as KKM_F32 or KKM_BF16");
        return KKM_ERR_ARG;
    }
    if (k > KKM_MAX_K) {
        set_error("kkm_kernel_kmeanspp: k=%d exceeds KKM_MAX_K=%d", k, KKM_MAX_K);
        return KKM_ERR_UNSUPPORTED;
    }
    for (int32_t t = 0; t < k; ++t)
        if (!(uniforms[t] >= 0.0 && uniforms[t] < 1.0)) {
            set_error("kkm_kernel_kmeanspp: uniforms must lie in [0, 1)");
            return KKM_ERR_ARG;
        }
    const size_t need = kkm_kernel_kmeanspp_workspace_bytes(n, k);
    if (!ws || ws_bytes < need) {
        set_error("kkm_kernel_kmeanspp: workspace of %zu bytes is smaller than %zu", ws_bytes,
                  need);
        return KKM_ERR_NOMEM;
    }
    hipStream_t s = (hipStream_t)stream;
    Carver c(ws);
    float *dmin = c.take<float>((size_t)n);
    KppSums q;
    q.bsum = c.take<double>((size_t)((n + kKppRows - 1) / kKppRows));
    q.gsum = c.take<double>((size_t)((n + kKppGroup - 1) / kKppGroup));
    const int64_t first = (int64_t)(uniforms[0] * (double)n);
    hipLaunchKernelGGL(fill_one_i32, dim3(1), dim3(1), 0, s, seeds,
                       (int32_t)(first < n ? first : n - 1));
    const dim3 g((unsigned)((n + kKppGroup - 1) / kKppGroup)), b(256);
    for (int32_t t = 0; t + 1 < k; ++t) {
        if (k_store == KKM_F32)
            hipLaunchKernelGGL(kkpp_update<float>, g, b, 0, s, static_cast<const float *>(K), ldk,
                               diagK, n, seeds, t, dmin, q);
        else
            hipLaunchKernelGGL(kkpp_update<uint16_t>, g, b, 0, s,
                               static_cast<const uint16_t *>(K), ldk, diagK, n, seeds, t, dmin, q);
        hipLaunchKernelGGL(kpp_select, dim3(1), dim3(256), 0, s, q, dmin, n, uniforms[t + 1],
                           seeds + t + 1);
        KKM_HIP(hipGetLastError());
    }
    const size_t lds = sizeof(int32_t) * (size_t)k;
    if (k_store == KKM_F32)
        hipLaunchKernelGGL(kkpp_assign<float>, g, b, lds, s, static_cast<const float *>(K), ldk,
                           diagK, n, k, seeds, labels_out);
    else
        hipLaunchKernelGGL(kkpp_assign<uint16_t>, g, b, lds, s, static_cast<const uint16_t *>(K),
                           ldk, diagK, n, k, seeds, labels_out);
    KKM_HIP(hipGetLastError());
    return KKM_OK;
}

extern "C" size_t kkm_feature_lloyd_workspace_bytes(int64_t n, int64_t f, int32_t k) {
    if (n < 1 || f < 1 || k < 1) return 0;
    size_t bytes = 0;
    carve_lloyd(nullptr, n, f, k, &bytes);
    return bytes;
}

extern "C" kkm_status kkm_feature_lloyd(const float *F, int64_t n, int64_t f, int64_t ldf,
                                        int32_t k, const int32_t *labels0, int32_t max_iter,
                                        int32_t *labels_out, int32_t *iters,
                                        int64_t *changed_trace, double *objective, void *ws,
                                        size_t ws_bytes,
                                        void *stream) {
    if (n < 1 || f < 1 || ldf < f || k < 1 || k > n || max_iter < 0 || !F || !labels0 ||
        !labels_out || !iters) {
        set_error("kkm_feature_lloyd: bad sizes or NULL pointer");
        return KKM_ERR_ARG;
    }
    if (k > KKM_MAX_K) {
        set_error("kkm_feature_lloyd: k=%d exceeds KKM_MAX_K=%d", k, KKM_MAX_K);
        return KKM_ERR_UNSUPPORTED;
    }
    size_t need = 0;
    LloydWs w = carve_lloyd(ws, n, f, k, &need);
    if (!ws || ws_bytes < need) {
        set_error("kkm_feature_lloyd: workspace of %zu bytes is smaller than %zu", ws_bytes, need);
        return KKM_ERR_NOMEM;
    }
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(feature_sqnorms, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, F, n, f,
                       ldf, w.fn);
    KKM_HIP(hipGetLastError());
    KKM_HIP(hipMemcpyAsync(w.lab[0], labels0, (size_t)n * 4, hipMemcpyDeviceToDevice, s));
    const int64_t nchunk = (n + kRows - 1) / kRows;
    int cur = 0;
    int32_t t = 0;
    int64_t hc = -1;
    int32_t herr = 0;
    for (; t < max_iter; ++t) {
        KKM_TRY(vcsr_build(w.lab[cur], n, k, w.blk_hist, w.blk_bad, w.err, w.counts, w.perm,
                           w.offsets, w.counts_out, w.changed, s));
        if (t == 0) {
            KKM_HIP(hipMemcpyAsync(&herr, w.err, sizeof herr, hipMemcpyDeviceToHost, s));
            KKM_HIP(hipStreamSynchronize(s));
            if (herr) {
                set_error("kkm_feature_lloyd: a label of labels0 lies outside [0, %d)", k);
                return KKM_ERR_LABEL;
            }
        }
        hipLaunchKernelGGL(centroid_partials, dim3((unsigned)((nchunk + 3) / 4), (unsigned)((f + 255) / 256)),
                           dim3(256), 0, s, F, n, f, ldf, k, nchunk, w.perm, w.offsets, w.Cp);
        hipLaunchKernelGGL(centroid_finalize, dim3((unsigned)k), dim3(256), 0, s, w.Cp, f, k,
                           w.offsets, w.C, w.cn);
        KKM_HIP(hipGetLastError());
        GemmArgs g{};
        g.A = w.C;
        g.lda = f;
        g.B = F;
        g.ldb = ldf;
        g.M = k;
        g.N = n;
        g.K = f;
        g.alpha = 1.0f;
        g.C = w.G;
        g.ldc = n;
        KKM_TRY(gemm_launch(GEMM_F32, true, true, EPI_STORE, g, s));
        hipLaunchKernelGGL(feature_assign, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, w.G,
                           w.fn, w.cn, w.offsets, n, k, w.lab[cur], w.lab[cur ^ 1], w.changed,
                           w.part);
        KKM_HIP(hipGetLastError());
        KKM_HIP(hipMemcpyAsync(&hc, w.changed, sizeof hc, hipMemcpyDeviceToHost, s));
        KKM_HIP(hipStreamSynchronize(s));
        if (changed_trace) changed_trace[t] = hc;
        cur ^= 1;
        if (hc == 0) {
            ++t;
            break;
        }
    }
    KKM_HIP(hipMemcpyAsync(labels_out, w.lab[cur], (size_t)n * 4, hipMemcpyDeviceToDevice, s));
    double obj = 0.0;
    if (objective && t > 0) {
        // sum_i min_c d_ic of the last step (the objective of labels_out when it changed nothing)
        hipLaunchKernelGGL(sum_blocks, dim3(1), dim3(256), 0, s, w.part, (n + 255) / 256, w.obj);
        KKM_HIP(hipGetLastError());
        KKM_HIP(hipMemcpyAsync(&obj, w.obj, sizeof obj, hipMemcpyDeviceToHost, s));
    }
    KKM_HIP(hipStreamSynchronize(s));
    *iters = t;
    if (objective) *objective = (t > 0) ? obj : __builtin_nan("");
    return KKM_OK;
}
