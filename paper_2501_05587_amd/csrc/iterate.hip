// One reassignment step of the paper's Algorithm 2 on gfx950.
//
//   1. V from the labels (Sec. 4.1): cluster sizes by a reduction of the label
//      array, then V in CSR form.  V's values are all 1/|c| within a row, so
//      the CSR arrays reduce to the row pointers (cluster offsets) and the
//      column indices (point indices grouped by cluster, stable).
//   2. E = K V^T (Eq. dist_sp_1).  K is symmetric, so row c of E^T is the sum
//      of the K rows of cluster c's members, scaled by 1/|c|.  Walking V's CSR
//      rows visits K's rows cluster by cluster: every row read has one label
//      for the whole wavefront, and each lane keeps a running compensated sum
//      per column in registers that is flushed once per cluster segment.  K is
//      read exactly once, in 1 KiB contiguous pieces per wavefront.
//   3. ||c_c||^2 = (V z)_c with z_i = E_{i,a(i)} (Eq. c_norm, Eq. cnorms_gemv):
//      the sweep folds z into per-segment partials as it flushes, a small
//      kernel reduces them per cluster.
//   4. D_ic = K_ii - 2 E_ic + ||c_c||^2 (Eq. dist_sp_1), argmin over c, the new
//      cluster-size histogram, the number of changed labels and the FP64
//      objective of the input labels, fused in one pass over the points.
//
// No floating-point atomics are used: every reduction runs in a fixed order,
// so a step is bitwise repeatable.
#include "kkm_common.h"

namespace kkm {

namespace {

constexpr int kPtsPerBlock = 256;          // points per block in the label kernels
constexpr int kSweepThreads = 256;         // 4 waves
constexpr int kSweepCols = kSweepThreads * 4;  // columns per sweep workgroup (float4 per lane)
constexpr int kWaveCols = kWave * 4;       // columns per wave strip

struct IterWs {
    int32_t *perm;      // [n]      V's column indices: points grouped by cluster
    int32_t *offsets;   // [k+1]    V's row pointers
    int32_t *counts;    // [k]      cluster sizes of labels_in
    int32_t *blk_hist;  // [k][nblk] per-block histograms, then exclusive prefixes
    int32_t *blk_bad;   // [nblk]   per-block count of out-of-range labels
    int32_t *err;       // [1]
    float *P;           // [slots][ldp] per-segment column sums of K
    float *Zp;          // [slots][nws] per-segment sums of the own-cluster entries
    float *ctilde;      // [k]
    double *Jpart;      // [nblk]
    uint32_t *ticket;   // [1]
};

struct Geometry {
    int64_t n;
    int32_t k;
    int64_t nblk;   // label blocks
    int64_t L;      // rows of K per sweep chunk
    int64_t nchunk;
    int64_t slots;  // nchunk + k
    int64_t ldp;
    int64_t nws;    // wave strips of columns (FP32 K: the most; sizes the partial buffer)
    int64_t nstrip; // workgroup strips of columns
};

Geometry make_geometry(int64_t n, int32_t k) {
    Geometry g;
    g.n = n;
    g.k = k;
    g.nblk = (n + kPtsPerBlock - 1) / kPtsPerBlock;
    g.nstrip = (n + kSweepCols - 1) / kSweepCols;
    g.nws = (n + kWaveCols - 1) / kWaveCols;
    // chunk rows: the largest power of two in [64, 4096] that still gives
    // about 8192 sweep workgroups (the partial sums cost slots * n floats)
    int64_t L = 4096;
    while (L > 64 && ((n + L - 1) / L) * g.nstrip < 8192) L >>= 1;
    g.L = L;
    g.nchunk = (n + L - 1) / L;
    g.slots = g.nchunk + k;
    g.ldp = (n + 63) & ~int64_t(63);
    return g;
}

IterWs carve(void *base, const Geometry &g, size_t *bytes) {
    Carver c(base);
    IterWs w;
    w.perm = c.take<int32_t>((size_t)g.n);
    w.offsets = c.take<int32_t>((size_t)g.k + 1);
    w.counts = c.take<int32_t>((size_t)g.k);
    w.blk_hist = c.take<int32_t>((size_t)g.k * (size_t)g.nblk);
    w.blk_bad = c.take<int32_t>((size_t)g.nblk);
    w.err = c.take<int32_t>(1);
    w.P = c.take<float>((size_t)g.slots * (size_t)g.ldp);
    w.Zp = c.take<float>((size_t)g.slots * (size_t)g.nws);
    w.ctilde = c.take<float>((size_t)g.k);
    w.Jpart = c.take<double>((size_t)g.nblk);
    w.ticket = c.take<uint32_t>(1);
    if (bytes) *bytes = c.bytes();
    return w;
}

// ---------------------------------------------------------------- 1. V in CSR form

// Per-block label histogram (column-major [k][nblk]) and range check.
__global__ __launch_bounds__(kPtsPerBlock) void v_block_hist(const int32_t *labels, int64_t n,
                                                             int32_t k, int64_t nblk,
                                                             int32_t *blk_hist,
                                                             int32_t *blk_bad) {
    extern __shared__ int32_t sh[];  // [k] + 1
    int32_t *hist = sh;
    int32_t *bad = sh + k;
    for (int c = threadIdx.x; c < k; c += blockDim.x) hist[c] = 0;
    if (threadIdx.x == 0) *bad = 0;
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * kPtsPerBlock + threadIdx.x;
    if (i < n) {
        const int32_t c = labels[i];
        if (c < 0 || c >= k)
            atomicAdd(bad, 1);
        else
            atomicAdd(&hist[c], 1);
    }
    __syncthreads();
    for (int c = threadIdx.x; c < k; c += blockDim.x)
        blk_hist[(int64_t)c * nblk + blockIdx.x] = hist[c];
    if (threadIdx.x == 0) blk_bad[blockIdx.x] = *bad;
}

// One workgroup per cluster: exclusive prefix of its per-block counts (in
// place) and its size.  Workgroup 0 also folds the range-check counts.
__global__ __launch_bounds__(256) void v_cluster_scan(int32_t *blk_hist, int64_t nblk,
                                                      int32_t *counts, const int32_t *blk_bad,
                                                      int32_t *err) {
    __shared__ int32_t part[256];
    __shared__ int32_t carry;
    const int c = blockIdx.x;
    int32_t *row = blk_hist + (int64_t)c * nblk;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < nblk; base += 256) {
        const int64_t b = base + threadIdx.x;
        const int32_t v = (b < nblk) ? row[b] : 0;
        part[threadIdx.x] = v;
        __syncthreads();
        // Hillis-Steele inclusive scan over 256 entries
        for (int off = 1; off < 256; off <<= 1) {
            const int32_t add = (threadIdx.x >= off) ? part[threadIdx.x - off] : 0;
            __syncthreads();
            part[threadIdx.x] += add;
            __syncthreads();
        }
        if (b < nblk) row[b] = carry + part[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 255) carry += part[255];
        __syncthreads();
    }
    if (threadIdx.x == 0) counts[c] = carry;
    if (c == 0) {
        int32_t s = 0;
        for (int64_t b = threadIdx.x; b < nblk; b += 256) s += blk_bad[b];
        part[threadIdx.x] = s;
        __syncthreads();
        if (threadIdx.x == 0) {
            int32_t t = 0;
            for (int u = 0; u < 256; ++u) t += part[u];
            *err = t;
        }
    }
}

// Stable scatter of point indices into V's CSR order.  Block 0 also publishes
// the row pointers and clears the step's counters.
__global__ __launch_bounds__(kPtsPerBlock) void v_scatter(
    const int32_t *labels, int64_t n, int32_t k, int64_t nblk, const int32_t *blk_hist,
    const int32_t *counts, const int32_t *err, int32_t *perm, int32_t *offsets,
    int32_t *counts_out, int64_t *n_changed, uint32_t *ticket) {
    extern __shared__ int32_t sh[];  // off[k+1], wcnt[4][k]
    int32_t *off = sh;
    int32_t *wcnt = sh + (k + 1);
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    if (*err != 0) return;

    // exclusive scan of the cluster sizes (k <= KKM_MAX_K; one thread, then share)
    if (tid == 0) {
        int32_t run = 0;
        for (int c = 0; c < k; ++c) {
            off[c] = run;
            run += counts[c];
        }
        off[k] = run;
    }
    for (int c = tid; c < 4 * k; c += kPtsPerBlock) wcnt[c] = 0;
    __syncthreads();
    if (blockIdx.x == 0) {
        for (int c = tid; c <= k; c += kPtsPerBlock) offsets[c] = off[c];
        for (int c = tid; c < k; c += kPtsPerBlock) counts_out[c] = 0;
        if (tid == 0) {
            *n_changed = 0;
            *ticket = 0u;
        }
    }

    const int64_t i = (int64_t)blockIdx.x * kPtsPerBlock + tid;
    const bool valid = i < n;
    const int32_t c = valid ? labels[i] : -1;
    // rank among equal labels earlier in this wave, by matching label groups
    uint64_t pending = __ballot(valid);
    int32_t rank = 0;
    while (pending) {
        const int leader = __ffsll((unsigned long long)pending) - 1;
        const int32_t lc = __shfl(c, leader, kWave);
        const uint64_t m = __ballot(valid && c == lc);
        if (valid && c == lc) {
            const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
            rank = __popcll(m & below);
            if (lane == leader) wcnt[wave * k + c] = __popcll(m);
        }
        pending &= ~m;
    }
    __syncthreads();
    if (valid) {
        int32_t before = 0;
        for (int w = 0; w < wave; ++w) before += wcnt[w * k + c];
        const int64_t pos = off[c] + blk_hist[(int64_t)c * nblk + blockIdx.x] + before + rank;
        perm[pos] = (int32_t)i;
    }
}

// ---------------------------------------------------------------- 2. row sweep of K

// Entries of K as FP32 (4 per 16-byte load) or bfloat16 (8 per 16-byte load),
// widened to float for the sums.
template <typename T> struct KRow;
template <> struct KRow<float> {
    static constexpr int E = 4;
    template <bool VEC>
    static __device__ __forceinline__ void load(const float *row, int64_t col, int64_t n,
                                                float (&v)[E]) {
        if (VEC && col + E - 1 < n) {
            const f32x4 w = *reinterpret_cast<const f32x4 *>(row + col);
#pragma unroll
            for (int u = 0; u < E; ++u) v[u] = w[u];
        } else {
#pragma unroll
            for (int u = 0; u < E; ++u) v[u] = (col + u < n) ? row[col + u] : 0.f;
        }
    }
};
template <> struct KRow<uint16_t> {
    static constexpr int E = 8;
    template <bool VEC>
    static __device__ __forceinline__ void load(const uint16_t *row, int64_t col, int64_t n,
                                                float (&v)[E]) {
        if (VEC && col + E - 1 < n) {
            const uint4 w = *reinterpret_cast<const uint4 *>(row + col);
            const uint32_t p[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                v[2 * u] = __uint_as_float(p[u] << 16);
                v[2 * u + 1] = __uint_as_float(p[u] & 0xffff0000u);
            }
        } else {
#pragma unroll
            for (int u = 0; u < E; ++u)
                v[u] = (col + u < n) ? __uint_as_float((uint32_t)row[col + u] << 16) : 0.f;
        }
    }
};

// Grid (column strips, chunks of L positions in V's CSR order).  Each lane owns
// E consecutive columns (one 16-byte load per row); a wave covers 64 E columns
// and the workgroup 256 E columns of every row it visits.  A chunk may span
// several clusters: the running sums are flushed to the partial-buffer slot
// (chunk + cluster) whenever the cluster changes; the slot is unique per
// (chunk, cluster) pair.
template <typename T, bool VEC>
__global__ __launch_bounds__(kSweepThreads) void spmm_row_sweep(
    const T *__restrict__ K, int64_t ldk, int64_t n, int32_t k,
    const int32_t *__restrict__ perm, const int32_t *__restrict__ offsets,
    const int32_t *__restrict__ labels, int64_t L, float *__restrict__ P, int64_t ldp,
    float *__restrict__ Zp, int64_t nws, const int32_t *err) {
    constexpr int E = KRow<T>::E;
    if (*err != 0) return;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int64_t wave_strip = (int64_t)blockIdx.x * (kSweepThreads / kWave) + (tid >> 6);
    const int64_t col = wave_strip * (kWave * E) + (int64_t)lane * E;
    const int64_t q = blockIdx.y;
    const int64_t p_begin = q * L;
    const int64_t p_end = min(n, p_begin + L);

    // labels of this lane's columns (for z: the own-cluster entries)
    int32_t own[E];
#pragma unroll
    for (int u = 0; u < E; ++u) own[u] = (col + u < n) ? labels[col + u] : -1;

    // cluster holding position p_begin: last c with offsets[c] <= p_begin
    int32_t lo = 0, hi = k - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (offsets[mid] <= p_begin) lo = mid;
        else hi = mid - 1;
    }
    int32_t c = lo;

    int64_t p = p_begin;
    while (p < p_end) {
        while (offsets[c + 1] <= p) ++c;  // skip empty clusters
        const int64_t seg_end = min(p_end, (int64_t)offsets[c + 1]);
        float s[E], e[E];
#pragma unroll
        for (int u = 0; u < E; ++u) s[u] = e[u] = 0.f;
        for (; p + 8 <= seg_end; p += 8) {
            float v[8][E];
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const int64_t j = __builtin_amdgcn_readfirstlane(perm[p + r]);
                KRow<T>::template load<VEC>(K + j * ldk, col, n, v[r]);
            }
#pragma unroll
            for (int u = 0; u < E; ++u) {
                const float blk = ((v[0][u] + v[1][u]) + (v[2][u] + v[3][u])) +
                                  ((v[4][u] + v[5][u]) + (v[6][u] + v[7][u]));
                float t, er;
                two_sum(s[u], blk, t, er);
                s[u] = t;
                e[u] += er;
            }
        }
        if (p < seg_end) {
            float blk[E];
#pragma unroll
            for (int u = 0; u < E; ++u) blk[u] = 0.f;
            for (; p < seg_end; ++p) {
                const int64_t j = __builtin_amdgcn_readfirstlane(perm[p]);
                float v[E];
                KRow<T>::template load<VEC>(K + j * ldk, col, n, v);
#pragma unroll
                for (int u = 0; u < E; ++u) blk[u] += v[u];
            }
#pragma unroll
            for (int u = 0; u < E; ++u) {
                float t, er;
                two_sum(s[u], blk[u], t, er);
                s[u] = t;
                e[u] += er;
            }
        }
        float tot[E];
#pragma unroll
        for (int u = 0; u < E; ++u) tot[u] = s[u] + e[u];
        const int64_t slot = q + c;
        if (col < n) {
            float *dst = P + slot * ldp + col;
            if (col + E - 1 < n) {
#pragma unroll
                for (int u = 0; u < E; u += 4) {
                    const f32x4 w = {tot[u], tot[u + 1], tot[u + 2], tot[u + 3]};
                    *reinterpret_cast<f32x4 *>(dst + u) = w;
                }
            } else {
#pragma unroll
                for (int u = 0; u < E; ++u)
                    if (col + u < n) dst[u] = tot[u];
            }
        }
        float z = 0.f;
#pragma unroll
        for (int u = 0; u < E; ++u)
            if (own[u] == c) z += tot[u];
        z = wave_sum(z);
        if (lane == 0 && wave_strip < nws) Zp[slot * nws + wave_strip] = z;
    }
}

// ---------------------------------------------------------------- 3. centroid norms

// One workgroup per cluster: ||c_c||^2 = (1/|c|^2) sum_{i in c} S_ic, summing
// the z partials of the cluster's segments in a fixed order.
__global__ __launch_bounds__(256) void centroid_norms(const float *Zp, int64_t nws,
                                                     const int32_t *offsets, int64_t L,
                                                     int32_t k, float *ctilde,
                                                     float *ctilde_out, const int32_t *err) {
    __shared__ float ss[256], sc[256];
    if (*err != 0) return;
    const int c = blockIdx.x;
    const int64_t a = offsets[c], b = offsets[c + 1];
    const int64_t cnt = b - a;
    float s = 0.f, comp = 0.f;
    if (cnt > 0) {
        const int64_t q0 = a / L, q1 = (b - 1) / L;
        const int64_t per = nws;
        const int64_t total = (q1 - q0 + 1) * per;
        for (int64_t t = threadIdx.x; t < total; t += 256) {
            const int64_t q = q0 + t / per;
            const int64_t w = t % per;
            float u, er;
            two_sum(s, Zp[(q + c) * nws + w], u, er);
            s = u;
            comp += er;
        }
    }
    ss[threadIdx.x] = s;
    sc[threadIdx.x] = comp;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            float u, er;
            two_sum(ss[threadIdx.x], ss[threadIdx.x + h], u, er);
            ss[threadIdx.x] = u;
            sc[threadIdx.x] += sc[threadIdx.x + h] + er;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        float v = 0.f;
        if (cnt > 0) {
            const float fc = (float)cnt;
            v = ((ss[0] + sc[0]) / fc) / fc;
        }
        ctilde[c] = v;
        if (ctilde_out) ctilde_out[c] = v;
    }
}

// ---------------------------------------------------------------- 4. distances + argmin + histogram

__global__ __launch_bounds__(kPtsPerBlock) void assign_fused(
    const float *__restrict__ P, int64_t ldp, const int32_t *__restrict__ offsets, int64_t L,
    const float *__restrict__ ctilde, const float *__restrict__ diagK,
    const int32_t *__restrict__ labels_in, int64_t n, int32_t k, int32_t empty_policy,
    int32_t *__restrict__ labels_out, int32_t *counts_out, int64_t *n_changed, double *J_in,
    double *Jpart, uint32_t *ticket, float *D_out, const int32_t *err) {
    extern __shared__ int32_t sh[];  // off[k+1], hist[k], then doubles
    int32_t *off = sh;
    int32_t *hist = sh + (k + 1);
    __shared__ double wJ[kPtsPerBlock / kWave];
    __shared__ long long wC[kPtsPerBlock / kWave];
    __shared__ bool last;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    if (*err != 0) {
        if (blockIdx.x == 0 && tid == 0) {
            *n_changed = -1;
            *J_in = __builtin_nan("");
        }
        return;
    }
    for (int c = tid; c <= k; c += kPtsPerBlock) off[c] = offsets[c];
    for (int c = tid; c < k; c += kPtsPerBlock) hist[c] = 0;
    __syncthreads();

    const int64_t i = (int64_t)blockIdx.x * kPtsPerBlock + tid;
    const bool valid = i < n;
    double own_d = 0.0;
    long long changed = 0;
    if (valid) {
        const float dii = diagK[i];
        const int32_t a_in = labels_in[i];
        float best = __builtin_inff();
        int32_t arg = -1;
        float own = 0.f;
        for (int32_t c = 0; c < k; ++c) {
            const int64_t lo = off[c], hi = off[c + 1];
            float dic;
            if (hi > lo) {
                float s = 0.f, comp = 0.f;
                for (int64_t q = lo / L; q <= (hi - 1) / L; ++q) {
                    float u, er;
                    two_sum(s, P[(q + c) * ldp + i], u, er);
                    s = u;
                    comp += er;
                }
                const float e = (s + comp) / (float)(hi - lo);
                dic = fmaf(-2.0f, e, dii) + ctilde[c];
            } else {
                dic = (empty_policy == KKM_EMPTY_ZERO_CENTROID) ? dii : __builtin_inff();
            }
            if (D_out) D_out[i * k + c] = dic;
            if (c == a_in) own = dic;
            if (dic < best) {
                best = dic;
                arg = c;
            }
        }
        if (arg < 0) arg = a_in;
        labels_out[i] = arg;
        atomicAdd(&hist[arg], 1);
        changed = (arg != a_in);
        own_d = (double)own;
    }
    // block reductions in a fixed order
    const double wj = wave_sum(own_d);
    const long long wc = wave_sum(changed);
    if (lane == 0) {
        wJ[wave] = wj;
        wC[wave] = wc;
    }
    __syncthreads();
    if (tid == 0) {
        double bj = 0.0;
        long long bc = 0;
        for (int w = 0; w < kPtsPerBlock / kWave; ++w) {
            bj += wJ[w];
            bc += wC[w];
        }
        Jpart[blockIdx.x] = bj;
        if (bc) atomicAdd((unsigned long long *)n_changed, (unsigned long long)bc);
    }
    for (int c = tid; c < k; c += kPtsPerBlock)
        if (hist[c]) atomicAdd(&counts_out[c], hist[c]);

    // the last block to finish sums the block partials of J in block order
    __threadfence();
    __syncthreads();
    if (tid == 0) last = (atomicAdd(ticket, 1u) == gridDim.x - 1);
    __syncthreads();
    if (!last) return;
    __threadfence();
    double s = 0.0;
    for (int64_t b = tid; b < (int64_t)gridDim.x; b += kPtsPerBlock) s += Jpart[b];
    const double ws = wave_sum(s);
    if (lane == 0) wJ[wave] = ws;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int w = 0; w < kPtsPerBlock / kWave; ++w) t += wJ[w];
        *J_in = t;
    }
}

}  // namespace

// V in CSR form from labels in [0, k): cluster sizes, row pointers (offsets)
// and column indices (perm, stable).  blk_hist holds k * ceil(n/256) ints and
// blk_bad ceil(n/256) ints; *err ends up non-zero when a label is out of range
// (perm is then incomplete).  counts_out[k], *n_changed and *ticket are
// cleared on the way, for a following assignment kernel.
kkm_status vcsr_build(const int32_t *labels, int64_t n, int32_t k, int32_t *blk_hist,
                      int32_t *blk_bad, int32_t *err, int32_t *counts, int32_t *perm,
                      int32_t *offsets, int32_t *counts_out, int64_t *n_changed,
                      uint32_t *ticket, hipStream_t stream) {
    const int64_t nblk = (n + kPtsPerBlock - 1) / kPtsPerBlock;
    hipLaunchKernelGGL(v_block_hist, dim3((unsigned)nblk), dim3(kPtsPerBlock),
                       (k + 1) * sizeof(int32_t), stream, labels, n, k, nblk, blk_hist, blk_bad);
    KKM_HIP(hipGetLastError());
    hipLaunchKernelGGL(v_cluster_scan, dim3((unsigned)k), dim3(256), 0, stream, blk_hist, nblk,
                       counts, blk_bad, err);
    KKM_HIP(hipGetLastError());
    hipLaunchKernelGGL(v_scatter, dim3((unsigned)nblk), dim3(kPtsPerBlock),
                       (size_t)(k + 1 + 4 * k) * sizeof(int32_t), stream, labels, n, k, nblk,
                       blk_hist, counts, err, perm, offsets, counts_out, n_changed, ticket);
    KKM_HIP(hipGetLastError());
    return KKM_OK;
}

size_t iterate_workspace_bytes(int64_t n, int32_t k) {
    size_t bytes = 0;
    carve(nullptr, make_geometry(n, k), &bytes);
    return bytes;
}

kkm_status iterate_launch(const void *K, int32_t k_store, int64_t ldk, const float *diagK,
                          int64_t n, int32_t k, const int32_t *labels_in, int32_t empty_policy,
                          int32_t *labels_out, int32_t *counts_out, int64_t *n_changed,
                          double *J_in, float *D_out, float *ctilde_out, void *ws,
                          size_t ws_bytes, hipStream_t stream) {
    const Geometry g = make_geometry(n, k);
    size_t need = 0;
    IterWs w = carve(ws, g, &need);
    if (ws == nullptr || ws_bytes < need) {
        set_error("kkm_iterate: workspace of %zu bytes is smaller than %zu", ws_bytes, need);
        return KKM_ERR_NOMEM;
    }
    const unsigned nblk = (unsigned)g.nblk;
    const TimedSpan whole = timing_begin(TK_ITERATE, stream);
    KKM_TRY(vcsr_build(labels_in, n, k, w.blk_hist, w.blk_bad, w.err, w.counts, w.perm,
                       w.offsets, counts_out, n_changed, w.ticket, stream));
    // one 16-byte load per lane and row: 4 FP32 or 8 BF16 columns
    const int E = (k_store == KKM_BF16) ? 8 : 4;
    const int64_t cols_per_wg = (int64_t)kSweepThreads * E;
    const int64_t nstrip = (n + cols_per_wg - 1) / cols_per_wg;
    const int64_t nws = (n + kWave * E - 1) / (kWave * E);
    const bool vec = ((ldk % E) == 0) && ((reinterpret_cast<uintptr_t>(K) & 15) == 0);
    const dim3 sgrid((unsigned)nstrip, (unsigned)g.nchunk);
    const dim3 sblk(kSweepThreads);
    const TimedSpan span = timing_begin(TK_SWEEP, stream);
    if (k_store == KKM_F32) {
        const float *Kf = static_cast<const float *>(K);
        if (vec)
            hipLaunchKernelGGL((spmm_row_sweep<float, true>), sgrid, sblk, 0, stream, Kf, ldk, n,
                               k, w.perm, w.offsets, labels_in, g.L, w.P, g.ldp, w.Zp, nws, w.err);
        else
            hipLaunchKernelGGL((spmm_row_sweep<float, false>), sgrid, sblk, 0, stream, Kf, ldk, n,
                               k, w.perm, w.offsets, labels_in, g.L, w.P, g.ldp, w.Zp, nws, w.err);
    } else {
        const uint16_t *Kh = static_cast<const uint16_t *>(K);
        if (vec)
            hipLaunchKernelGGL((spmm_row_sweep<uint16_t, true>), sgrid, sblk, 0, stream, Kh, ldk,
                               n, k, w.perm, w.offsets, labels_in, g.L, w.P, g.ldp, w.Zp, nws,
                               w.err);
        else
            hipLaunchKernelGGL((spmm_row_sweep<uint16_t, false>), sgrid, sblk, 0, stream, Kh, ldk,
                               n, k, w.perm, w.offsets, labels_in, g.L, w.P, g.ldp, w.Zp, nws,
                               w.err);
    }
    KKM_HIP(hipGetLastError());
    timing_end(span, stream);
    hipLaunchKernelGGL(centroid_norms, dim3((unsigned)k), dim3(256), 0, stream, w.Zp, nws,
                       w.offsets, g.L, k, w.ctilde, ctilde_out, w.err);
    KKM_HIP(hipGetLastError());
    hipLaunchKernelGGL(assign_fused, dim3(nblk), dim3(kPtsPerBlock),
                       (size_t)(2 * k + 1) * sizeof(int32_t), stream, w.P, g.ldp, w.offsets,
                       g.L, w.ctilde, diagK, labels_in, n, k, empty_policy, labels_out,
                       counts_out, n_changed, J_in, w.Jpart, w.ticket, D_out, w.err);
    KKM_HIP(hipGetLastError());
    timing_end(whole, stream);
    return KKM_OK;
}

}  // namespace kkm
