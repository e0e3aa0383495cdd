// One reassignment step of the paper's Algorithm 2 on gfx950, for one
// clustering problem or for many independent ones at once.
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
// Every kernel takes an instance set: either one problem passed by value, or a
// device table of live problems whose blocks are laid end to end in one grid
// (a block finds its problem by binary search in a prefix array; blocks past
// the live total exit).  The table is rewritten on the device between steps,
// so a captured sequence of launches can be replayed while problems converge
// one by one.
//
// No floating-point atomics are used: every reduction runs in a fixed order,
// so a step is bitwise repeatable.
#include "iterate.h"

namespace kkm {

namespace {

constexpr int kPtsPerBlock = 256;          // points per block in the label kernels
constexpr int kSweepThreads = 256;         // 4 waves
constexpr int kSlotWindow = 1024;          // slot -> cluster entries per LDS window

// The problem and the block index within it for a flattened grid position g;
// false when g lies past the live problems of a table.  MULTI selects the
// table form at compile time: a run-time choice between the two sources would
// leave the problem's fields in vector registers.
template <bool MULTI>
__device__ __forceinline__ bool locate(const InstSet &s, const int64_t *start, int64_t g, Inst &in,
                                       int64_t &local) {
    if constexpr (MULTI) {
        if (g >= uniform_load(start + s.count)) return false;
        const int32_t b = find_inst(start, s.count, g);
        local = g - uniform_load(start + b);
        in = uniform_load(s.table + b);
    } else {
        local = g;
        in = s.one;
    }
    return true;
}

// ---------------------------------------------------------------- 1. V in CSR form

// Per-block label histogram (column-major [k][nblk]) and range check.
template <bool MULTI>
__global__ __launch_bounds__(kPtsPerBlock) void v_block_hist(InstSet s, const int32_t *labels_all) {
    extern __shared__ int32_t sh[];  // [k] + 1
    Inst in;
    int64_t lb;
    if (!locate<MULTI>(s, s.blk_start, blockIdx.x, in, lb)) return;
    const int32_t k = in.k;
    const int32_t *labels = labels_all + in.lab_off;
    int32_t *hist = sh;
    int32_t *bad = sh + k;
    for (int c = threadIdx.x; c < k; c += blockDim.x) hist[c] = 0;
    if (threadIdx.x == 0) *bad = 0;
    __syncthreads();
    const int64_t i = lb * kPtsPerBlock + threadIdx.x;
    if (i < in.n) {
        const int32_t c = labels[i];
        if (c < 0 || c >= k)
            atomicAdd(bad, 1);
        else
            atomicAdd(&hist[c], 1);
    }
    __syncthreads();
    for (int c = threadIdx.x; c < k; c += blockDim.x) in.blk_hist[(int64_t)c * in.nblk + lb] = hist[c];
    if (threadIdx.x == 0) in.blk_bad[lb] = *bad;
}

// One workgroup per (problem, cluster): exclusive prefix of its per-block counts
// (in place) and its size.  Cluster 0's workgroup also folds the range check.
template <bool MULTI>
__global__ __launch_bounds__(256) void v_cluster_scan(InstSet s) {
    __shared__ int32_t part[256];
    __shared__ int32_t carry;
    Inst in;
    int64_t c;
    if (!locate<MULTI>(s, s.cl_start, blockIdx.x, in, c)) return;
    const int64_t nblk = in.nblk;
    int32_t *row = in.blk_hist + c * nblk;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < nblk; base += 256) {
        const int64_t i = base + threadIdx.x;
        const int32_t v = (i < nblk) ? row[i] : 0;
        part[threadIdx.x] = v;
        __syncthreads();
        // Hillis-Steele inclusive scan over 256 entries
        for (int off = 1; off < 256; off <<= 1) {
            const int32_t add = (threadIdx.x >= off) ? part[threadIdx.x - off] : 0;
            __syncthreads();
            part[threadIdx.x] += add;
            __syncthreads();
        }
        if (i < nblk) row[i] = carry + part[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 255) carry += part[255];
        __syncthreads();
    }
    if (threadIdx.x == 0) in.counts[c] = carry;
    if (c == 0) {
        int32_t t = 0;
        for (int64_t i = threadIdx.x; i < nblk; i += 256) t += in.blk_bad[i];
        part[threadIdx.x] = t;
        __syncthreads();
        if (threadIdx.x == 0) {
            int32_t u = 0;
            for (int w = 0; w < 256; ++w) u += part[w];
            *in.err = u;
        }
    }
}

// Stable scatter of point indices into V's CSR order.  Block 0 of each problem
// also publishes the row pointers and clears the step's counters.
template <bool MULTI>
__global__ __launch_bounds__(kPtsPerBlock) void v_scatter(InstSet s, const int32_t *labels_all) {
    extern __shared__ int32_t sh[];  // off[k+1], wcnt[4][k]
    Inst in;
    int64_t lb;
    if (!locate<MULTI>(s, s.blk_start, blockIdx.x, in, lb)) return;
    const int32_t k = in.k;
    const int32_t *labels = labels_all + in.lab_off;
    int32_t *off = sh;
    int32_t *wcnt = sh + (k + 1);
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    if (*in.err != 0) return;

    // exclusive scan of the cluster sizes (k <= KKM_MAX_K; one thread, then share)
    if (tid == 0) {
        int32_t run = 0;
        for (int c = 0; c < k; ++c) {
            off[c] = run;
            run += in.counts[c];
        }
        off[k] = run;
    }
    for (int c = tid; c < 4 * k; c += kPtsPerBlock) wcnt[c] = 0;
    __syncthreads();
    if (lb == 0) {
        for (int c = tid; c <= k; c += kPtsPerBlock) in.offsets[c] = off[c];
        for (int c = tid; c < k; c += kPtsPerBlock) in.counts_out[c] = 0;
        if (tid == 0) *in.n_changed = 0;
    }

    const int64_t i = lb * kPtsPerBlock + tid;
    const bool valid = i < in.n;
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
        const int64_t pos = off[c] + in.blk_hist[(int64_t)c * in.nblk + lb] + before + rank;
        in.perm[pos] = (int32_t)i;
    }
}

// ---------------------------------------------------------------- 2. row sweep of K

// Entries of K as FP32 (4 per 16-byte load) or bfloat16 (8 per 16-byte load),
// widened to float for the sums.
template <typename T> struct KRow;
template <> struct KRow<float> {
    static constexpr int E = 4;
    // 16-byte rows go through 64-bit global addresses: measured faster for FP32
    // K than buffer loads (25.7 vs 26.3 ms per 160 GB sweep)
    static constexpr bool kBuffer = false;
    static __device__ __forceinline__ void load_vec(const float *row, int64_t col, int64_t n,
                                                    float (&v)[E]) {
        if (col + E - 1 < n) {
            const f32x4 w = *reinterpret_cast<const f32x4 *>(row + col);
#pragma unroll
            for (int u = 0; u < E; ++u) v[u] = w[u];
        } else {
#pragma unroll
            for (int u = 0; u < E; ++u) v[u] = (col + u < n) ? row[col + u] : 0.f;
        }
    }
    // element loads of a row of any alignment (0 past column n)
    static __device__ __forceinline__ void load(const float *row, int64_t col, int64_t n,
                                                float (&v)[E]) {
#pragma unroll
        for (int u = 0; u < E; ++u) v[u] = (col + u < n) ? row[col + u] : 0.f;
    }
    // 16-byte load at byte offset voff of the row described by r (0 past its end)
    static __device__ __forceinline__ void load_buf(__amdgpu_buffer_rsrc_t r, uint32_t voff,
                                                    float (&v)[E]) {
        const auto w = __builtin_amdgcn_raw_buffer_load_b128(r, voff, 0, 0);
#pragma unroll
        for (int u = 0; u < E; ++u) v[u] = __uint_as_float(w[u]);
    }
};
template <> struct KRow<uint16_t> {
    static constexpr int E = 8;
    // buffer loads: one shared 32-bit lane offset instead of a 64-bit address
    // per row lets the unpacked rows fit 80 VGPRs (6 waves per SIMD instead of
    // 4); measured 13.2 vs 15.1 ms per 80 GB sweep
    static constexpr bool kBuffer = true;
    static __device__ __forceinline__ void load(const uint16_t *row, int64_t col, int64_t n,
                                                float (&v)[E]) {
#pragma unroll
        for (int u = 0; u < E; ++u)
            v[u] = (col + u < n) ? __uint_as_float((uint32_t)row[col + u] << 16) : 0.f;
    }
    static __device__ __forceinline__ void load_buf(__amdgpu_buffer_rsrc_t r, uint32_t voff,
                                                    float (&v)[E]) {
        const auto w = __builtin_amdgcn_raw_buffer_load_b128(r, voff, 0, 0);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            v[2 * u] = __uint_as_float(w[u] << 16);
            v[2 * u + 1] = __uint_as_float(w[u] & 0xffff0000u);
        }
    }
};

// Buffer resource of one K row (gfx9 raw buffer: stride 0, range in bytes,
// 32-bit data format word).  Loads through it take one 32-bit lane offset
// shared by every row, and return 0 beyond the range.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const void *row, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(row), (short)0, (int)bytes,
                                             0x00020000);
}

// The E entries of one K row at this lane's columns.  VEC: rows 16-byte
// aligned (ldk a multiple of E); otherwise element loads.
template <typename T, bool VEC>
__device__ __forceinline__ void load_row(const T *row, int64_t col, int64_t n, uint32_t voff,
                                         uint32_t rbytes, float (&v)[KRow<T>::E]) {
    if constexpr (VEC && KRow<T>::kBuffer)
        KRow<T>::load_buf(row_rsrc(row, rbytes), voff, v);
    else if constexpr (VEC)
        KRow<T>::load_vec(row, col, n, v);
    else
        KRow<T>::load(row, col, n, v);
}

// One work item = (column strip, chunk of L positions in V's CSR order).  Each
// lane owns E consecutive columns (one 16-byte load per row); a wave covers
// 64 E columns and the workgroup 256 E columns of every row it visits.  A chunk
// may span several clusters: the running sums are flushed to the partial-buffer
// slot (chunk + cluster) whenever the cluster changes; the slot is unique per
// (chunk, cluster) pair.
template <typename T, bool VEC>
__device__ __forceinline__ void sweep_item(const Inst &in, int64_t item, const int32_t *labels_all) {
    constexpr int E = KRow<T>::E;
    if (*in.err != 0) return;
    const int64_t n = in.n;
    const int32_t k = in.k;
    const int64_t L = in.L;
    const T *__restrict__ K = static_cast<const T *>(in.K);
    const int64_t ldk = in.ldk;
    const int32_t *__restrict__ perm = in.perm;
    const int32_t *__restrict__ offsets = in.offsets;
    const int32_t *__restrict__ labels = labels_all + in.lab_off;
    const int64_t nws = in.nws;
    const int64_t strip = (uint32_t)item % (uint32_t)in.nstrip;
    const int64_t q = (uint32_t)item / (uint32_t)in.nstrip;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int64_t wave_strip = strip * (kSweepThreads / kWave) + (tid >> 6);
    const int64_t col = wave_strip * (kWave * E) + (int64_t)lane * E;
    const int64_t p_begin = q * L;
    const int64_t p_end = min(n, p_begin + L);
    // VEC: every row is read with 16-byte buffer loads at this lane's byte
    // offset; columns in [n, ldk) are read but never used (their sums are not
    // stored and their labels are -1), and the range ends the row at ldk.
    const uint32_t voff = (uint32_t)(col * (int64_t)sizeof(T));
    const uint32_t rbytes = (uint32_t)(ldk * (int64_t)sizeof(T));

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
        float sum[E], e[E];
#pragma unroll
        for (int u = 0; u < E; ++u) sum[u] = e[u] = 0.f;
        for (; p + 8 <= seg_end; p += 8) {
            // pairwise sum of 8 rows, ((r0+r1)+(r2+r3)) + ((r4+r5)+(r6+r7)), taken
            // as two halves so that only four rows are unpacked at a time
            float blk[E];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                float v[4][E];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t j = __builtin_amdgcn_readfirstlane(perm[p + 4 * h + r]);
                    load_row<T, VEC>(K + j * ldk, col, n, voff, rbytes, v[r]);
                }
#pragma unroll
                for (int u = 0; u < E; ++u) {
                    const float q = (v[0][u] + v[1][u]) + (v[2][u] + v[3][u]);
                    blk[u] = h ? blk[u] + q : q;
                }
            }
#pragma unroll
            for (int u = 0; u < E; ++u) {
                float t, er;
                two_sum(sum[u], blk[u], t, er);
                sum[u] = t;
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
                load_row<T, VEC>(K + j * ldk, col, n, voff, rbytes, v);
#pragma unroll
                for (int u = 0; u < E; ++u) blk[u] += v[u];
            }
#pragma unroll
            for (int u = 0; u < E; ++u) {
                float t, er;
                two_sum(sum[u], blk[u], t, er);
                sum[u] = t;
                e[u] += er;
            }
        }
        float tot[E];
#pragma unroll
        for (int u = 0; u < E; ++u) tot[u] = sum[u] + e[u];
        const int64_t slot = q + c;
        if (col < n) {
            float *dst = in.P + slot * in.ldp + col;
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
        if (lane == 0 && wave_strip < nws) in.Zp[slot * nws + wave_strip] = z;
    }
}

// One workgroup per item.  For a table the grid covers the items of every
// problem the table can hold and workgroups past the live total exit.  (A
// persistent grid looping over contiguous item ranges measured 4.5% slower:
// its loop raised the kernel from 64 to 76 VGPRs, 6 waves per SIMD instead of
// 8.)
template <typename T, bool VEC, bool MULTI>
__global__ __launch_bounds__(kSweepThreads) void spmm_row_sweep(InstSet s,
                                                                const int32_t *labels_all) {
    Inst in;
    int64_t item;
    if (!locate<MULTI>(s, s.item_start, blockIdx.x, in, item)) return;
    sweep_item<T, VEC>(in, item, labels_all);
}

// ---------------------------------------------------------------- 3. centroid norms

// One workgroup per (problem, cluster): ||c_c||^2 = (1/|c|^2) sum_{i in c} S_ic,
// summing the z partials of the cluster's segments in a fixed order.
template <int E, bool MULTI>
__global__ __launch_bounds__(256) void centroid_norms(InstSet s) {
    __shared__ float ss[256], sc[256];
    Inst in;
    int64_t c;
    if (!locate<MULTI>(s, s.cl_start, blockIdx.x, in, c)) return;
    if (*in.err != 0) return;
    const int64_t nws = in.nws;
    const int64_t a = in.offsets[c], e = in.offsets[c + 1];
    const int64_t cnt = e - a;
    float sum = 0.f, comp = 0.f;
    if (cnt > 0) {
        const int64_t q0 = a / in.L, q1 = (e - 1) / in.L;
        const int64_t total = (q1 - q0 + 1) * nws;
        for (int64_t t = threadIdx.x; t < total; t += 256) {
            const int64_t q = q0 + t / nws;
            const int64_t w = t % nws;
            float u, er;
            two_sum(sum, in.Zp[(q + c) * nws + w], u, er);
            sum = u;
            comp += er;
        }
    }
    ss[threadIdx.x] = sum;
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
        in.ctilde[c] = v;
        if (in.ctilde_out) in.ctilde_out[c] = v;
    }
}

// ---------------------------------------------------------------- 4. distances + argmin + histogram

template <bool MULTI>
__global__ __launch_bounds__(kPtsPerBlock) void assign_fused(InstSet s,
                                                             const int32_t *labels_in_all,
                                                             int32_t *labels_out_all) {
    extern __shared__ int32_t sh[];  // off[k+1], hist[k], seg[kSlotWindow]
    __shared__ double wJ[kPtsPerBlock / kWave];
    __shared__ long long wC[kPtsPerBlock / kWave];
    Inst in;
    int64_t lb;
    if (!locate<MULTI>(s, s.blk_start, blockIdx.x, in, lb)) return;
    const int32_t k = in.k;
    const int64_t L = in.L, ldp = in.ldp;
    const float *__restrict__ P = in.P;
    const int32_t *__restrict__ labels_in = labels_in_all + in.lab_off;
    int32_t *__restrict__ labels_out = labels_out_all + in.lab_off;
    int32_t *off = sh;
    int32_t *hist = sh + (k + 1);
    int32_t *seg = hist + k;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    if (*in.err != 0) {
        if (lb == 0 && tid == 0) {
            *in.n_changed = -1;
            *in.J_in = __builtin_nan("");
        }
        return;
    }
    for (int c = tid; c <= k; c += kPtsPerBlock) off[c] = in.offsets[c];
    for (int c = tid; c < k; c += kPtsPerBlock) hist[c] = 0;
    __syncthreads();

    const int64_t i = lb * kPtsPerBlock + tid;
    const bool valid = i < in.n;
    const float dii = valid ? in.diag[i] : 0.f;
    const int32_t a_in = valid ? labels_in[i] : -1;
    float best = __builtin_inff();
    int32_t arg = -1;
    float own = 0.f;
    auto visit = [&](int32_t c, float dic) {
        if (in.D_out) in.D_out[i * k + c] = dic;
        if (c == a_in) own = dic;
        if (dic < best) {
            best = dic;
            arg = c;
        }
    };
    const float empty_d = (in.empty_policy == KKM_EMPTY_ZERO_CENTROID) ? dii : __builtin_inff();
    // S_ic of cluster `cur` is the compensated sum of its segments' partials, in
    // CSR order; clusters without a segment are empty
    int32_t cur = -1;
    float sum = 0.f, comp = 0.f;
    auto close = [&]() {
        const float e = (sum + comp) / (float)(off[cur + 1] - off[cur]);
        visit(cur, fmaf(-2.0f, e, dii) + in.ctilde[cur]);
    };
    // Segment (q, c) of the sweep sits in slot q + c; slots rise with CSR
    // position.  A window of the slot -> cluster map is built in LDS, then each
    // thread reads its column of the window's partials eight loads at a time.
    const int64_t nslot = (in.n + L - 1) / L + k;
    for (int64_t s0 = 0; s0 < nslot; s0 += kSlotWindow) {
        const int w = (int)min((int64_t)kSlotWindow, nslot - s0);
        for (int t = tid; t < w; t += kPtsPerBlock) seg[t] = -1;
        __syncthreads();
        for (int c = tid; c < k; c += kPtsPerBlock) {
            const int64_t lo = off[c], hi = off[c + 1];
            if (hi > lo) {
                const int64_t a = max(lo / L + c, s0), b = min((hi - 1) / L + c, s0 + w - 1);
                for (int64_t t = a; t <= b; ++t) seg[t - s0] = c;
            }
        }
        __syncthreads();
        if (valid) {
            for (int t0 = 0; t0 < w; t0 += 8) {
                float v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int32_t c = (t0 + u < w) ? seg[t0 + u] : -1;
                    v[u] = (c >= 0) ? P[(s0 + t0 + u) * ldp + i] : 0.f;
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int32_t c = (t0 + u < w) ? seg[t0 + u] : -1;
                    if (c < 0) continue;
                    if (c != cur) {
                        if (cur >= 0) close();
                        for (int32_t e = cur + 1; e < c; ++e) visit(e, empty_d);
                        cur = c;
                        sum = comp = 0.f;
                    }
                    float x, er;
                    two_sum(sum, v[u], x, er);
                    sum = x;
                    comp += er;
                }
            }
        }
        __syncthreads();
    }
    double own_d = 0.0;
    long long changed = 0;
    if (valid) {
        if (cur >= 0) close();
        for (int32_t e = cur + 1; e < k; ++e) visit(e, empty_d);
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
        in.Jpart[lb] = bj;
        if (bc) atomicAdd((unsigned long long *)in.n_changed, (unsigned long long)bc);
    }
    for (int c = tid; c < k; c += kPtsPerBlock)
        if (hist[c]) atomicAdd(&in.counts_out[c], hist[c]);
}

// J of the input labels: each problem's block partials summed in a fixed
// order by one workgroup (a kernel of its own: a device-wide release fence
// in every assignment workgroup costs far more than this launch).
template <bool MULTI>
__global__ __launch_bounds__(kPtsPerBlock) void j_finalize(InstSet s) {
    __shared__ double wJ[kPtsPerBlock / kWave];
    Inst in;
    if constexpr (MULTI) {
        const int32_t b = blockIdx.x;
        if (b >= s.count) return;
        if (uniform_load(s.blk_start + b) >= uniform_load(s.blk_start + s.count)) return;
        in = uniform_load(s.table + b);
    } else {
        in = s.one;
    }
    if (*in.err != 0) return;  // the assignment has published NaN
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double acc = 0.0;
    for (int64_t t = tid; t < in.nblk; t += kPtsPerBlock) acc += in.Jpart[t];
    const double ws = wave_sum(acc);
    if (lane == 0) wJ[wave] = ws;
    __syncthreads();
    if (tid == 0) {
        double tot = 0.0;
        for (int w = 0; w < kPtsPerBlock / kWave; ++w) tot += wJ[w];
        *in.J_in = tot;
    }
}

// Geometry shared by the workspace sizing and the kernels.
int64_t chunk_rows(int64_t n) {
    // the largest power of two in [64, 4096] that still gives about 8192 sweep
    // workgroups of 1024 FP32 columns (the partial sums cost slots * n floats)
    const int64_t nstrip = (n + 1023) / 1024;
    int64_t L = 4096;
    while (L > 64 && ((n + L - 1) / L) * nstrip < 8192) L >>= 1;
    return L;
}

}  // namespace

InstGeom inst_geometry(int64_t n, int32_t k, int64_t L) {
    InstGeom g;
    g.n = n;
    g.k = k;
    g.L = (L > 0) ? L : chunk_rows(n);
    g.nblk = (n + kPtsPerBlock - 1) / kPtsPerBlock;
    g.nchunk = (n + g.L - 1) / g.L;
    g.slots = g.nchunk + k;
    g.ldp = (n + 63) & ~int64_t(63);
    g.nws_max = (n + kWave * 4 - 1) / (kWave * 4);  // FP32 K: the most wave strips
    return g;
}

size_t inst_workspace_bytes(const InstGeom &g) {
    size_t bytes = 0;
    inst_carve(nullptr, g, nullptr, &bytes);
    return bytes;
}

void inst_carve(void *base, const InstGeom &g, Inst *in, size_t *bytes) {
    Carver c(base);
    int32_t *perm = c.take<int32_t>((size_t)g.n);
    int32_t *offsets = c.take<int32_t>((size_t)g.k + 1);
    int32_t *counts = c.take<int32_t>((size_t)g.k);
    int32_t *blk_hist = c.take<int32_t>((size_t)g.k * (size_t)g.nblk);
    int32_t *blk_bad = c.take<int32_t>((size_t)g.nblk);
    int32_t *err = c.take<int32_t>(1);
    float *P = c.take<float>((size_t)g.slots * (size_t)g.ldp);
    float *Zp = c.take<float>((size_t)g.slots * (size_t)g.nws_max);
    float *ctilde = c.take<float>((size_t)g.k);
    double *Jpart = c.take<double>((size_t)g.nblk);
    if (bytes) *bytes = c.bytes();
    if (!in) return;
    in->n = g.n;
    in->k = g.k;
    in->L = g.L;
    in->nblk = g.nblk;
    in->ldp = g.ldp;
    in->perm = perm;
    in->offsets = offsets;
    in->counts = counts;
    in->blk_hist = blk_hist;
    in->blk_bad = blk_bad;
    in->err = err;
    in->P = P;
    in->Zp = Zp;
    in->ctilde = ctilde;
    in->Jpart = Jpart;
}

int64_t inst_sweep_items(const InstGeom &g, int32_t k_store) {
    const int64_t cols = (int64_t)kSweepThreads * ((k_store == KKM_BF16) ? 8 : 4);
    return ((g.n + cols - 1) / cols) * g.nchunk;
}

void inst_set_store(Inst *in, int32_t k_store) {
    const int64_t E = (k_store == KKM_BF16) ? 8 : 4;
    in->nstrip = (in->n + kSweepThreads * E - 1) / (kSweepThreads * E);
    in->nws = (in->n + kWave * E - 1) / (kWave * E);
}

namespace {

template <bool MULTI>
kkm_status step_launch_t(const InstSet &s, int64_t total_blocks, int64_t total_clusters,
                         int64_t sweep_grid, int32_t max_k, int32_t k_store, bool vec,
                         const int32_t *labels_in, int32_t *labels_out, hipStream_t stream) {
    const dim3 pb(kPtsPerBlock);
    const TimedSpan whole = timing_begin(TK_ITERATE, stream);
    hipLaunchKernelGGL(v_block_hist<MULTI>, dim3((unsigned)total_blocks), pb,
                       (size_t)(max_k + 1) * sizeof(int32_t), stream, s, labels_in);
    KKM_HIP(hipGetLastError());
    hipLaunchKernelGGL(v_cluster_scan<MULTI>, dim3((unsigned)total_clusters), dim3(256), 0, stream, s);
    KKM_HIP(hipGetLastError());
    hipLaunchKernelGGL(v_scatter<MULTI>, dim3((unsigned)total_blocks), pb,
                       (size_t)(max_k + 1 + 4 * max_k) * sizeof(int32_t), stream, s, labels_in);
    KKM_HIP(hipGetLastError());
    const dim3 sg((unsigned)sweep_grid), sb(kSweepThreads);
    const TimedSpan span = timing_begin(TK_SWEEP, stream);
    if (k_store == KKM_F32) {
        if (vec)
            hipLaunchKernelGGL((spmm_row_sweep<float, true, MULTI>), sg, sb, 0, stream, s, labels_in);
        else
            hipLaunchKernelGGL((spmm_row_sweep<float, false, MULTI>), sg, sb, 0, stream, s, labels_in);
    } else {
        if (vec)
            hipLaunchKernelGGL((spmm_row_sweep<uint16_t, true, MULTI>), sg, sb, 0, stream, s, labels_in);
        else
            hipLaunchKernelGGL((spmm_row_sweep<uint16_t, false, MULTI>), sg, sb, 0, stream, s, labels_in);
    }
    KKM_HIP(hipGetLastError());
    timing_end(span, stream);
    if (k_store == KKM_F32)
        hipLaunchKernelGGL((centroid_norms<4, MULTI>), dim3((unsigned)total_clusters), dim3(256), 0, stream, s);
    else
        hipLaunchKernelGGL((centroid_norms<8, MULTI>), dim3((unsigned)total_clusters), dim3(256), 0, stream, s);
    KKM_HIP(hipGetLastError());
    hipLaunchKernelGGL(assign_fused<MULTI>, dim3((unsigned)total_blocks), pb,
                       (size_t)(2 * max_k + 1 + kSlotWindow) * sizeof(int32_t), stream, s,
                       labels_in, labels_out);
    KKM_HIP(hipGetLastError());
    hipLaunchKernelGGL(j_finalize<MULTI>, dim3(MULTI ? (unsigned)s.count : 1u), pb, 0, stream, s);
    KKM_HIP(hipGetLastError());
    timing_end(whole, stream);
    return KKM_OK;
}

}  // namespace

kkm_status step_launch(const InstSet &s, int64_t total_blocks, int64_t total_clusters,
                       int64_t sweep_grid, int32_t max_k, int32_t k_store, bool vec,
                       const int32_t *labels_in, int32_t *labels_out, hipStream_t stream) {
    if (s.table)
        return step_launch_t<true>(s, total_blocks, total_clusters, sweep_grid, max_k, k_store,
                                   vec, labels_in, labels_out, stream);
    return step_launch_t<false>(s, total_blocks, total_clusters, sweep_grid, max_k, k_store, vec,
                                labels_in, labels_out, stream);
}

// One step of a single problem whose sweep is supplied by the caller: the CSR
// build of V, then `sweep` (it fills in.P and in.Zp as spmm_row_sweep does:
// slot q + c of P holds, for every column, the sum over the positions of
// chunk q in cluster c, and Zp[(q + c) nws + w] that slot's own-cluster sum
// over the w-th strip of in.n / in.nws columns), then the centroid norms, the
// fused assignment and the objective.
kkm_status step_launch_custom(const Inst &in, const int32_t *labels_in, int32_t *labels_out,
                              const std::function<kkm_status(hipStream_t)> &sweep,
                              hipStream_t stream) {
    InstSet s{};
    s.count = 1;
    s.one = in;
    const int32_t k = in.k;
    const dim3 pb(kPtsPerBlock);
    const TimedSpan whole = timing_begin(TK_ITERATE, stream);
    hipLaunchKernelGGL(v_block_hist<false>, dim3((unsigned)in.nblk), pb,
                       (size_t)(k + 1) * sizeof(int32_t), stream, s, labels_in);
    KKM_HIP(hipGetLastError());
    hipLaunchKernelGGL(v_cluster_scan<false>, dim3((unsigned)k), dim3(256), 0, stream, s);
    KKM_HIP(hipGetLastError());
    hipLaunchKernelGGL(v_scatter<false>, dim3((unsigned)in.nblk), pb,
                       (size_t)(k + 1 + 4 * k) * sizeof(int32_t), stream, s, labels_in);
    KKM_HIP(hipGetLastError());
    KKM_TRY(sweep(stream));  // times its own launches
    hipLaunchKernelGGL((centroid_norms<4, false>), dim3((unsigned)k), dim3(256), 0, stream, s);
    KKM_HIP(hipGetLastError());
    hipLaunchKernelGGL(assign_fused<false>, dim3((unsigned)in.nblk), pb,
                       (size_t)(2 * k + 1 + kSlotWindow) * sizeof(int32_t), stream, s, labels_in,
                       labels_out);
    KKM_HIP(hipGetLastError());
    hipLaunchKernelGGL(j_finalize<false>, dim3(1u), pb, 0, stream, s);
    KKM_HIP(hipGetLastError());
    timing_end(whole, stream);
    return KKM_OK;
}

// V in CSR form for one problem (used by the feature-space Lloyd iterations):
// the first three kernels of a step on a set of one.
kkm_status vcsr_build(const int32_t *labels, int64_t n, int32_t k, int32_t *blk_hist,
                      int32_t *blk_bad, int32_t *err, int32_t *counts, int32_t *perm,
                      int32_t *offsets, int32_t *counts_out, int64_t *n_changed,
                      hipStream_t stream) {
    InstSet s{};
    s.count = 1;
    Inst &in = s.one;
    in.n = n;
    in.k = k;
    in.nblk = (n + kPtsPerBlock - 1) / kPtsPerBlock;
    in.blk_hist = blk_hist;
    in.blk_bad = blk_bad;
    in.err = err;
    in.counts = counts;
    in.perm = perm;
    in.offsets = offsets;
    in.counts_out = counts_out;
    in.n_changed = n_changed;
    const dim3 pb(kPtsPerBlock);
    hipLaunchKernelGGL(v_block_hist<false>, dim3((unsigned)in.nblk), pb, (size_t)(k + 1) * sizeof(int32_t),
                       stream, s, labels);
    KKM_HIP(hipGetLastError());
    hipLaunchKernelGGL(v_cluster_scan<false>, dim3((unsigned)k), dim3(256), 0, stream, s);
    KKM_HIP(hipGetLastError());
    hipLaunchKernelGGL(v_scatter<false>, dim3((unsigned)in.nblk), pb,
                       (size_t)(k + 1 + 4 * k) * sizeof(int32_t), stream, s, labels);
    KKM_HIP(hipGetLastError());
    return KKM_OK;
}

size_t iterate_workspace_bytes(int64_t n, int32_t k) {
    return inst_workspace_bytes(inst_geometry(n, k, 0));
}

kkm_status iterate_launch(const void *K, int32_t k_store, int64_t ldk, const float *diagK,
                          int64_t n, int32_t k, const int32_t *labels_in, int32_t empty_policy,
                          int32_t *labels_out, int32_t *counts_out, int64_t *n_changed,
                          double *J_in, float *D_out, float *ctilde_out, void *ws,
                          size_t ws_bytes, hipStream_t stream) {
    const InstGeom g = inst_geometry(n, k, 0);
    size_t need = 0;
    inst_carve(nullptr, g, nullptr, &need);
    if (ws == nullptr || ws_bytes < need) {
        set_error("kkm_iterate: workspace of %zu bytes is smaller than %zu", ws_bytes, need);
        return KKM_ERR_NOMEM;
    }
    InstSet s{};
    s.count = 1;
    Inst &in = s.one;
    inst_carve(ws, g, &in, nullptr);
    in.K = K;
    in.ldk = ldk;
    in.diag = diagK;
    in.lab_off = 0;
    in.empty_policy = empty_policy;
    in.counts_out = counts_out;
    in.n_changed = n_changed;
    in.J_in = J_in;
    in.D_out = D_out;
    in.ctilde_out = ctilde_out;
    inst_set_store(&in, k_store);
    const int E = (k_store == KKM_BF16) ? 8 : 4;
    const bool vec = ((ldk % E) == 0) && ((reinterpret_cast<uintptr_t>(K) & 15) == 0);
    return step_launch(s, g.nblk, k, inst_sweep_items(g, k_store), k, k_store, vec, labels_in,
                       labels_out, stream);
}

}  // namespace kkm
