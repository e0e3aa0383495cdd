// The reassignment step on a strip-packed symmetric K (the upper triangle in
// strips of W columns, packed_row_offset): every stored entry is read once
// per step, about n^2/2 entries instead of n^2.
//
// The paper streams the whole symmetric K through a sparse product (Sec. 4.3)
// and notes that a packed triangular K is what its SYRK route lacked
// (Sec. 4.2).  With only one triangle, a stored entry K_ij (i in a strip to
// the left of j's) has to feed both S_{j,a(i)} (column j, the cluster of its
// row) and S_{i,a(j)} (row i, the cluster of its column):
//
//   column part: rows in V's CSR order, each lane owning columns of the strip
//     and keeping compensated running sums per column, flushed per (chunk,
//     cluster) segment into the stored-K sweep's partial-sum slots;
//   row part: the entries of a row left of the strip are summed per cluster
//     of their columns (the row staged in LDS in the strip's cluster-sorted
//     column order, then summed run by run), and the k sums of every (row,
//     strip) pair go to a row-part buffer; a second
//     kernel adds them up over the strips in a fixed order and folds them into
//     the cluster's first slot (and the own-cluster sums of the centroid norms).
//
// Rows of the diagonal W x W block of a strip are stored whole and take the
// column part only, so every pair is counted once in each direction.  The
// centroid norms and the fused assignment of the stored-K step then run
// unchanged.
#include "iterate.h"

namespace kkm {
namespace {

constexpr int PK_THREADS = 256;       // 4 waves, each walking its own rows over the whole strip
constexpr int PK_MAXK = 128;          // bins per row


template <typename T> struct PkRow;
template <> struct PkRow<float> {
    static constexpr int E = 4;     // elements per 16-byte load
    static constexpr int LOADS = 4; // 16-byte loads per lane and row: 16 columns
    static constexpr int ROWS = 2;  // rows per wave pass (4: two waves per SIMD instead of three, slower)
    static constexpr int BLOCKS = 2;  // workgroups per CU (VGPR budget)
    static __device__ __forceinline__ void unpack(const uint4 &w, float (&v)[E]) {
        v[0] = __uint_as_float(w.x);
        v[1] = __uint_as_float(w.y);
        v[2] = __uint_as_float(w.z);
        v[3] = __uint_as_float(w.w);
    }
};
template <> struct PkRow<uint16_t> {
    static constexpr int E = 8;
    // two 16-byte loads per lane and row: the same 16 columns per lane and
    // 1024-column strips as FP32 (32 columns per lane held the kernel's
    // registers past 256 and spilled them to memory)
    static constexpr int LOADS = 2;
    static constexpr int ROWS = 2;
    static constexpr int BLOCKS = 3;
    static __device__ __forceinline__ void unpack(const uint4 &w, float (&v)[E]) {
        const uint32_t u[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            v[2 * t] = __uint_as_float(u[t] << 16);
            v[2 * t + 1] = __uint_as_float(u[t] & 0xFFFF0000u);
        }
    }
};

struct PkArgs {
    const void *K;   // strip-packed
    int lgw;         // log2 of the strip width
    int64_t ns;      // strips
    // row-part bins by strip and CSR position: the k sums of the row at
    // position p over the columns of strip s at R + (s n + p) k (written for
    // the rows left of the strip), so that the work items of a strip write
    // their rows' sums in position order, one contiguous stretch per item
    float *R;
    int32_t *pos;    // CSR position of each point (the inverse of perm)
};

// Offset of row j's segment in strip s (s >= s_j) in the packed K, in
// elements: packed_row_offset(j) + (s - s_j) W, taken with 32-bit partial
// products (ns < 2^16 is checked on the host).
__device__ __forceinline__ int64_t pk_segment(uint32_t j, int lgw, uint32_t ns, uint32_t s) {
    const uint32_t sj = j >> lgw, u = j - (sj << lgw);
    const uint32_t tri = sj * ns - ((sj * (sj - 1)) >> 1);
    return ((int64_t)tri << (2 * lgw)) + ((int64_t)(u * (ns - sj) + (s - sj)) << lgw);
}

// One work item = (strip s, chunk q of L positions in V's CSR order).
//
// The row part of a row left of the strip: the row's W values are written to
// LDS at their column's position in the strip's columns sorted by cluster
// (a counting sort done once per item, stable, so the order is fixed), read
// back as contiguous runs of one cluster, summed run by run within a lane,
// and each cluster's run sums are added over the lanes its run spans, in lane
// order: no atomics, and every sum is taken in a fixed order.
template <typename T>
__global__ __launch_bounds__(PK_THREADS, PkRow<T>::BLOCKS) void packed_sweep(PkArgs a, Inst in,
                                                           const int32_t *labels) {
    constexpr int E = PkRow<T>::E;
    constexpr int NL = PkRow<T>::LOADS;  // 16-byte loads per lane and row
    constexpr int C = NL * E;       // columns per lane
    constexpr int W = kWave * C;    // strip width: 1024 columns
    constexpr int G = W / 256;      // 256-column groups of the own-cluster sums
    constexpr int PK_ROWS = PkRow<T>::ROWS;  // rows per wave pass
    static_assert(PK_ROWS == 2, "the row part stages the pass's two rows as pairs");
    // per wave: the staged row in sorted order, then the run sums; the flush
    // reuses the same memory for the other waves' column sums
    __shared__ __attribute__((aligned(16))) float stage[4][2][W];
    __shared__ uint16_t rank[W];          // column -> position in the sorted strip
    __shared__ uint8_t slab8[W];          // strip column labels (k for columns past n)
    __shared__ int32_t cstart[PK_MAXK + 2];  // first sorted position of each label
    if (*in.err != 0) return;
    const int64_t n = in.n;
    const int32_t k = in.k;
    const int64_t ns = a.ns;
    // items by decreasing strip: an item of strip s reads the rows of strips
    // 0 .. s, so the longest items start first and the short ones fill the end
    const int64_t nq = (n + in.L - 1) / in.L;
    const int64_t s = ns - 1 - (int64_t)blockIdx.x / nq;
    const int64_t q = (int64_t)blockIdx.x % nq;
    const int64_t p_begin = q * in.L;
    const int64_t p_end = min(n, p_begin + in.L);
    const int32_t *__restrict__ perm = in.perm;
    const int32_t *__restrict__ offsets = in.offsets;
    const T *__restrict__ K = static_cast<const T *>(a.K);

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t col0 = s * W;

    // ---- the strip's columns sorted by label (stable): rank[] and cstart[]
    for (int t = tid; t < W; t += PK_THREADS) {
        const int64_t col = col0 + t;
        slab8[t] = (uint8_t)((col < n) ? labels[col] : k);
    }
    __syncthreads();
    if (tid <= k) {  // thread t counts, then places, the columns of label t
        int32_t cnt = 0;
        for (int t = 0; t < W; ++t) cnt += (slab8[t] == tid);
        cstart[tid + 1] = cnt;
    }
    __syncthreads();
    if (tid == 0) {
        cstart[0] = 0;
        for (int t = 1; t <= k + 1; ++t) cstart[t] += cstart[t - 1];
    }
    __syncthreads();
    if (tid <= k) {
        int32_t pos = cstart[tid];
        for (int t = 0; t < W; ++t)
            if (slab8[t] == tid) rank[t] = (uint16_t)pos++;
    }
    __syncthreads();

    // Staging slot (in pairs of floats) of sorted position P: the chunk of
    // lane P / C, whose 16-byte slots (two positions each) are rotated by that
    // lane so that eight neighbouring lanes reading their chunks in step touch
    // different banks.
    auto staged = [](int P) -> int {
        const int L = P / C, o = P % C;
        return L * C + ((((o >> 1) ^ (L & 7)) << 1) | (o & 1));
    };
    // this lane's columns: col0 + u 64 E + lane E + e (u < NL, e < E); their
    // labels (own-cluster sums) and staging slots of their sorted positions,
    // packed
    uint32_t labp[C / 4];
    uint32_t rk[C / 2];
#pragma unroll
    for (int t = 0; t < C / 4; ++t) {
        uint32_t w = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int idx = 4 * t + b;
            w |= (uint32_t)slab8[(idx / E) * (kWave * E) + lane * E + (idx % E)] << (8 * b);
        }
        labp[t] = w;
    }
#pragma unroll
    for (int t = 0; t < C / 2; ++t) {
        const int i0 = 2 * t, i1 = 2 * t + 1;
        rk[t] = (uint32_t)staged(rank[(i0 / E) * (kWave * E) + lane * E + (i0 % E)]) |
                ((uint32_t)staged(rank[(i1 / E) * (kWave * E) + lane * E + (i1 % E)]) << 16);
    }
    auto lab_of = [&](int idx) -> uint32_t { return (labp[idx >> 2] >> (8 * (idx & 3))) & 0xFFu; };
    auto rank_of = [&](int idx) -> uint32_t { return (rk[idx >> 1] >> (16 * (idx & 1))) & 0xFFFFu; };
    // run starts within this lane's sorted chunk [lane C, lane C + C): bit e
    // set where position lane C + e begins a label's run or the chunk
    uint32_t runbits = 1u;
    {
        // the sorted label at position p is the largest t with cstart[t] <= p
        int32_t t = 0;
        for (int e = 0; e < C; ++e) {
            const int32_t pos = lane * C + e;
            while (cstart[t + 1] <= pos) ++t;
            if (e > 0 && cstart[t] == pos) runbits |= 1u << e;
        }
    }
    // Cluster t = lane + 64 h (h < 2: k <= 128) has its run in the chunks of
    // lanes a0 / C .. (a1 - 1) / C; its piece in each is the running sum at the
    // chunk's last position, or at a1 - 1 in the run's last chunk.  The staging
    // slots of the first three pieces and their count, packed by 16 bits.
    uint32_t pc01[2], pc2n[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int t = lane + kWave * h;
        const int32_t a0 = (t < k) ? cstart[t] : 0, a1 = (t < k) ? cstart[t + 1] : 0;
        const int32_t np = (a1 > a0) ? (a1 - 1) / C - a0 / C + 1 : 0;
        auto piece = [&](int32_t m) -> uint32_t {
            return (uint32_t)staged(m == np - 1 ? a1 - 1 : (a0 / C + m + 1) * C - 1);
        };
        const uint32_t p0 = np > 0 ? piece(0) : 0u;
        const uint32_t p1 = np > 1 ? piece(1) : p0, p2 = np > 2 ? piece(2) : p0;
        pc01[h] = p0 | (p1 << 16);
        pc2n[h] = p2 | ((uint32_t)np << 16);
    }
    float *const stg = &stage[wave][0][0];  // 2 W floats: a pair per sorted position

    float sum[C], comp[C];
#pragma unroll
    for (int u = 0; u < C; ++u) sum[u] = comp[u] = 0.f;

    int32_t lo = 0, hi = k - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (offsets[mid] <= p_begin) lo = mid;
        else hi = mid - 1;
    }
    int32_t c = lo;

    const uint32_t s32 = (uint32_t)s, ns32 = (uint32_t)ns;
    const int lgw = a.lgw;
    int32_t p = (int32_t)p_begin;
    while (p < p_end) {
        while (offsets[c + 1] <= p) ++c;  // skip empty clusters
        const int32_t seg_end = min((int32_t)p_end, offsets[c + 1]);
        // wave w takes positions pp .. pp + PK_ROWS - 1 of every 4 PK_ROWS; a
        // segment lists its points in increasing order (the CSR build is a
        // stable sort), so once a row lies right of strip s, so do the rest
        // of the segment and the wave is done with it
        auto rows_at = [&](int32_t pr0, int32_t (&jj)[PK_ROWS]) {
#pragma unroll
            for (int r = 0; r < PK_ROWS; ++r) jj[r] = (pr0 + r < seg_end) ? perm[pr0 + r] : -1;
        };
        // the rows' segments in strip s: buffer loads whose range is empty
        // (so they read zeros) for a row right of the strip or past the segment
        auto fetch = [&](const int32_t (&jj)[PK_ROWS], uint4 (&raw)[PK_ROWS][NL]) {
#pragma unroll
            for (int r = 0; r < PK_ROWS; ++r) {
                const bool here = jj[r] >= 0 && ((uint32_t)jj[r] >> lgw) <= s32;
                const T *row = here ? K + pk_segment((uint32_t)jj[r], lgw, ns32, s32) : K;
                const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                    const_cast<T *>(row), (short)0, here ? (int)(W * sizeof(T)) : 0, 0x00020000);
#pragma unroll
                for (int u = 0; u < NL; ++u) {
                    const uint32_t off = (uint32_t)((u * kWave + lane) * E * sizeof(T));
                    const auto w = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
                    raw[r][u] = make_uint4(w[0], w[1], w[2], w[3]);
                }
            }
        };
        // one pass: the column part of the pass's rows, then their row part
        auto process = [&](const uint4 (&raw)[PK_ROWS][NL], const int32_t (&jr)[PK_ROWS], int32_t pr0) {
            bool up[PK_ROWS];
#pragma unroll
            for (int r = 0; r < PK_ROWS; ++r) up[r] = jr[r] >= 0 && ((uint32_t)jr[r] >> lgw) < s32;
            // column part: the pass's rows added pairwise, then compensated
#pragma unroll
            for (int u = 0; u < NL; ++u) {
                float f[PK_ROWS][E];
#pragma unroll
                for (int r = 0; r < PK_ROWS; ++r) PkRow<T>::unpack(raw[r][u], f[r]);
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    float b = f[0][e] + f[1][e];
                    float t, er;
                    two_sum(sum[u * E + e], b, t, er);
                    sum[u * E + e] = t;
                    comp[u * E + e] += er;
                }
            }
            // row part, the pass's two rows together: each sorted position holds
            // the pair (row 0, row 1) (rows not left of the strip carry values
            // that are summed but not stored)
            if (!(up[0] || up[1])) return;  // wave-uniform
#pragma unroll
            for (int u = 0; u < NL; ++u) {
                float f0[E], f1[E];
                PkRow<T>::unpack(raw[0][u], f0);
                PkRow<T>::unpack(raw[1][u], f1);
#pragma unroll
                for (int e = 0; e < E; ++e)
                    *reinterpret_cast<float2 *>(stg + 2 * rank_of(u * E + e)) = make_float2(f0[e], f1[e]);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // this lane's sorted chunk, in place: running sums that restart
            // where a run starts, so the value at a run's last position in
            // the lane is that run's piece (branch-free; every position is
            // written)
            float acc0 = 0.f, acc1 = 0.f;
#pragma unroll
            for (int e2 = 0; e2 < C / 2; ++e2) {
                float *slot = stg + 2 * (lane * C) + 4 * (e2 ^ (lane & 7));
                const f32x4 w = *reinterpret_cast<const f32x4 *>(slot);
                const int ea = 2 * e2, eb = 2 * e2 + 1;
                f32x4 o;
                acc0 = ((runbits >> ea) & 1u) ? w[0] : acc0 + w[0];
                acc1 = ((runbits >> ea) & 1u) ? w[1] : acc1 + w[1];
                o[0] = acc0;
                o[1] = acc1;
                acc0 = ((runbits >> eb) & 1u) ? w[2] : acc0 + w[2];
                acc1 = ((runbits >> eb) & 1u) ? w[3] : acc1 + w[3];
                o[2] = acc0;
                o[3] = acc1;
                *reinterpret_cast<f32x4 *>(slot) = o;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // cluster t: its run's pieces, lane by lane.  A row not left of the
            // strip writes its sums to a scratch stretch past the bins instead
            // of skipping the stores, so every pass issues the same stores and
            // the wait for the next pass's rows, loaded before them, need not
            // wait for them too.
            float *const junk = a.R + ns * n * k;
            float *dst0 = up[0] ? a.R + (s * n + pr0) * k : junk;  // positions pr0, pr0 + 1
            float *dst1 = up[1] ? a.R + (s * n + pr0 + 1) * k : junk + k;
            const float2 *stg2 = reinterpret_cast<const float2 *>(stg);
#pragma unroll
            for (int h = 0; h < 2; ++h) {  // clusters lane, lane + 64 (k <= 128)
                if (kWave * h >= k) break;  // wave-uniform
                const int t = lane + kWave * h;
                const int32_t np = (int32_t)(pc2n[h] >> 16);
                const float2 r0 = stg2[pc01[h] & 0xFFFFu], r1 = stg2[pc01[h] >> 16],
                             r2 = stg2[pc2n[h] & 0xFFFFu];
                // the pieces in chunk order (adding 0 for the missing ones)
                float v0 = np > 0 ? r0.x : 0.f, v1 = np > 0 ? r0.y : 0.f;
                v0 += np > 1 ? r1.x : 0.f;
                v1 += np > 1 ? r1.y : 0.f;
                v0 += np > 2 ? r2.x : 0.f;
                v1 += np > 2 ? r2.y : 0.f;
                if (np > 3) {
                    const int32_t a0 = cstart[t], a1 = cstart[t + 1];
                    for (int32_t m = 3; m < np; ++m) {
                        const float2 r =
                            stg2[staged(m == np - 1 ? a1 - 1 : (a0 / C + m + 1) * C - 1)];
                        v0 += r.x;
                        v1 += r.y;
                    }
                }
                if (t < k) {
                    dst0[t] = v0;
                    dst1[t] = v1;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        };
        // row indices two passes ahead, row segments one pass ahead (issued
        // before this pass's stores); the loop is taken twice per turn so that
        // the two register sets swap roles without copies
        int32_t pp = p + wave * PK_ROWS;
        int32_t jc[PK_ROWS], jn[PK_ROWS], jq[PK_ROWS];
        rows_at(pp, jc);
        rows_at(pp + 4 * PK_ROWS, jn);
        auto advance = [&]() {
#pragma unroll
            for (int r = 0; r < PK_ROWS; ++r) {
                jc[r] = jn[r];
                jn[r] = jq[r];
            }
            pp += 4 * PK_ROWS;
        };
        auto live = [&]() { return pp < seg_end && ((uint32_t)jc[0] >> lgw) <= s32; };
        uint4 rawA[PK_ROWS][NL], rawB[PK_ROWS][NL];
        fetch(jc, rawA);
        while (true) {
            if (!live()) break;
            fetch(jn, rawB);
            rows_at(pp + 8 * PK_ROWS, jq);
            process(rawA, jc, pp);
            advance();
            if (!live()) break;
            fetch(jn, rawA);
            rows_at(pp + 8 * PK_ROWS, jq);
            process(rawB, jc, pp);
            advance();
        }
        // flush segment (q, c): the four waves' column sums, added in wave order
        __syncthreads();  // every wave is done with its staging memory
        float *const cs = &stage[0][0][0];  // [3][W] sums, then [3][W] compensations
        float *const cc = cs + 3 * W;
        if (wave > 0) {
#pragma unroll
            for (int u = 0; u < C; ++u) {
                const int lc = (u / E) * (kWave * E) + lane * E + (u % E);
                cs[(wave - 1) * W + lc] = sum[u];
                cc[(wave - 1) * W + lc] = comp[u];
            }
        }
        __syncthreads();
        if (wave == 0) {
            const int64_t slot = q + c;
            float zg[G];
#pragma unroll
            for (int g = 0; g < G; ++g) zg[g] = 0.f;
#pragma unroll
            for (int u = 0; u < C; ++u) {
                const int lc = (u / E) * (kWave * E) + lane * E + (u % E);
                float sm = sum[u], cm = comp[u];
#pragma unroll
                for (int w = 0; w < 3; ++w) {
                    float t, er;
                    two_sum(sm, cs[w * W + lc], t, er);
                    sm = t;
                    cm += cc[w * W + lc] + er;
                }
                const float tot = sm + cm;
                const int64_t col = col0 + lc;
                if (col < n) in.P[slot * in.ldp + col] = tot;
                if (lab_of(u) == (uint32_t)c) zg[lc >> 8] += tot;
            }
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const float z = wave_sum(zg[g]);
                const int64_t wg = s * G + g;
                if (lane == 0 && col0 + 256 * g < n) in.Zp[slot * in.nws + wg] = z;
            }
        }
#pragma unroll
        for (int u = 0; u < C; ++u) sum[u] = comp[u] = 0.f;
        __syncthreads();  // the column sums are read before any wave stages a row again
        p = seg_end;
    }
}

// CSR position of every point: pos[perm[p]] = p.
__global__ __launch_bounds__(256) void pk_positions(Inst in, int32_t *pos) {
    if (*in.err != 0) return;
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p < in.n) pos[in.perm[p]] = (int32_t)p;
}

// Row part of the step: for every point i and live cluster c, the bins of
// row i over the strips right of its own (fixed order, compensated), added
// to the partial sum of the cluster's first slot; a workgroup per 256 points
// (FOLD_THREADS threads, so that enough loads are in flight) also adds its
// points' own-cluster values to that slot's own-cluster sum of its 256-column
// group (point order).
constexpr int FOLD_THREADS = 1024;
__global__ __launch_bounds__(FOLD_THREADS) void packed_fold(PkArgs a, Inst in, const int32_t *labels) {
    __shared__ float own[256];
    __shared__ int32_t lab[256];
    if (*in.err != 0) return;
    const int64_t n = in.n;
    const int32_t k = in.k;
    const int64_t g = blockIdx.x;
    const int64_t i0 = g * 256;
    const int tid = threadIdx.x;
    const int32_t *__restrict__ offsets = in.offsets;
    if (tid < 256) {
        const int64_t i = i0 + tid;
        lab[tid] = (i < n) ? labels[i] : -1;
        own[tid] = 0.f;
    }
    __syncthreads();
    const int64_t pairs = (int64_t)256 * k;
    for (int64_t t = tid; t < pairs; t += FOLD_THREADS) {
        const int64_t il = t / k;
        const int32_t cl = (int32_t)(t % k);
        const int64_t i = i0 + il;
        if (i >= n) continue;
        const int64_t a0 = offsets[cl], a1 = offsets[cl + 1];
        if (a1 == a0) continue;  // empty: no column has this cluster
        const int64_t si = i >> a.lgw;
        const int64_t sk = n * k;  // floats from one strip's bins to the next
        const float *src = a.R + ((si + 1) * n + a.pos[i]) * k + cl;
        float sm = 0.f, cm = 0.f;
        const int64_t cnt = a.ns - si - 1;
        int64_t u = 0;
        for (; u + 16 <= cnt; u += 16) {  // sixteen loads in flight, added in order
            float v[16];
#pragma unroll
            for (int b = 0; b < 16; ++b) v[b] = src[(u + b) * sk];
#pragma unroll
            for (int b = 0; b < 16; ++b) {
                float x, er;
                two_sum(sm, v[b], x, er);
                sm = x;
                cm += er;
            }
        }
        for (; u < cnt; ++u) {
            float x, er;
            two_sum(sm, src[u * sk], x, er);
            sm = x;
            cm += er;
        }
        const float s1 = sm + cm;
        const int64_t slot = a0 / in.L + cl;
        in.P[slot * in.ldp + i] += s1;
        if (lab[il] == cl) own[il] = s1;
    }
    __syncthreads();
    for (int32_t cl = tid; cl < k; cl += FOLD_THREADS) {
        const int64_t a0 = offsets[cl], a1 = offsets[cl + 1];
        if (a1 == a0) continue;
        float z = 0.f;
        for (int t = 0; t < 256; ++t)
            if (lab[t] == cl) z += own[t];
        in.Zp[(a0 / in.L + cl) * in.nws + g] += z;
    }
}

int64_t pk_chunk(int64_t n) {
    // the largest power of two in [64, 8192] that still cuts the positions into
    // 24 chunks: an item's counting sort of its strip and its run pieces are
    // paid once per item, so long items win while every strip still has
    // enough of them.  Measured against the earlier rule (at most 4096, about
    // 8192 items): FP32 step 1.50 -> 0.59 ms at n=20000, 3.73 -> 2.15 ms at
    // n=60000, 5.20 -> 4.73 ms at n=100000, 19.2 -> 17.4 ms at n=200000
    int64_t L = 8192;
    while (L > 64 && (n + L - 1) / L < 24) L >>= 1;
    return L;
}

struct PkLayout {
    InstGeom g;
    int lgw;
    int64_t ns;
    size_t inst_bytes, rowpart_floats;
    int64_t n;
};

PkLayout pk_layout(int64_t n, int32_t k, int32_t k_store) {
    PkLayout m;
    m.lgw = packed_lgw(k_store);
    m.ns = packed_strips(n, m.lgw);
    m.g = inst_geometry(n, k, pk_chunk(n));
    m.inst_bytes = inst_workspace_bytes(m.g);
    // by strip and position, then 2 k floats the sweep writes for rows without sums
    m.rowpart_floats = (size_t)m.ns * (size_t)n * (size_t)k + 2 * (size_t)k;
    m.n = n;
    return m;
}

size_t pk_carve(void *base, const PkLayout &m, void **inst, float **rowpart, int32_t **pos) {
    Carver c(base);
    void *p = c.take<char>(m.inst_bytes);
    float *r = c.take<float>(m.rowpart_floats);
    int32_t *q = c.take<int32_t>((size_t)m.n);
    if (inst) *inst = p;
    if (rowpart) *rowpart = r;
    if (pos) *pos = q;
    return c.bytes();
}

kkm_status pk_step(const void *K, int32_t k_store, const float *diagK, int64_t n, int32_t k,
                   const int32_t *labels_in, int32_t empty_policy, int32_t *labels_out,
                   int32_t *counts_out, int64_t *n_changed, double *J_in, float *D_out,
                   float *ctilde_out, void *ws, size_t ws_bytes, hipStream_t stream) {
    const PkLayout m = pk_layout(n, k, k_store);
    void *iws = nullptr;
    float *rowpart = nullptr;
    int32_t *pos = nullptr;
    const size_t need = pk_carve(nullptr, m, nullptr, nullptr, nullptr);
    if (!ws || ws_bytes < need) {
        set_error("kkm_iterate_packed: workspace of %zu bytes is smaller than %zu", ws_bytes, need);
        return KKM_ERR_NOMEM;
    }
    pk_carve(ws, m, &iws, &rowpart, &pos);
    Inst in{};
    inst_carve(iws, m.g, &in, nullptr);
    in.K = K;
    in.ldk = 0;
    in.diag = diagK;
    in.lab_off = 0;
    in.empty_policy = empty_policy;
    in.counts_out = counts_out;
    in.n_changed = n_changed;
    in.J_in = J_in;
    in.D_out = D_out;
    in.ctilde_out = ctilde_out;
    in.nws = (n + 255) / 256;  // own-cluster sums per 256 columns
    PkArgs a;
    a.K = K;
    a.lgw = m.lgw;
    a.ns = m.ns;
    a.R = rowpart;
    a.pos = pos;
    const int64_t items = m.ns * m.g.nchunk;
    if (items > 0x7fffffff) {
        set_error("kkm_iterate_packed: n=%lld needs more than 2^31 work items", (long long)n);
        return KKM_ERR_UNSUPPORTED;
    }
    auto sweep = [&](hipStream_t st) -> kkm_status {
        const TimedSpan span = timing_begin(TK_SWEEP, st);
        if (k_store == KKM_F32)
            hipLaunchKernelGGL(packed_sweep<float>, dim3((unsigned)items), dim3(PK_THREADS), 0, st,
                               a, in, labels_in);
        else
            hipLaunchKernelGGL(packed_sweep<uint16_t>, dim3((unsigned)items), dim3(PK_THREADS), 0,
                               st, a, in, labels_in);
        KKM_HIP(hipGetLastError());
        timing_end(span, st);
        const TimedSpan fold = timing_begin(TK_FOLD, st);
        hipLaunchKernelGGL(pk_positions, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, in, pos);
        KKM_HIP(hipGetLastError());
        hipLaunchKernelGGL(packed_fold, dim3((unsigned)((n + 255) / 256)), dim3(FOLD_THREADS), 0, st,
                           a, in, labels_in);
        KKM_HIP(hipGetLastError());
        timing_end(fold, st);
        return KKM_OK;
    };
    return step_launch_custom(in, labels_in, labels_out, sweep, stream);
}

kkm_status pk_check(const char *who, int64_t n, int32_t k, int32_t k_store, int32_t empty_policy) {
    if (n < 1 || k < 1 || k > n) {
        set_error("%s: bad sizes (n=%lld k=%d)", who, (long long)n, k);
        return KKM_ERR_ARG;
    }
    if (k > PK_MAXK) {
        set_error("%s: k=%d exceeds the %d clusters of the packed form", who, k, PK_MAXK);
        return KKM_ERR_UNSUPPORTED;
    }
    if (k_store != KKM_F32 && k_store != KKM_BF16) {
        set_error("%s: invalid k_store %d", who, k_store);
        return KKM_ERR_ARG;
    }
    if (empty_policy != KKM_EMPTY_INF && empty_policy != KKM_EMPTY_ZERO_CENTROID) {
        set_error("%s: unknown empty-cluster policy %d", who, empty_policy);
        return KKM_ERR_ARG;
    }
    if (packed_strips(n, packed_lgw(k_store)) >= 65536) {  // the sweep's 32-bit offsets
        set_error("%s: n=%lld exceeds the packed form's 65535 strips", who, (long long)n);
        return KKM_ERR_UNSUPPORTED;
    }
    return KKM_OK;
}

}  // namespace
}  // namespace kkm

using namespace kkm;

extern "C" size_t kkm_packed_elements(int64_t n, int32_t k_store) {
    if (n < 1 || (k_store != KKM_F32 && k_store != KKM_BF16)) return 0;
    return (size_t)packed_elements(n, packed_lgw(k_store));
}

extern "C" size_t kkm_iterate_packed_workspace_bytes(int64_t n, int32_t k, int32_t k_store) {
    if (n < 1 || k < 1 || k > PK_MAXK || (k_store != KKM_F32 && k_store != KKM_BF16)) return 0;
    return pk_carve(nullptr, pk_layout(n, k, k_store), nullptr, nullptr, nullptr);
}

extern "C" kkm_status kkm_gram_packed(const float *X, int64_t n, int64_t d, int64_t ldx,
                                      int32_t kernel_type, double gamma, double coef0,
                                      int32_t degree, int32_t gram_prec, int32_t k_store, void *K,
                                      float *diagK, void *ws, size_t ws_bytes, void *stream) {
    if (n < 1 || d < 1 || ldx < d || !X || !K || !diagK) {
        set_error("kkm_gram_packed: bad sizes or NULL pointer (n=%lld d=%lld ldx=%lld)",
                  (long long)n, (long long)d, (long long)ldx);
        return KKM_ERR_ARG;
    }
    KKM_TRY(check_kernel(kernel_type, gamma, coef0, degree));
    KKM_TRY(check_dtypes(gram_prec, k_store));
    return gram_launch(X, n, d, ldx, kernel_type, gamma, coef0, degree, gram_prec, k_store, K, 0,
                       diagK, ws, ws_bytes, (hipStream_t)stream, KKM_GRAM_TRIANGLE, true);
}

extern "C" kkm_status kkm_iterate_packed(const void *K, int32_t k_store, const float *diagK,
                                         int64_t n, int32_t k, const int32_t *labels_in,
                                         int32_t empty_policy, int32_t *labels_out,
                                         int32_t *counts_out, int64_t *n_changed, double *J_in,
                                         float *D_out, float *ctilde_out, void *ws,
                                         size_t ws_bytes, void *stream) {
    KKM_TRY(pk_check("kkm_iterate_packed", n, k, k_store, empty_policy));
    if (!K || !diagK || !labels_in || !labels_out || !counts_out || !n_changed || !J_in) {
        set_error("kkm_iterate_packed: NULL pointer");
        return KKM_ERR_ARG;
    }
    if (labels_in == labels_out) {
        set_error("kkm_iterate_packed: labels_out must not alias labels_in");
        return KKM_ERR_ARG;
    }
    if ((reinterpret_cast<uintptr_t>(K) & 15) != 0) {
        set_error("kkm_iterate_packed: K must be 16-byte aligned");
        return KKM_ERR_ARG;
    }
    return pk_step(K, k_store, diagK, n, k, labels_in, empty_policy, labels_out, counts_out,
                   n_changed, J_in, D_out, ctilde_out, ws, ws_bytes, (hipStream_t)stream);
}

extern "C" kkm_status kkm_fit_packed(const float *X, int64_t n, int64_t d, int64_t ldx, int32_t k,
                                     int32_t kernel_type, double gamma, double coef0,
                                     int32_t degree, int32_t gram_prec, int32_t k_store,
                                     int32_t empty_policy, const int32_t *labels0,
                                     int32_t max_iter, int32_t check_convergence,
                                     int32_t *labels_out, double *objective, int32_t *iters,
                                     void *K_ws, double *J_trace, int64_t *changed_trace,
                                     double *times_ms, void *stream) {
    KKM_TRY(pk_check("kkm_fit_packed", n, k, k_store, empty_policy));
    if (d < 1 || ldx < d || max_iter < 0 || !X || !labels0 || !labels_out || !objective || !iters) {
        set_error("kkm_fit_packed: bad sizes or NULL pointer (n=%lld d=%lld max_iter=%d)",
                  (long long)n, (long long)d, max_iter);
        return KKM_ERR_ARG;
    }
    KKM_TRY(check_kernel(kernel_type, gamma, coef0, degree));
    KKM_TRY(check_dtypes(gram_prec, k_store));
    if (K_ws && (reinterpret_cast<uintptr_t>(K_ws) & 15) != 0) {
        set_error("kkm_fit_packed: K_ws must be 16-byte aligned");
        return KKM_ERR_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    const size_t gws = gram_workspace_bytes(n, d, gram_prec);
    void *block = nullptr, *K_own = nullptr;
    int32_t *hflag = nullptr;
    struct Guard {
        void **b, **k;
        int32_t **h;
        ~Guard() {
            if (*b) (void)hipFree(*b);
            if (*k) (void)hipFree(*k);
            if (*h) (void)hipHostFree(*h);
        }
    } guard{&block, &K_own, &hflag};
    void *K = K_ws;
    if (!K) {
        const size_t kbytes = (size_t)packed_elements(n, packed_lgw(k_store)) * elem_bytes(k_store);
        hipError_t e = hipMalloc(&K_own, kbytes);
        if (e != hipSuccess) {
            set_error("kkm_fit_packed: cannot allocate %zu bytes for K (%s)", kbytes,
                      hipGetErrorString(e));
            return KKM_ERR_NOMEM;
        }
        K = K_own;
    }
    Carver c(nullptr);
    c.take<char>(gws);
    c.take<float>((size_t)n);
    c.take<int32_t>(1);
    KKM_HIP(hipMalloc(&block, c.bytes()));
    KKM_HIP(hipHostMalloc((void **)&hflag, sizeof(int32_t), hipHostMallocDefault));
    Carver w(block);
    void *gram_ws = w.take<char>(gws);
    float *diag = w.take<float>((size_t)n);
    int32_t *flag = w.take<int32_t>(1);
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
    KKM_TRY(gram_launch(X, n, d, ldx, kernel_type, gamma, coef0, degree, gram_prec, k_store, K, 0,
                        diag, gram_ws, gws, s, KKM_GRAM_TRIANGLE, true));
    flag_nonfinite(diag, n, flag, s);
    KKM_HIP(hipGetLastError());
    KKM_HIP(hipEventRecord(ev[1], s));
    KKM_HIP(hipMemcpyAsync(hflag, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    KKM_HIP(hipStreamSynchronize(s));
    if (*hflag != 0) {
        set_error("kkm_fit_packed: diag(K) has a non-finite entry (NaN or infinity in X?)");
        return KKM_ERR_NONFINITE;
    }
    const StepFn step = [&](const int32_t *lin, int32_t *lout, int32_t *counts, int64_t *changed,
                            double *J, void *ws, size_t ws_bytes, hipStream_t st) {
        return pk_step(K, k_store, diag, n, k, lin, empty_policy, lout, counts, changed, J,
                       nullptr, nullptr, ws, ws_bytes, st);
    };
    double loop_ms[2] = {0.0, 0.0};
    KKM_TRY(run_steps(step, kkm_iterate_packed_workspace_bytes(n, k, k_store), n, k, labels0,
                      max_iter, check_convergence, labels_out, objective, iters, J_trace,
                      changed_trace, loop_ms, "kkm_fit_packed", s));
    if (times_ms) {
        float t0 = 0.f;
        (void)hipEventElapsedTime(&t0, ev[0], ev[1]);
        times_ms[0] = t0;
        times_ms[1] = loop_ms[0];
        times_ms[2] = loop_ms[1];
    }
    return KKM_OK;
}
