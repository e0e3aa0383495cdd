// Batched Kernel K-means: many independent problems of uneven sizes (each
// the paper's Algorithm 2 on its own points) sharing every launch.
//
// One run:
//   1. prologue   one wave per row of every problem: squared norm (FP32
//                 product) or the row rounded to BF16 / FP8 with its norm.
//   2. Gram       one persistent launch; workgroups pop chunks of 128 x 128
//                 upper-triangle tiles from a device counter.  Problems are
//                 queued costliest tile first (largest d, then largest n), so
//                 the cheapest tiles fill the tail of the queue.
//   3. loop       the six step kernels over a device table of the problems
//                 still running, then a control kernel that retires the
//                 problems whose step changed no label (or that reached
//                 max_iter) and rewrites the table in place.  The grid sizes
//                 are those of the whole batch, so the same launches can be
//                 captured once (one graph per label-buffer parity) and
//                 replayed.
//   4. final pass one more step over the problems that stopped at max_iter,
//                 for the objective of their final labels.
//
// Each problem's arithmetic is exactly that of the single-problem path (the
// same tile code, the same step kernels, the same chunking when chunk_rows
// is 0), so its labels, iteration count and objective match kkm_fit_ex bit
// for bit.
#include <stdio.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include <type_traits>

#include "gram_tile.h"
#include "iterate.h"

namespace kkm {

namespace {

using namespace gt;

constexpr int kQueueChunk = 4;     // tiles per queue pop
constexpr int kCtlThreads = 1024;  // the control kernel is one workgroup

enum : int32_t { ST_LIVE = 0, ST_CONVERGED = 1, ST_FINAL = 2, ST_DONE = 3, ST_BADLABEL = -1 };

// Prologue view of one problem.
struct RowSrc {
    const float *X;
    int64_t ldx, d, dpad;
    unsigned char *Xq;  // [n][dpad] elements of the product's type, or null
    float *nrm, *scale;
};

// Product view of one problem (only the member of its precision is used).
struct GramSrc {
    F32Tile f;
    LowpTile q;
};

// ---------------------------------------------------------------- 1. prologue

template <int PREC>
__global__ __launch_bounds__(256) void batch_prologue(const RowSrc *tab, const int64_t *row_start,
                                                      int32_t count) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t row = (int64_t)blockIdx.x * 4 + wave;
    if (row >= uniform_load(row_start + count)) return;
    const int32_t b = find_inst(row_start, count, row);
    const RowSrc r = uniform_load(tab + b);
    const int64_t i = row - uniform_load(row_start + b);
    const int lane = threadIdx.x & 63;
    if constexpr (PREC == KKM_F32) {
        sqnorm_row(r.X + i * r.ldx, r.d, r.nrm + i, lane);
    } else {
        const int64_t eb = (PREC == KKM_BF16) ? 2 : 1;
        quantize_row<PREC>(r.X + i * r.ldx, r.d, r.dpad, r.Xq + i * r.dpad * eb, r.nrm + i,
                           r.scale + i, lane);
    }
}

// ---------------------------------------------------------------- 2. Gram

// Persistent: every workgroup pops chunks of kQueueChunk tiles until the
// counter passes the tile total, so every wave reaches the exit.  Two
// workgroups per CU, double-buffered slabs (the persistent loop keeps more
// state live than the single-problem kernel, which fits three).
template <int PREC, typename OUT>
__global__ __launch_bounds__(GTHREADS, 2) void batch_gram(const GramSrc *tab,
                                                          const int64_t *tile_start,
                                                          int32_t count,
                                                          unsigned long long *queue) {
    __shared__ __attribute__((aligned(16))) std::conditional_t<PREC == KKM_F32, F32Lds, LowpLds<true>> lds;
    __shared__ long long next;
    const int64_t total = uniform_load(tile_start + count);
    for (;;) {
        if (threadIdx.x == 0) next = (long long)atomicAdd(queue, (unsigned long long)kQueueChunk);
        __syncthreads();
        const int64_t t0 = next;
        __syncthreads();
        if (t0 >= total) break;
        const int64_t t1 = min(total, t0 + (int64_t)kQueueChunk);
        for (int64_t t = t0; t < t1; ++t) {
            const int32_t b = find_inst(tile_start, count, t);
            int64_t bi, bj;
            tile_coords(t - uniform_load(tile_start + b), bi, bj);
            if constexpr (PREC == KKM_F32)
                f32_tile<OUT>(uniform_load(&tab[b].f), bi, bj, lds);
            else
                lowp_tile<PREC, OUT>(uniform_load(&tab[b].q), bi, bj, lds);
        }
    }
}

__global__ void fill_u64(unsigned long long *p, unsigned long long v) { *p = v; }

// ---------------------------------------------------------------- 3. control

struct Ctl {
    const Inst *full;  // every problem, in input order
    Inst *live;        // the table the step kernels read
    int64_t *blk_start, *cl_start, *item_start;  // [count + 1]
    int32_t *status, *iters;                     // [count]
    double *objective;                           // [count]
    const int64_t *n_changed;                    // [count], written by the step
    const double *J;                             // [count], written by the step
    int32_t *step;                               // steps taken so far
    int32_t *n_live;                             // size of the live table
    int32_t count, max_iter, check_convergence;
};

enum : int32_t { CTL_INIT = 0, CTL_AFTER_STEP = 1, CTL_SELECT_FINAL = 2, CTL_AFTER_FINAL = 3 };

// Exclusive prefix sums of v[0..3] over the workgroup, in thread order, and
// their totals.
__device__ void block_scan4(const int64_t v[4], int64_t excl[4], int64_t tot[4]) {
    __shared__ int64_t wsum[kCtlThreads / kWave][4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int64_t inc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        long long x = v[q];
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const long long y = __shfl_up(x, off, kWave);
            if (lane >= off) x += y;
        }
        inc[q] = x;
        if (lane == kWave - 1) wsum[wave][q] = x;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        int64_t before = 0, all = 0;
        for (int w = 0; w < kCtlThreads / kWave; ++w) {
            if (w < wave) before += wsum[w][q];
            all += wsum[w][q];
        }
        excl[q] = before + inc[q] - v[q];
        tot[q] = all;
    }
    __syncthreads();
}

// Rewrites the live table with the problems whose status is `want`, in
// input order, and fills the prefix arrays (entries past the last one hold
// the totals).
__device__ void compact(const Ctl &c, int32_t want) {
    int64_t base[4] = {0, 0, 0, 0};
    for (int32_t b0 = 0; b0 < c.count; b0 += kCtlThreads) {
        const int32_t b = b0 + (int32_t)threadIdx.x;
        const bool sel = b < c.count && c.status[b] == want;
        int64_t v[4] = {0, 0, 0, 0};
        if (sel) {
            const Inst &in = c.full[b];
            v[0] = 1;
            v[1] = in.nblk;
            v[2] = in.k;
            v[3] = in.nstrip * ((in.n + in.L - 1) / in.L);
        }
        int64_t ex[4], tot[4];
        block_scan4(v, ex, tot);
        if (sel) {
            const int64_t pos = base[0] + ex[0];
            c.live[pos] = c.full[b];
            c.blk_start[pos] = base[1] + ex[1];
            c.cl_start[pos] = base[2] + ex[2];
            c.item_start[pos] = base[3] + ex[3];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) base[q] += tot[q];
    }
    for (int64_t p = base[0] + threadIdx.x; p <= c.count; p += kCtlThreads) {
        c.blk_start[p] = base[1];
        c.cl_start[p] = base[2];
        c.item_start[p] = base[3];
    }
    if (threadIdx.x == 0) *c.n_live = (int32_t)base[0];
}

__global__ __launch_bounds__(kCtlThreads) void batch_control(Ctl c, int32_t mode) {
    const int32_t t = *c.step;
    __syncthreads();
    for (int32_t b = threadIdx.x; b < c.count; b += kCtlThreads) {
        if (mode == CTL_INIT) {
            c.status[b] = (c.max_iter > 0) ? ST_LIVE : ST_FINAL;
            c.iters[b] = 0;
            c.objective[b] = 0.0;
        } else if (mode == CTL_AFTER_STEP && c.status[b] == ST_LIVE) {
            const int64_t ch = c.n_changed[b];
            if (ch < 0) {
                c.status[b] = ST_BADLABEL;
            } else if (c.check_convergence && ch == 0) {
                // the step's input labels are final: its J is their objective
                c.status[b] = ST_CONVERGED;
                c.iters[b] = t + 1;
                c.objective[b] = c.J[b];
            } else if (t + 1 >= c.max_iter) {
                c.status[b] = ST_FINAL;
                c.iters[b] = c.max_iter;
            }
        } else if (mode == CTL_AFTER_FINAL && c.status[b] == ST_FINAL) {
            if (c.n_changed[b] < 0) {
                c.status[b] = ST_BADLABEL;
            } else {
                c.status[b] = ST_DONE;
                c.objective[b] = c.J[b];
            }
        }
    }
    __syncthreads();
    if (mode == CTL_INIT || mode == CTL_AFTER_STEP) compact(c, ST_LIVE);
    else if (mode == CTL_SELECT_FINAL) compact(c, ST_FINAL);
    if (threadIdx.x == 0) {
        if (mode == CTL_INIT) *c.step = 0;
        else if (mode == CTL_AFTER_STEP) *c.step = t + 1;
    }
}

// ---------------------------------------------------------------- host plan

struct Plan {
    int32_t count = 0;
    int64_t total_n = 0, total_blocks = 0, total_clusters = 0, total_items = 0, total_tiles = 0;
    int32_t max_k = 0;
    size_t bytes = 0;
    // device pointers (valid when carved from a real base)
    float *diag = nullptr;
    int32_t *lab[2] = {nullptr, nullptr};
    Inst *full = nullptr, *live = nullptr;
    GramSrc *gtab = nullptr;
    RowSrc *rtab = nullptr;
    int64_t *blk_start = nullptr, *cl_start = nullptr, *item_start = nullptr;
    int64_t *tile_start = nullptr, *row_start = nullptr;
    int32_t *status = nullptr, *iters = nullptr, *step = nullptr, *n_live = nullptr;
    int32_t *flag = nullptr;
    double *objective = nullptr, *J = nullptr;
    int64_t *n_changed = nullptr;
    unsigned long long *queue = nullptr;
    // host tables
    std::vector<Inst> h_full;
    std::vector<GramSrc> h_gtab;
    std::vector<RowSrc> h_rtab;
    std::vector<int64_t> h_tile_start, h_row_start;
};

kkm_status check_instances(const kkm_instance *inst, int32_t count, int32_t gram_prec,
                           int32_t k_store) {
    if (!inst || count < 1) {
        set_error("kkm_fit_batched: need at least one problem (count=%d)", count);
        return KKM_ERR_ARG;
    }
    KKM_TRY(check_dtypes(gram_prec, k_store));
    for (int32_t b = 0; b < count; ++b) {
        const kkm_instance &p = inst[b];
        if (!p.X || p.n < 1 || p.d < 1 || p.ldx < p.d || p.k < 1 || p.k > p.n) {
            set_error("kkm_fit_batched: problem %d has bad sizes or a NULL X (n=%lld d=%lld "
                      "ldx=%lld k=%d)", b, (long long)p.n, (long long)p.d, (long long)p.ldx, p.k);
            return KKM_ERR_ARG;
        }
        if (p.k > KKM_MAX_K) {
            set_error("kkm_fit_batched: problem %d has k=%d > KKM_MAX_K=%d", b, p.k, KKM_MAX_K);
            return KKM_ERR_UNSUPPORTED;
        }
        if (gram_prec != KKM_F32 && !lowp_rows_fit(p.d, gram_prec)) {
            set_error("kkm_fit_batched: problem %d has d=%lld, too large for the BF16 / FP8 "
                      "product's 32-bit row ranges", b, (long long)p.d);
            return KKM_ERR_UNSUPPORTED;
        }
        if (p.chunk_rows < 0 || p.chunk_rows > (1 << 20)) {
            set_error("kkm_fit_batched: problem %d has chunk_rows=%d outside [0, 2^20]", b,
                      p.chunk_rows);
            return KKM_ERR_ARG;
        }
        const kkm_status st = check_kernel(p.kernel_type, p.gamma, p.coef0, p.degree);
        if (st != KKM_OK) {
            char why[256];
            snprintf(why, sizeof(why), "%s", kkm_last_error());
            set_error("kkm_fit_batched: problem %d: %s", b, why);
            return st;
        }
    }
    return KKM_OK;
}

// Lays the workspace out (sizes only when base == nullptr) and, with a base,
// fills the host tables whose pointers refer to it.
void make_plan(const kkm_instance *inst, int32_t count, int32_t gram_prec, int32_t k_store,
               int32_t empty_policy, void *base, Plan &p) {
    p.count = count;
    Carver c(base);
    const size_t es = elem_bytes(k_store);
    const int64_t eb = (gram_prec == KKM_BF16) ? 2 : 1;
    std::vector<int64_t> row_off(count + 1, 0);
    for (int32_t b = 0; b < count; ++b) row_off[b + 1] = row_off[b] + inst[b].n;
    p.total_n = row_off[count];

    std::vector<void *> K(count);
    std::vector<unsigned char *> Xq(count, nullptr);
    std::vector<std::pair<InstGeom, size_t>> geo(count);
    for (int32_t b = 0; b < count; ++b) {
        const int64_t n = inst[b].n, ldk = (n + 63) & ~int64_t(63);
        K[b] = c.take<char>((size_t)n * (size_t)ldk * es);
    }
    for (int32_t b = 0; b < count && gram_prec != KKM_F32; ++b)
        Xq[b] = c.take<unsigned char>((size_t)inst[b].n *
                                      (size_t)padded_d(inst[b].d, gram_prec) * (size_t)eb);
    std::vector<void *> iws(count);
    for (int32_t b = 0; b < count; ++b) {
        geo[b].first = inst_geometry(inst[b].n, inst[b].k, inst[b].chunk_rows);
        geo[b].second = inst_workspace_bytes(geo[b].first);
        iws[b] = c.take<char>(geo[b].second);
    }
    p.diag = c.take<float>((size_t)p.total_n);
    float *nrm = c.take<float>((size_t)p.total_n);
    float *scale = c.take<float>((size_t)p.total_n);
    p.lab[0] = c.take<int32_t>((size_t)p.total_n);
    p.lab[1] = c.take<int32_t>((size_t)p.total_n);
    int64_t total_k = 0;
    for (int32_t b = 0; b < count; ++b) total_k += inst[b].k;
    int32_t *counts_out = c.take<int32_t>((size_t)total_k);
    p.n_changed = c.take<int64_t>((size_t)count);
    p.J = c.take<double>((size_t)count);
    p.objective = c.take<double>((size_t)count);
    p.status = c.take<int32_t>((size_t)count);
    p.iters = c.take<int32_t>((size_t)count);
    p.full = c.take<Inst>((size_t)count);
    p.live = c.take<Inst>((size_t)count);
    p.gtab = c.take<GramSrc>((size_t)count);
    p.rtab = c.take<RowSrc>((size_t)count);
    p.blk_start = c.take<int64_t>((size_t)count + 1);
    p.cl_start = c.take<int64_t>((size_t)count + 1);
    p.item_start = c.take<int64_t>((size_t)count + 1);
    p.tile_start = c.take<int64_t>((size_t)count + 1);
    p.row_start = c.take<int64_t>((size_t)count + 1);
    p.step = c.take<int32_t>(1);
    p.n_live = c.take<int32_t>(1);
    p.flag = c.take<int32_t>(1);
    p.queue = c.take<unsigned long long>(1);
    p.bytes = c.bytes();

    p.total_blocks = p.total_clusters = p.total_items = 0;
    p.max_k = 0;
    for (int32_t b = 0; b < count; ++b) {
        p.total_blocks += geo[b].first.nblk;
        p.total_items += inst_sweep_items(geo[b].first, k_store);
        p.total_clusters += inst[b].k;
        p.max_k = std::max(p.max_k, inst[b].k);
    }
    // the costliest tiles first: a tile's cost grows with d; ties by n
    std::vector<int32_t> order(count);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        if (inst[a].d != inst[b].d) return inst[a].d > inst[b].d;
        return inst[a].n > inst[b].n;
    });
    p.h_tile_start.assign(count + 1, 0);
    for (int32_t r = 0; r < count; ++r) {
        const int64_t nb = (inst[order[r]].n + GM - 1) / GM;
        p.h_tile_start[r + 1] = p.h_tile_start[r] + nb * (nb + 1) / 2;
    }
    p.total_tiles = p.h_tile_start[count];
    if (!base) return;

    p.h_full.assign(count, Inst{});
    p.h_rtab.assign(count, RowSrc{});
    p.h_gtab.assign(count, GramSrc{});
    p.h_row_start = row_off;
    int64_t koff = 0;
    for (int32_t b = 0; b < count; ++b) {
        const kkm_instance &q = inst[b];
        const int64_t ldk = (q.n + 63) & ~int64_t(63);
        Inst &in = p.h_full[b];
        inst_carve(iws[b], geo[b].first, &in, nullptr);
        in.empty_policy = empty_policy;
        in.K = K[b];
        in.ldk = ldk;
        in.diag = p.diag + row_off[b];
        in.lab_off = row_off[b];
        in.counts_out = counts_out + koff;
        in.n_changed = p.n_changed + b;
        in.J_in = p.J + b;
        in.D_out = nullptr;
        in.ctilde_out = nullptr;
        inst_set_store(&in, k_store);
        koff += q.k;

        RowSrc &r = p.h_rtab[b];
        r.X = q.X;
        r.ldx = q.ldx;
        r.d = q.d;
        r.dpad = (gram_prec == KKM_F32) ? q.d : padded_d(q.d, gram_prec);
        r.Xq = Xq[b];
        r.nrm = nrm + row_off[b];
        r.scale = scale + row_off[b];
    }
    for (int32_t rnk = 0; rnk < count; ++rnk) {
        const int32_t b = order[rnk];
        const kkm_instance &q = inst[b];
        const Inst &in = p.h_full[b];
        Epi e;
        e.n = q.n;
        e.ldk = in.ldk;
        e.kernel = q.kernel_type;
        e.gamma = epi_gamma(q.kernel_type, q.gamma);
        e.coef0 = (float)q.coef0;
        e.degree = q.degree;
        e.nrm = p.h_rtab[b].nrm;
        e.scale = (gram_prec == KKM_FP8_ROWSCALED) ? p.h_rtab[b].scale : nullptr;
        e.K = K[b];
        e.diag = p.diag + row_off[b];
        e.vec_k = 1;  // ldk is a multiple of 64 and each K starts 256-byte aligned
        e.plgw = 0;
        e.pns = 0;
        GramSrc &g = p.h_gtab[rnk];
        g.f.X = q.X;
        g.f.d = q.d;
        g.f.ldx = q.ldx;
        g.f.vec_x = ((q.ldx % 4) == 0) && ((reinterpret_cast<uintptr_t>(q.X) & 15) == 0);
        g.f.e = e;
        g.q.Xq = Xq[b];
        g.q.ldq_bytes = p.h_rtab[b].dpad * eb;
        g.q.nslab = g.q.ldq_bytes / SLAB;
        g.q.e = e;
    }
}

// Device buffers owned by one kkm_fit_batched call.
struct BatchBuffers {
    hipStream_t stream = nullptr;  // the caller's: drained before anything is freed
    void *ws_own = nullptr;
    int32_t *host = nullptr;
    hipStream_t cap = nullptr;
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    hipEvent_t ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    ~BatchBuffers() {
        (void)hipStreamSynchronize(stream);
        for (auto &x : exec)
            if (x) (void)hipGraphExecDestroy(x);
        for (auto &g : graph)
            if (g) (void)hipGraphDestroy(g);
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
        if (cap) (void)hipStreamDestroy(cap);
        if (host) (void)hipHostFree(host);
        if (ws_own) (void)hipFree(ws_own);
    }
};

kkm_status launch_prologue(const Plan &p, int32_t gram_prec, hipStream_t s) {
    const dim3 g((unsigned)((p.total_n + 3) / 4)), b(256);
    if (gram_prec == KKM_F32)
        hipLaunchKernelGGL(batch_prologue<KKM_F32>, g, b, 0, s, p.rtab, p.row_start, p.count);
    else if (gram_prec == KKM_BF16)
        hipLaunchKernelGGL(batch_prologue<KKM_BF16>, g, b, 0, s, p.rtab, p.row_start, p.count);
    else
        hipLaunchKernelGGL(batch_prologue<KKM_FP8_ROWSCALED>, g, b, 0, s, p.rtab, p.row_start,
                           p.count);
    KKM_HIP(hipGetLastError());
    return KKM_OK;
}

kkm_status launch_gram(const Plan &p, int32_t gram_prec, int32_t k_store, int cus,
                       hipStream_t s) {
    hipLaunchKernelGGL(fill_u64, dim3(1), dim3(1), 0, s, p.queue, 0ull);
    KKM_HIP(hipGetLastError());
    const int64_t want = (p.total_tiles + kQueueChunk - 1) / kQueueChunk;
    const dim3 g((unsigned)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)cus * 2)));
    const dim3 b(GTHREADS);
    const TimedSpan span = timing_begin(TK_GRAM, s);
    if (gram_prec == KKM_F32 && k_store == KKM_F32)
        hipLaunchKernelGGL((batch_gram<KKM_F32, float>), g, b, 0, s, p.gtab, p.tile_start, p.count, p.queue);
    else if (gram_prec == KKM_F32)
        hipLaunchKernelGGL((batch_gram<KKM_F32, uint16_t>), g, b, 0, s, p.gtab, p.tile_start, p.count, p.queue);
    else if (gram_prec == KKM_BF16 && k_store == KKM_F32)
        hipLaunchKernelGGL((batch_gram<KKM_BF16, float>), g, b, 0, s, p.gtab, p.tile_start, p.count, p.queue);
    else if (gram_prec == KKM_BF16)
        hipLaunchKernelGGL((batch_gram<KKM_BF16, uint16_t>), g, b, 0, s, p.gtab, p.tile_start, p.count, p.queue);
    else if (k_store == KKM_F32)
        hipLaunchKernelGGL((batch_gram<KKM_FP8_ROWSCALED, float>), g, b, 0, s, p.gtab, p.tile_start, p.count, p.queue);
    else
        hipLaunchKernelGGL((batch_gram<KKM_FP8_ROWSCALED, uint16_t>), g, b, 0, s, p.gtab, p.tile_start, p.count, p.queue);
    KKM_HIP(hipGetLastError());
    timing_end(span, s);
    return KKM_OK;
}

kkm_status launch_control(const Ctl &c, int32_t mode, hipStream_t s) {
    hipLaunchKernelGGL(batch_control, dim3(1), dim3(kCtlThreads), 0, s, c, mode);
    KKM_HIP(hipGetLastError());
    return KKM_OK;
}

}  // namespace

}  // namespace kkm

using namespace kkm;

extern "C" size_t kkm_fit_batched_workspace_bytes(const kkm_instance *inst, int32_t count,
                                                  int32_t gram_prec, int32_t k_store) {
    if (check_instances(inst, count, gram_prec, k_store) != KKM_OK) return 0;
    Plan p;
    make_plan(inst, count, gram_prec, k_store, KKM_EMPTY_INF, nullptr, p);
    return p.bytes;
}

extern "C" kkm_status kkm_fit_batched(const kkm_instance *inst, int32_t count, int32_t gram_prec,
                                      int32_t k_store, int32_t empty_policy,
                                      const int32_t *labels0, int32_t max_iter,
                                      int32_t check_convergence, int32_t use_graph,
                                      int32_t *labels_out, double *objective, int32_t *iters,
                                      double *times_ms, void *ws, size_t ws_bytes, void *stream) {
    KKM_TRY(check_instances(inst, count, gram_prec, k_store));
    if (!labels0 || !labels_out || !objective || !iters || max_iter < 0) {
        set_error("kkm_fit_batched: NULL label/result pointer or max_iter < 0");
        return KKM_ERR_ARG;
    }
    if (empty_policy != KKM_EMPTY_INF && empty_policy != KKM_EMPTY_ZERO_CENTROID) {
        set_error("kkm_fit_batched: unknown empty-cluster policy %d", empty_policy);
        return KKM_ERR_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    Plan p;
    make_plan(inst, count, gram_prec, k_store, empty_policy, nullptr, p);
    if ((p.total_n + 255) / 4 > 0x7fffffffLL || p.total_blocks > 0x7fffffffLL ||
        p.total_clusters > 0x7fffffffLL || p.total_items > 0x7fffffffLL) {
        set_error("kkm_fit_batched: the batch is too large for one grid");
        return KKM_ERR_UNSUPPORTED;
    }
    BatchBuffers bb;
    bb.stream = s;
    if (ws) {
        if (ws_bytes < p.bytes) {
            set_error("kkm_fit_batched: workspace of %zu bytes is smaller than %zu", ws_bytes,
                      p.bytes);
            return KKM_ERR_NOMEM;
        }
    } else {
        const hipError_t e = hipMalloc(&bb.ws_own, p.bytes);
        if (e != hipSuccess) {
            set_error("kkm_fit_batched: cannot allocate %zu bytes (%s)", p.bytes,
                      hipGetErrorString(e));
            return KKM_ERR_NOMEM;
        }
        ws = bb.ws_own;
    }
    make_plan(inst, count, gram_prec, k_store, empty_policy, ws, p);

    int dev = 0, cus = 0;
    KKM_HIP(hipGetDevice(&dev));
    KKM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int64_t sweep_grid = p.total_items;

    // tables (pageable host memory: wait for the copies before it goes away)
    KKM_HIP(hipMemcpyAsync(p.full, p.h_full.data(), sizeof(Inst) * count, hipMemcpyHostToDevice, s));
    KKM_HIP(hipMemcpyAsync(p.gtab, p.h_gtab.data(), sizeof(GramSrc) * count, hipMemcpyHostToDevice, s));
    KKM_HIP(hipMemcpyAsync(p.rtab, p.h_rtab.data(), sizeof(RowSrc) * count, hipMemcpyHostToDevice, s));
    KKM_HIP(hipMemcpyAsync(p.tile_start, p.h_tile_start.data(), sizeof(int64_t) * (count + 1),
                           hipMemcpyHostToDevice, s));
    KKM_HIP(hipMemcpyAsync(p.row_start, p.h_row_start.data(), sizeof(int64_t) * (count + 1),
                           hipMemcpyHostToDevice, s));
    KKM_HIP(hipStreamSynchronize(s));
    KKM_HIP(hipHostMalloc((void **)&bb.host, sizeof(int32_t) * 4, hipHostMallocDefault));
    for (auto &e : bb.ev) KKM_HIP(hipEventCreate(&e));

    // 1-2. prologue and Gram
    KKM_HIP(hipEventRecord(bb.ev[0], s));
    KKM_TRY(launch_prologue(p, gram_prec, s));
    KKM_TRY(launch_gram(p, gram_prec, k_store, cus, s));
    flag_nonfinite(p.diag, p.total_n, p.flag, s);
    KKM_HIP(hipGetLastError());
    KKM_HIP(hipEventRecord(bb.ev[1], s));
    KKM_HIP(hipMemcpyAsync(bb.host, p.flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    KKM_HIP(hipStreamSynchronize(s));
    if (bb.host[0] != 0) {
        set_error("kkm_fit_batched: diag(K) has a non-finite entry (NaN or infinity in X?)");
        return KKM_ERR_NONFINITE;
    }

    // 3. loop
    Ctl c;
    c.full = p.full;
    c.live = p.live;
    c.blk_start = p.blk_start;
    c.cl_start = p.cl_start;
    c.item_start = p.item_start;
    c.status = p.status;
    c.iters = p.iters;
    c.objective = p.objective;
    c.n_changed = p.n_changed;
    c.J = p.J;
    c.step = p.step;
    c.n_live = p.n_live;
    c.count = count;
    c.max_iter = max_iter;
    c.check_convergence = check_convergence;
    InstSet set{};
    set.table = p.live;
    set.blk_start = p.blk_start;
    set.cl_start = p.cl_start;
    set.item_start = p.item_start;
    set.count = count;

    KKM_HIP(hipMemcpyAsync(p.lab[0], labels0, sizeof(int32_t) * (size_t)p.total_n,
                           hipMemcpyDeviceToDevice, s));
    fill_i32(p.step, 1, 0, s);
    KKM_TRY(launch_control(c, CTL_INIT, s));

    auto one_step = [&](int par, hipStream_t st) -> kkm_status {
        KKM_TRY(step_launch(set, p.total_blocks, p.total_clusters, sweep_grid, p.max_k, k_store,
                            true, p.lab[par], p.lab[par ^ 1], st));
        return launch_control(c, CTL_AFTER_STEP, st);
    };
    if (use_graph && max_iter > 0) {
        KKM_HIP(hipStreamCreateWithFlags(&bb.cap, hipStreamNonBlocking));
        for (int par = 0; par < 2; ++par) {
            KKM_HIP(hipStreamBeginCapture(bb.cap, hipStreamCaptureModeThreadLocal));
            const kkm_status st = one_step(par, bb.cap);
            hipGraph_t g = nullptr;
            const hipError_t e = hipStreamEndCapture(bb.cap, &g);
            bb.graph[par] = g;
            if (st != KKM_OK) return st;
            KKM_HIP(e);
            KKM_HIP(hipGraphInstantiate(&bb.exec[par], g, nullptr, nullptr, 0));
        }
    }
    // launch step t, then look at the live count after step t-1: one step of
    // look-ahead keeps the queue full (a step over no live problem does nothing)
    int32_t T = 0;
    for (int32_t t = 0; t < max_iter; ++t) {
        if (bb.exec[0]) {
            KKM_HIP(hipGraphLaunch(bb.exec[t & 1], s));
        } else {
            KKM_TRY(one_step(t & 1, s));
        }
        T = t + 1;
        KKM_HIP(hipMemcpyAsync(bb.host + (t & 1), p.n_live, sizeof(int32_t),
                               hipMemcpyDeviceToHost, s));
        KKM_HIP(hipEventRecord(bb.ev[4 + (t & 1)], s));
        if (t >= 1) {
            KKM_HIP(hipEventSynchronize(bb.ev[4 + ((t - 1) & 1)]));
            if (bb.host[(t - 1) & 1] == 0) break;
        }
    }
    KKM_HIP(hipEventRecord(bb.ev[2], s));

    // 4. final objective of the problems that stopped at max_iter (their
    // labels are in buffer T & 1; a retired problem holds its final labels in
    // both buffers, since its last step changed nothing)
    KKM_TRY(launch_control(c, CTL_SELECT_FINAL, s));
    KKM_TRY(step_launch(set, p.total_blocks, p.total_clusters, sweep_grid, p.max_k, k_store, true,
                        p.lab[T & 1], p.lab[(T & 1) ^ 1], s));
    KKM_TRY(launch_control(c, CTL_AFTER_FINAL, s));
    KKM_HIP(hipEventRecord(bb.ev[3], s));
    KKM_HIP(hipMemcpyAsync(labels_out, p.lab[T & 1], sizeof(int32_t) * (size_t)p.total_n,
                           hipMemcpyDeviceToDevice, s));

    std::vector<int32_t> hstat(count), hit(count);
    KKM_HIP(hipMemcpyAsync(hstat.data(), p.status, sizeof(int32_t) * count, hipMemcpyDeviceToHost, s));
    KKM_HIP(hipMemcpyAsync(hit.data(), p.iters, sizeof(int32_t) * count, hipMemcpyDeviceToHost, s));
    KKM_HIP(hipMemcpyAsync(objective, p.objective, sizeof(double) * count, hipMemcpyDeviceToHost, s));
    KKM_HIP(hipStreamSynchronize(s));
    for (int32_t b = 0; b < count; ++b) {
        if (hstat[b] == ST_BADLABEL) {
            set_error("kkm_fit_batched: labels0 of problem %d holds a label outside [0, %d)", b,
                      inst[b].k);
            return KKM_ERR_LABEL;
        }
        if (hstat[b] != ST_CONVERGED && hstat[b] != ST_DONE) {
            set_error("kkm_fit_batched: problem %d ended in state %d", b, hstat[b]);
            return KKM_ERR_HIP;
        }
        iters[b] = hit[b];
    }
    if (times_ms) {
        float a = 0.f, b2 = 0.f, c3 = 0.f;
        (void)hipEventElapsedTime(&a, bb.ev[0], bb.ev[1]);
        (void)hipEventElapsedTime(&b2, bb.ev[1], bb.ev[2]);
        (void)hipEventElapsedTime(&c3, bb.ev[2], bb.ev[3]);
        times_ms[0] = a;
        times_ms[1] = b2;
        times_ms[2] = c3;
    }
    return KKM_OK;
}
