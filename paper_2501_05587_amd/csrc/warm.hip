// The learned warm start as one call: F = phi_theta(X), then `restarts`
// independent k-means++ seedings (the D^2 sampling the paper's Sec. 2.1 names
// for K-means), each followed by Lloyd's iterations with explicit centroids on
// the rows of F, and the labelling with the lowest feature-space objective.
// It replaces the random initial labels of Sec. 3.4; kkm_fit_ex then refines
// it with the exact method.
//
// The restarts run concurrently on internal streams of default priority, one
// host thread per stream (each restart's calls are synchronous on its own
// stream).  Each restart computes exactly what it computes alone, so the result
// does not depend on the number of streams.
#include <string>
#include <thread>
#include <vector>

#include "kkm_common.h"

namespace kkm {
namespace {

struct WarmGeom {
    size_t fwd, kpp, lloyd;
};

WarmGeom warm_geom(int64_t n, int64_t d, int64_t h1, int64_t h2, int64_t out, int32_t k) {
    WarmGeom g;
    g.fwd = kkm_mlp_forward_workspace_bytes(n, d, h1, h2, out);
    g.kpp = kkm_feature_kmeanspp_workspace_bytes(n, out, k);
    g.lloyd = kkm_feature_lloyd_workspace_bytes(n, out, k);
    return g;
}

// Buffers of one stream's worker: its seeding and Lloyd workspaces, the seeds,
// the seeded labels and two candidate labellings (the best so far and the
// current restart's).
struct Lane {
    void *kpp_ws, *lloyd_ws;
    int32_t *seeds, *seeded, *cand[2];
};

size_t carve_warm(void *base, int64_t n, int32_t k, int64_t out, const WarmGeom &g,
                  int32_t streams, float **F, void **fwd_ws, std::vector<Lane> *lanes) {
    Carver c(base);
    float *f = c.take<float>((size_t)n * (size_t)out);
    void *fw = c.take<char>(g.fwd);
    if (F) *F = f;
    if (fwd_ws) *fwd_ws = fw;
    for (int32_t t = 0; t < streams; ++t) {
        Lane l;
        l.kpp_ws = c.take<char>(g.kpp);
        l.lloyd_ws = c.take<char>(g.lloyd);
        l.seeds = c.take<int32_t>((size_t)k);
        l.seeded = c.take<int32_t>((size_t)n);
        l.cand[0] = c.take<int32_t>((size_t)n);
        l.cand[1] = c.take<int32_t>((size_t)n);
        if (lanes) lanes->push_back(l);
    }
    return c.bytes();
}

// Lower feature-space objective first, then the lower restart index; a NaN
// objective (no Lloyd step ran) ranks after every number.
bool better(double a, int32_t ra, double b, int32_t rb) {
    const bool an = a != a, bn = b != b;
    if (an != bn) return bn;
    if (!an && a != b) return a < b;
    return ra < rb;
}

}  // namespace
}  // namespace kkm

using namespace kkm;

extern "C" size_t kkm_warm_start_workspace_bytes(int64_t n, int64_t d, int64_t h1, int64_t h2,
                                                 int64_t out, int32_t k, int32_t streams) {
    if (n < 1 || d < 1 || h1 < 1 || h2 < 1 || out < 1 || k < 1 || streams < 1) return 0;
    const WarmGeom g = warm_geom(n, d, h1, h2, out, k);
    if (!g.fwd || !g.kpp || !g.lloyd) return 0;
    return carve_warm(nullptr, n, k, out, g, streams, nullptr, nullptr, nullptr);
}

extern "C" kkm_status kkm_warm_start(const float *params, int64_t d, int64_t h1, int64_t h2,
                                     int64_t out, const float *X, int64_t n, int64_t ldx,
                                     int32_t k, int32_t restarts, const double *uniforms,
                                     int32_t max_iter, int32_t streams, int32_t *labels_out,
                                     double *objective, int32_t *cheap_iters,
                                     int32_t *best_restart, void *ws, size_t ws_bytes,
                                     void *stream) {
    if (n < 1 || d < 1 || h1 < 1 || h2 < 1 || out < 1 || ldx < d || k < 1 || k > n ||
        restarts < 1 || max_iter < 0 || streams < 1 || !params || !X || !uniforms ||
        !labels_out) {
        set_error("kkm_warm_start: bad sizes or NULL pointer (n=%lld d=%lld k=%d restarts=%d "
                  "streams=%d)", (long long)n, (long long)d, k, restarts, streams);
        return KKM_ERR_ARG;
    }
    if (k > KKM_MAX_K) {
        set_error("kkm_warm_start: k=%d exceeds KKM_MAX_K=%d", k, KKM_MAX_K);
        return KKM_ERR_UNSUPPORTED;
    }
    for (int64_t t = 0; t < (int64_t)restarts * k; ++t)
        if (!(uniforms[t] >= 0.0 && uniforms[t] < 1.0)) {
            set_error("kkm_warm_start: uniforms must lie in [0, 1)");
            return KKM_ERR_ARG;
        }
    if (streams > restarts) streams = restarts;
    const WarmGeom g = warm_geom(n, d, h1, h2, out, k);
    const size_t need = carve_warm(nullptr, n, k, out, g, streams, nullptr, nullptr, nullptr);
    if (!ws || ws_bytes < need) {
        set_error("kkm_warm_start: workspace of %zu bytes is smaller than %zu", ws_bytes, need);
        return KKM_ERR_NOMEM;
    }
    float *F = nullptr;
    void *fwd_ws = nullptr;
    std::vector<Lane> lanes;
    carve_warm(ws, n, k, out, g, streams, &F, &fwd_ws, &lanes);
    hipStream_t s = (hipStream_t)stream;
    KKM_TRY(kkm_mlp_forward(params, d, h1, h2, out, X, n, ldx, F, out, fwd_ws, g.fwd, stream));

    // internal streams start after the features exist
    hipEvent_t ready = nullptr;
    KKM_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
    std::vector<hipStream_t> st((size_t)streams, nullptr);
    struct Guard {
        hipEvent_t *ev;
        std::vector<hipStream_t> *st;
        ~Guard() {
            for (hipStream_t x : *st)
                if (x) {
                    (void)hipStreamSynchronize(x);
                    (void)hipStreamDestroy(x);
                }
            if (*ev) (void)hipEventDestroy(*ev);
        }
    } guard{&ready, &st};
    KKM_HIP(hipEventRecord(ready, s));
    for (auto &x : st) {
        KKM_HIP(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
        KKM_HIP(hipStreamWaitEvent(x, ready, 0));
    }

    struct Result {
        kkm_status status = KKM_OK;
        std::string err;
        double obj = 0.0;
        int32_t best = -1, which = 0;
        int64_t iters = 0;
    };
    std::vector<Result> res((size_t)streams);
    auto worker = [&](int32_t t) {
        Result &r = res[(size_t)t];
        const Lane &l = lanes[(size_t)t];
        for (int32_t rs = t; rs < restarts; rs += streams) {
            kkm_status e = kkm_feature_kmeanspp(F, n, out, out, k, uniforms + (size_t)rs * k,
                                                l.seeds, l.seeded, l.kpp_ws, g.kpp, st[(size_t)t]);
            int32_t it = 0;
            double obj = 0.0;
            int32_t *dst = l.cand[r.which ^ 1];
            if (e == KKM_OK)
                e = kkm_feature_lloyd(F, n, out, out, k, l.seeded, max_iter, dst, &it, nullptr,
                                      &obj, l.lloyd_ws, g.lloyd, st[(size_t)t]);
            if (e != KKM_OK) {
                r.status = e;
                r.err = kkm_last_error();
                return;
            }
            r.iters += it;
            if (r.best < 0 || better(obj, rs, r.obj, r.best)) {
                r.obj = obj;
                r.best = rs;
                r.which ^= 1;  // dst now holds the best labelling
            }
        }
    };
    std::vector<std::thread> th;
    for (int32_t t = 1; t < streams; ++t) th.emplace_back(worker, t);
    worker(0);
    for (auto &x : th) x.join();
    int32_t win = -1;
    int64_t total = 0;
    for (int32_t t = 0; t < streams; ++t) {
        const Result &r = res[(size_t)t];
        if (r.status != KKM_OK) {
            set_error("kkm_warm_start: restart on stream %d: %s", t, r.err.c_str());
            return r.status;
        }
        total += r.iters;
        if (win < 0 || better(r.obj, r.best, res[(size_t)win].obj, res[(size_t)win].best)) win = t;
    }
    const Result &w = res[(size_t)win];
    // every restart has finished (the Lloyd calls synchronise their stream)
    KKM_HIP(hipMemcpyAsync(labels_out, lanes[(size_t)win].cand[w.which], (size_t)n * sizeof(int32_t),
                           hipMemcpyDeviceToDevice, s));
    KKM_HIP(hipStreamSynchronize(s));
    if (objective) *objective = w.obj;
    if (cheap_iters) *cheap_iters = (int32_t)total;
    if (best_restart) *best_restart = w.best;
    return KKM_OK;
}
