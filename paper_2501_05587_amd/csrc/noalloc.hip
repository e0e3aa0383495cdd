// kkm_iterate without a workspace argument, for callers that cannot allocate
// device memory (code under stream capture, tight serving loops): the step's
// scratch (V in CSR form, per-block histograms, segment partials, objective
// partials) lives in one file-scope device array of fixed size, and the call
// itself allocates nothing.
//
// Each GPU the library runs on holds its own copy of the array from the first
// call on that device until the process ends.  The array's device address is
// looked up once per device (hipGetSymbolAddress, with that device current)
// and only that address is ever handed to kernels: in host code the array's
// name is a host-side stand-in, not a device pointer.
//
// Every call on one GPU shares that GPU's array, which keeps the contents of
// the last call.  Nothing in it has to start at zero: every step kernel writes
// what a later kernel of the same step reads.  Calls that overlap on one GPU
// (two streams, two host threads) race on the array and must be serialised by
// the caller.
#include <mutex>

#include "kkm_common.h"

namespace kkm {
namespace {

static __device__ __align__(256) unsigned char scratch[KKM_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on `dev` (the current device).
kkm_status scratch_address(int dev, void **out) {
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("kkm_iterate_noalloc: device %d outside the supported range [0, %d)", dev,
                  kMaxDevices);
        return KKM_ERR_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        KKM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) {
            set_error("kkm_iterate_noalloc: no device address for the scratch array on device %d",
                      dev);
            return KKM_ERR_HIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return KKM_OK;
}

}  // namespace
}  // namespace kkm

using namespace kkm;

extern "C" size_t kkm_iterate_noalloc_max_bytes(void) { return KKM_NOALLOC_SCRATCH_BYTES; }

extern "C" kkm_status kkm_iterate_noalloc(const void *K, int32_t k_store, int64_t ldk,
                                          const float *diagK, int64_t n, int32_t k,
                                          const int32_t *labels_in, int32_t empty_policy,
                                          int32_t *labels_out, int32_t *counts_out,
                                          int64_t *n_changed, double *J_in, float *D_out,
                                          float *ctilde_out, void *stream) {
    if (n < 1 || k < 1) {
        set_error("kkm_iterate_noalloc: bad sizes (n=%lld k=%d)", (long long)n, k);
        return KKM_ERR_ARG;
    }
    const size_t need = kkm_iterate_workspace_bytes(n, k);
    if (need > KKM_NOALLOC_SCRATCH_BYTES) {
        set_error("kkm_iterate_noalloc: n=%lld, k=%d needs %zu bytes of scratch, more than the "
                  "%zu the library holds per device; use kkm_iterate with a workspace",
                  (long long)n, k, need, (size_t)KKM_NOALLOC_SCRATCH_BYTES);
        return KKM_ERR_UNSUPPORTED;
    }
    int dev = -1;
    KKM_HIP(hipGetDevice(&dev));
    if (stream) {
        const int sdev = hipGetStreamDeviceId((hipStream_t)stream);
        if (sdev != dev) {
            set_error("kkm_iterate_noalloc: the stream belongs to device %d but device %d is "
                      "current", sdev, dev);
            return KKM_ERR_ARG;
        }
    }
    void *ptr = nullptr;
    KKM_TRY(scratch_address(dev, &ptr));
    return kkm_iterate(K, k_store, ldk, diagK, n, k, labels_in, empty_policy, labels_out,
                       counts_out, n_changed, J_in, D_out, ctilde_out, ptr,
                       (size_t)KKM_NOALLOC_SCRATCH_BYTES, stream);
}
