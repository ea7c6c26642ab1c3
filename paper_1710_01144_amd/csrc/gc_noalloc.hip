// Allocation-free marginal gains (gc_marginal_gains_noalloc): the device
// scratch of the gain path lives in one file-scope device array instead of a
// caller workspace, for callers that cannot allocate device memory.
//
// The array's name is a host-side stand-in in host code: its device address
// is looked up once per device (hipGetSymbolAddress, with that device
// current) and only that address is handed to the kernels and fills.
#include <hip/hip_runtime.h>

#include <mutex>

#include "gc.h"
#include "gc_internal.h"

namespace {

constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[GC_NOALLOC_SCRATCH_BYTES];

std::mutex g_mu;
void *g_scratch[kMaxDevices];  // device address of `scratch` per device, null until looked up

// Device address of the current device's copy of `scratch`.
int scratch_address(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return gck::set_error(GC_EDEVICE, "hipGetDevice failed");
    if (dev < 0 || dev >= kMaxDevices) return gck::set_error(GC_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return gck::set_error(GC_EDEVICE, "hipGetSymbolAddress of the scratch array failed");
        }
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return GC_OK;
}

}  // namespace

extern "C" int gc_marginal_gains_noalloc(const gc_graph *g, const void *d_dist, int32_t dist_bytes,
                                         const int32_t *d_cand, int32_t count, int64_t *d_gain,
                                         int64_t *d_edges, int32_t *d_visited, hipStream_t stream) {
    if (!g) return gck::set_error(GC_EINVAL, "graph is NULL");
    void *p = nullptr;
    int rc = scratch_address(&p);
    if (rc) return rc;
    return gck::gains_in_buffer(g, d_dist, dist_bytes, d_cand, count, d_gain, d_edges, d_visited, p,
                                (size_t)GC_NOALLOC_SCRATCH_BYTES, stream);
}
