// cc_count_noalloc: the plain count (cc_count) over a workspace that the library holds in a
// file-scope device array, for callers that cannot allocate device memory.
//
// The array is one per GPU the library runs on (each device holds its own copy, at its own
// address, until the process ends). Its device address is looked up once per device, on the first
// call there, with that device current; host code passes that address to the kernels, never the
// array's name (which is a host-side stand-in). Every call on one GPU shares the array: the count
// writes every byte it reads before reading it (tables, chunk partials, root counts, reduction
// scratch, neighbour colours, projected rows), so nothing has to be cleared between calls, but two
// calls that overlap on one GPU (different streams, or threads) race on it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "cc_host.h"
#include "cc_internal.h"

namespace {

static __device__ __align__(256) uint8_t scratch[CC_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on the current device (looked up on the first call there)
cc_status scratch_for_current_device(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return cc::host::hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return cc::host::fail(CC_EDEVICE, "device ordinal beyond the library's table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return cc::host::hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return cc::host::fail(CC_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return CC_OK;
}

}  // namespace

extern "C" {

cc_status cc_count_noalloc(const cc_plan* P, const cc_graph* G, const uint8_t* colours_dev, int32_t B,
                           double* X_dev, double* vertex_dev, void* stream) {
    if (!P || !G) return cc::host::fail(CC_EINVAL, "NULL plan or graph");
    if (P->profiling) return cc::host::fail(CC_EINVAL, "profiling creates events: disable it for cc_count_noalloc");
    size_t need = 0;
    cc_status st = cc_count_workspace_bytes(P, G, &need);
    if (st != CC_OK) return st;
    if (need > (size_t)CC_NOALLOC_SCRATCH_BYTES)
        return cc::host::fail(CC_ENOSPC, "this count needs " + std::to_string(need) +
                                             " bytes of workspace, more than the library's fixed " +
                                             std::to_string((size_t)CC_NOALLOC_SCRATCH_BYTES) +
                                             " bytes (use cc_count with a caller workspace)");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return cc::host::hip_fail(e, "hipGetDevice");
    if (dev != G->device) return cc::host::fail(CC_EINVAL, "the graph lives on another device than the current one");
    void* ws = nullptr;
    st = scratch_for_current_device(&ws);
    if (st != CC_OK) return st;
    return cc_count(P, G, colours_dev, B, ws, (size_t)CC_NOALLOC_SCRATCH_BYTES, X_dev, vertex_dev, stream);
}

}  // extern "C"
