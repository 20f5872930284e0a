// sg_noalloc.hip -- sg_bind_noalloc: bind a handle to a workspace the library
// holds in a statically allocated device array, for callers that cannot
// allocate device memory themselves (code under HIP graph capture, tight
// serving loops, harnesses that forbid allocation).
//
// The array is a file-scope __device__ variable: every GPU the library runs
// on holds one copy of kNoAllocBytes until the process ends.  On the host its
// name is only a stand-in for the device symbol, so the entry point asks the
// runtime for the array's device address once per device (with that device
// current) and uses that address everywhere.  Every handle bound this way on
// one GPU shares the same bytes: binding another handle overwrites the first
// one's structure and state, and calls that overlap on one GPU race.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "sg.h"

sg_status sg_internal_fail(sg_status code, const char* msg);
sg_status sg_internal_bind(sg_handle h, void* dev_ptr, uint64_t bytes, void* hip_stream, bool may_alloc);

namespace {

constexpr uint64_t kNoAllocBytes = SG_NOALLOC_MAX_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) uint8_t scratch[kNoAllocBytes];

std::mutex g_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of the array (looked up once per device).
sg_status scratch_address(void** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        char msg[256];
        std::snprintf(msg, sizeof msg, "sg_bind_noalloc: hipGetDevice: %s", hipGetErrorString(e));
        return sg_internal_fail(SG_EDEVICE, msg);
    }
    if (dev < 0 || dev >= kMaxDevices) return sg_internal_fail(SG_EDEVICE, "sg_bind_noalloc: device index out of range");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            char msg[256];
            std::snprintf(msg, sizeof msg, "sg_bind_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
            return sg_internal_fail(SG_EDEVICE, msg);
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SG_OK;
}

}  // namespace

extern "C" sg_status sg_bind_noalloc(sg_handle h, void* hip_stream)
{
    if (!h) return sg_internal_fail(SG_EINVAL, "null handle");
    uint64_t need = 0;
    sg_status s = sg_workspace_bytes(h, &need);
    if (s != SG_OK) return s;
    if (need > kNoAllocBytes) {
        char msg[256];
        std::snprintf(msg, sizeof msg, "sg_bind_noalloc: the handle needs %llu bytes, the static workspace holds %llu",
                      (unsigned long long)need, (unsigned long long)kNoAllocBytes);
        return sg_internal_fail(SG_ENOMEM, msg);
    }
    void* p = nullptr;
    s = scratch_address(&p);
    if (s != SG_OK) return s;
    return sg_internal_bind(h, p, kNoAllocBytes, hip_stream, false);
}
