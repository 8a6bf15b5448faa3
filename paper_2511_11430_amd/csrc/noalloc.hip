// Device memory of the no-allocation entry point (vpm_eval_velocity_stretching_noalloc): the
// source-split partial sums of small target sets live in this file-scope array instead of a
// caller workspace.  Each GPU holds its own copy for the life of the process.  In host code
// the name is only a handle, so its device address is looked up once per device, with that
// device current, and kept; every use (kernel arguments) goes through that address.
#include <hip/hip_runtime.h>

#include <mutex>

#include "vpm_internal.h"

namespace vpm {

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

hipError_t noalloc_scratch(void** ptr) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

}  // namespace vpm
