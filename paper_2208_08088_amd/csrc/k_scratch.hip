// The library's static device scratch: the partial sums of split-k plans
// for callers that cannot allocate (tsmm_execute_noalloc).  One array per
// device, in the code object's data, alive until the process ends; every
// call on a device shares it.
#include <map>
#include <mutex>

#include "tsmm_internal.h"

namespace {
// Device memory of the split-k partial sums (op T pass 1, k-slab parts):
// 32 MiB, P * m * n binary64 values with P * m * n <= 2^22 (e.g. P = 1024
// slices of a 64 x 64 output).
__device__ __align__(256) unsigned char scratch[tsmm::kScratchBytes];
}  // namespace

namespace tsmm {

// Device address of `scratch` on device `device`, looked up once per device
// with that device current (the array's name is a host-side stand-in, not a
// device address: only this pointer may reach a kernel or a copy).
hipError_t scratch_device_ptr(int device, void **out) {
    static std::mutex mu;
    static std::map<int, void *> ptrs;
    std::lock_guard<std::mutex> lock(mu);
    auto it = ptrs.find(device);
    if (it != ptrs.end()) {
        *out = it->second;
        return hipSuccess;
    }
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) {
        const hipError_t e2 = hipSetDevice(cur);
        if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    ptrs.emplace(device, p);
    *out = p;
    return hipSuccess;
}

}  // namespace tsmm
