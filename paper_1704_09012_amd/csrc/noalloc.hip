// Scratch memory for callers that cannot allocate: a file-scope device array that every
// GPU holds one copy of, for the life of the process.  In host code the array's name is
// only a stand-in, so its device address is looked up here with hipGetSymbolAddress, once
// per device, and that address is what the kernels are given.
#include "noalloc.h"

#include <mutex>

// S [kStaticSketchRows] of the sketch, then 64 words of flags (the error flags first).
static __device__ __align__(256) long long scratch[rl0::kStaticSketchRows + 64];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
long long* g_scratch[kMaxDevices] = {};

}  // namespace

namespace rl0 {

hipError_t static_scratch(long long** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch[dev] = static_cast<long long*>(p);
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

}  // namespace rl0
