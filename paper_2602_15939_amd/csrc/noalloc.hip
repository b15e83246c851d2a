// noalloc.hip — the device scratch of the entry points that allocate nothing.
//
// Callers that cannot allocate device memory (code under HIP graph capture, tight serving
// loops, harnesses that forbid hipMalloc) use entry points whose scratch lives in one
// file-scope device array.  Each GPU holds its own copy of the array, at its own address, from
// the first use until the process ends.  Host code never passes the array's name to a kernel
// (on the host it names a stand-in, not device memory): the device address comes from
// hipGetSymbolAddress, taken once per device with that device current, and is kept per device.
//
// Every call on one GPU shares that GPU's array and finds the last call's contents there;
// calls that overlap on one GPU race.
#include <mutex>

#include "pic_internal.h"

static __device__ __align__(256) unsigned char scratch[pic::kStaticScratchBytes];

namespace pic {

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch(void** ptr, size_t* bytes)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    *bytes = kStaticScratchBytes;
    return hipSuccess;
}

}  // namespace pic
