// Device scratch for callers that cannot allocate (code under HIP graph
// capture, serving loops, harnesses that forbid hipMalloc): one file-scope
// array per device, holding the EM workspace of ctis_em_iterate_static.
// Every call on a device shares that device's array (and keeps its last
// contents); calls that overlap on one device race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ctis_internal.h"

namespace ctis {
namespace {

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
void *g_ptr[kMaxDevices] = {};

}  // namespace

// Device address of the current device's scratch array (taken once per
// device with that device current; the array's name in host code is not a
// device address).
int static_scratch(void **ptr) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return (int)e;
    if (dev < 0 || dev >= kMaxDevices) return (int)hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return (int)e;
        g_ptr[dev] = p;
    }
    *ptr = g_ptr[dev];
    return 0;
}

}  // namespace ctis
