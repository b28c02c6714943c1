// scratch.hip -- the fixed device scratch of vm3dgs_frame_noalloc.
//
// One file-scope array per GPU, loaded with the library's code object and
// held until the process ends.  Its name is a host-side stand-in in host
// code: the device address is looked up once per device, with that device
// current, and only that address is handed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "vm3dgs_impl.h"

namespace vm {

static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_addr[kMaxDevices] = {};
}  // namespace

// the current device's scratch address (looked up on the first call per device)
hipError_t noalloc_scratch(void** out) {
    *out = nullptr;
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_addr[dev] = p;
    }
    *out = g_addr[dev];
    return hipSuccess;
}

}  // namespace vm
