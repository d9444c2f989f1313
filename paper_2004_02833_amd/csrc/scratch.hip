// The library's static device scratch (pm_check_noalloc), in a translation
// unit of its own, so that the code object of the sweep kernels holds no
// device variable (a profiler's counter mode failed to load the library
// while the array sat beside them).
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace pm {

// ---------------------------------------------------- static scratch memory --
// Partial results of pm_check_noalloc: kScratchPartials maxima (double) and
// as many counts (unsigned long long).  Each GPU the library runs on holds
// its own copy until the process ends.  Host code never uses the array's
// name as an address: scratch_device() takes the device address from
// hipGetSymbolAddress once per device and keeps it.
constexpr int kScratchPartials = 1024;
static __device__ __align__(256) unsigned char scratch[kScratchPartials * (sizeof(double) + sizeof(unsigned long long))];

constexpr int kMaxDevices = 64;

hipError_t scratch_device(void** ptr) {
    static void* addr[kMaxDevices] = {nullptr};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

int scratch_partials() { return kScratchPartials; }

}  // namespace pm
