// mhar_noalloc.hip -- the static device scratch behind mhar_run_noalloc.
//
// One file-scope device array per GPU (the code object is loaded on every
// device the library runs on, and each device holds its own copy until the
// process ends).  Host code never passes the array's name to a kernel or a
// copy: the name is a host-side stand-in, not a device address.  The address
// of each device's copy comes from hipGetSymbolAddress, taken once per device
// with that device current, and is kept per device.
#include <hip/hip_runtime.h>

#include <mutex>

namespace mhar {

constexpr size_t kNoAllocBytes = size_t(64) << 20;   // 64 MiB per device

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

hipError_t noalloc_scratch(void** ptr, size_t* bytes)
{
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
        e = hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    *bytes = kNoAllocBytes;
    return hipSuccess;
}

}  // namespace mhar
