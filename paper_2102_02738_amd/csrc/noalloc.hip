// Scratch memory of simus_rf_noalloc: a file-scope device array of
// NOALLOC_SCRATCH_BYTES, one copy per GPU, held from the code object's load
// until the process ends.  On the host the array's name is only a stand-in
// symbol, never a device address: the address is looked up once per device
// (with that device current) by hipGetSymbolAddress, kept, and passed to the
// kernels, copies and fills in its place.
#include <hip/hip_runtime.h>

#include <mutex>

#include "kernels.hpp"

namespace simus {

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

hipError_t noalloc_scratch(char** ptr)
{
    constexpr int MAX_DEVICES = 64;
    static std::mutex mu;
    static char* addr[MAX_DEVICES] = {};
    *ptr = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = static_cast<char*>(p);
    }
    *ptr = addr[dev];
    return hipSuccess;
}

}  // namespace simus
