// Fixed device scratch of integrate_depth_noalloc: the footprint pyramid of
// the frame and the candidate list of a compacted launch, in one file-scope
// device array instead of buffers the map allocates on first use.
//
// Host code never uses the array's name as an address (on the host it is a
// stand-in, not device memory): the device address is looked up once per
// device with hipGetSymbolAddress, with that device current, and kept.
#include <mutex>

#include "tsdf_internal.hpp"

namespace tsdf {

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 256;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];
}  // namespace

hipError_t noalloc_scratch(void **out)
{
    *out = nullptr;
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    if (dev < 0 || dev >= kMaxDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        if (!ptr)
            return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace tsdf
