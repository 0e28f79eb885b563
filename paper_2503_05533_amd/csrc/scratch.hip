// Fixed device scratch of the no-allocation entry point
// (mlmc_sample_level_noalloc): a file-scope device array that every GPU the
// library runs on holds from module load until the process ends.  In host
// code the array's name is only a host-side stand-in; its device address is
// taken once per device with hipGetSymbolAddress (with that device current)
// and only that address is handed to kernels and copies.
#include <hip/hip_runtime.h>

#include <mutex>

#include "kernels.h"

namespace mlmc {

__device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_addr[kMaxDevices] = {};
}  // namespace

hipError_t scratch_device_ptr(int device, void **out)
{
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_addr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_addr[device] = p;
    }
    *out = g_addr[device];
    return hipSuccess;
}

}  // namespace mlmc
