// Static device scratch for the entry point that allocates nothing
// (mf_sample_noalloc): a file-scope device array, one copy per GPU, whose
// address each device reports through hipGetSymbolAddress.  Host code never
// passes the array's name to a kernel (on the host it is only a stand-in for
// the symbol): it uses the per-device address obtained below.
#include <hip/hip_runtime.h>

#include <mutex>

#include "mf_static.hpp"

namespace mf {

namespace {

__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

hipError_t static_scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_ptr[device]) return hipSuccess;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;  // the device must be current
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[device] = ptr;
    return hipSuccess;
}

void* static_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    return g_ptr[device];
}

}  // namespace mf
