// The workspace of fbp_reconstruct_noalloc: a static device array, so that the
// entry point never allocates.  Each GPU that loads the library holds its own
// copy (at its own address) until the process ends.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/fbp.h"
#include "fbp_internal.hpp"

namespace fbp {
namespace {

static __device__ __align__(256) unsigned char scratch[FBP_NOALLOC_WORKSPACE_BYTES];

constexpr int kMaxDevices = 64;

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};   // device address of `scratch` on each device, once looked up

}  // namespace

// The array's device address on the current device.  In host code `scratch` is
// only a host-side stand-in for the symbol, so the address is looked up once per
// device (with that device current) and every later use goes through it.
hipError_t noalloc_workspace(void** ptr, size_t* bytes) {
    int device = 0;
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess) return e;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[device]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p || (reinterpret_cast<uintptr_t>(p) & 255u) != 0) return hipErrorInvalidSymbol;
        g_scratch[device] = p;
    }
    *ptr = g_scratch[device];
    *bytes = sizeof(scratch);
    return hipSuccess;
}

}  // namespace fbp
