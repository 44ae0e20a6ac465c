// Fixed device scratch of kpm_moments_noalloc: one file-scope device array
// per GPU, whose device address is looked up once per device when a system
// is created there.  In host code the array's name is only a host-side
// stand-in; every use goes through the looked-up address.
#include "kpm_internal.h"

#include <hip/hip_runtime.h>

#include <mutex>

namespace {

static __device__ __align__(256) unsigned char scratch[kpm::kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
void *g_addr[kMaxDevices] = {};

}  // namespace

namespace kpm {

hipError_t static_scratch(int device, void **ptr) {
    *ptr = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_addr[device]) {
        // the caller has made `device` current: the address is that GPU's copy
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_addr[device] = p;
    }
    *ptr = g_addr[device];
    return hipSuccess;
}

}  // namespace kpm
