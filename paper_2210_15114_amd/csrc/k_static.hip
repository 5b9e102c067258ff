// k_static.hip - the library's static device scratch, for callers that cannot
// allocate device memory (dm_matvec_static: code under graph capture, serving
// loops, harnesses that forbid allocation).
//
// `scratch` is one file-scope device array; every GPU the library runs on
// holds its own copy, at its own address, until the process ends.  Host code
// never passes the array's name to a kernel (in host code the name is a
// host-side stand-in, not a device address): the device address is taken once
// per device with hipGetSymbolAddress, with that device current, and kept.
#include <mutex>

#include "dm_internal.h"

namespace dm {

static __device__ __align__(256) char scratch[STATIC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
char* scratch_ptr[MAX_DEVICES];
}  // namespace

hipError_t static_scratch(char** out) {
    *out = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p || ((uintptr_t)p % 256) != 0) return hipErrorInvalidSymbol;
        scratch_ptr[dev] = (char*)p;
    }
    *out = scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace dm
