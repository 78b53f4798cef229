// Fixed device workspace of the allocation-free evaluation (bemc_eval_noalloc).
//
// The array lives in the code object: every GPU the library runs on holds its own copy of
// kNoAllocScratchBytes from the moment the code object is loaded there until the process
// ends.  Host code never uses the array's name as an address (on the host it only names a
// stand-in); it asks the runtime for the device address once per device and keeps it.
#include <mutex>

#include "bemc_internal.h"

namespace bemc {

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_mu;
void* g_ptr[kNoAllocMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch(int device, void** ptr)
{
    *ptr = nullptr;
    if (device < 0 || device >= kNoAllocMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;  // the caller makes `device` current
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_ptr[device] = p;
    }
    *ptr = g_ptr[device];
    return hipSuccess;
}

}  // namespace bemc
