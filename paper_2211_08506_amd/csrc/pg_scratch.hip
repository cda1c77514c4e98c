// pg_scratch.hip -- the library's fixed device scratch buffer, for the
// forward entry point that allocates nothing (pg_grid_forward_static).
//
// The array below lives in the code object: every device the library is
// loaded on holds its own copy, at its own address, until the process ends.
// Host code never passes the array's name to a kernel (on the host it is
// only a stand-in symbol); scratch_init() looks up the device address once
// per device, with that device current, and every later use goes through
// scratch_ptr().
#include <hip/hip_runtime.h>

#include <mutex>

#include "pg_launch.hpp"

namespace pg {

static __device__ __align__(256) unsigned char scratch[PG_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};
}  // namespace

hipError_t scratch_init(int device)
{
    if (device < 0 || device >= kMaxDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[device])
        return hipSuccess;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess)
        return e;
    if (cur != device)   // the caller makes the device current first
        return hipErrorInvalidDevice;
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess)
        return e;
    if (!ptr)
        return hipErrorInvalidSymbol;
    g_ptr[device] = ptr;
    return hipSuccess;
}

void *scratch_ptr(int device)
{
    if (device < 0 || device >= kMaxDevices)
        return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_ptr[device];
}

}  // namespace pg
