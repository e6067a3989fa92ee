// cc_static.hip -- the kick entry point that allocates nothing.
//
// cc_kick_static is cc_kick with its scratch memory (the three acceleration
// sums and the error flag) in a file-scope device array of the library
// instead of context buffers, for callers that cannot allocate device memory.
// The array's device address is taken once per device by cc_create (the
// library's set-up call) with the device current; host code uses only that
// address, never the array's name.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/cc.h"
#include "cc_launch.h"

namespace ccg {

// Scratch of cc_kick_static: 3 x CC_KICK_STATIC_MAX_N doubles, then the
// error flag (one int32 at the start of its own 256-byte block): 1.5 MiB per
// device, held until the process ends.
static_assert(STATIC_ACC_BYTES == (size_t)3 * CC_KICK_STATIC_MAX_N * sizeof(double), "static scratch size");
constexpr size_t STATIC_BYTES = STATIC_ACC_BYTES + 256;
static __device__ __align__(256) unsigned char scratch[STATIC_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};  // device address of `scratch` on each device (set up once)
}  // namespace

// With device `dev` current: looks up (once) the device address of the
// scratch array on that device.  Returns hipSuccess or the lookup's error.
hipError_t static_scratch_setup(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[dev]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_ptr[dev] = p;
    return hipSuccess;
}

// The scratch address on `dev`, or nullptr if it was never set up.
void *static_scratch(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_ptr[dev];
}

}  // namespace ccg
