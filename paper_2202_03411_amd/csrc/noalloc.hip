// Fixed device scratch for msft_simulate_noalloc: callers that cannot allocate
// (code under stream capture, serving loops, harnesses that forbid it) run the
// forward model with its workspace in this array instead of a buffer of theirs.
//
// Each device the library runs on holds its own copy of the array for the life
// of the process.  Host code never passes the array's name to a kernel (on the
// host it names a stand-in, not device memory): the device address of each
// copy is looked up once per device with hipGetSymbolAddress and kept.
#include <hip/hip_runtime.h>

#include <mutex>

#include "msft_internal.h"

static __device__ __align__(256) uint8_t scratch[MSFT_NOALLOC_MAX_BYTES];

namespace msft {

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_mutex;
void* g_scratch[MAX_DEVICES] = {};
}  // namespace

int static_scratch(int device, void** ptr)
{
    if (device < 0 || device >= MAX_DEVICES) return (int)hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_scratch[device]) {
        // the caller has made `device` current: this is that device's copy
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return (int)e;
        if (!p) return (int)hipErrorInvalidSymbol;
        g_scratch[device] = p;
    }
    *ptr = g_scratch[device];
    return 0;
}

}  // namespace msft
