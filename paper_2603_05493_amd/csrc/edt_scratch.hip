// Device-resident scratch of the allocation-free distance transform
// (wb_edt_noalloc): the two int32 intermediate planes of the three passes,
// for grids of up to WB_EDT_NOALLOC_MAX_VOXELS voxels, in a file-scope
// device array.  Each device that loads the library holds its own copy
// until the process ends.  Host code never passes the array's name to a
// kernel (in host code it is only a stand-in for the symbol): it looks up
// the array's device address once per device with hipGetSymbolAddress, with
// that device current, and hands out that address.
#include <hip/hip_runtime.h>
#include <mutex>
#include "wb.h"
#include "edt_scratch.h"

namespace wb {

static __device__ __align__(256) int32_t edt_scratch[2 * (size_t)WB_EDT_NOALLOC_MAX_VOXELS];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
int32_t *g_ptr[kMaxDevices] = {};
}  // namespace

// Device address of the scratch array on the current device (looked up on
// the first call per device, then cached).  Fails for a device index beyond
// kMaxDevices or when the runtime cannot resolve the symbol.
hipError_t edt_scratch_address(int32_t **out, size_t *bytes) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(edt_scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_ptr[dev] = static_cast<int32_t *>(p);
    }
    *out = g_ptr[dev];
    *bytes = sizeof(edt_scratch);
    return hipSuccess;
}

}  // namespace wb
