// Scratch memory of the entry points that allocate nothing
// (wnnc_winding_grad_x_noalloc): one file-scope device array per GPU, held
// until the process ends.  Host code never uses the array's name as an
// address: its device address on each GPU is taken once, at set-up, and
// passed to the kernels as an ordinary pointer.
#include <mutex>

#include "common.h"
#include "internal.h"

namespace wnnc {

namespace {

// grad F of up to kNoallocMaxPoints points (3 floats each): 12 MiB
__device__ __align__(256) float scratch[3 * kNoallocMaxPoints];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
float *g_ptr[kMaxDevices] = {};

}  // namespace

hipError_t noalloc_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_ptr[device]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_ptr[device] = (float *)p;
    return hipSuccess;
}

float *noalloc_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    return g_ptr[device];
}

}  // namespace wnnc
