// Fixed device scratch for the entry points that must not allocate
// (hinv_prior_apply_noalloc).  The array below is a file-scope device
// variable: every GPU the library runs on holds its own copy, at its own
// address, from the loading of the code object until the process ends.  In
// host code its name is only a stand-in for that memory, so its per-device
// address is looked up once per device (hipGetSymbolAddress, at context
// creation with the device current) and only that address reaches kernels.
#include <mutex>
#include <vector>

#include "noalloc.h"

namespace {
constexpr size_t kScratchDoubles = hinv::kNoAllocScratchDoubles;
}

static __device__ __align__(256) double scratch[kScratchDoubles];

namespace hinv {

namespace {
std::mutex g_mu;
std::vector<double*> g_ptr;  // device address of `scratch`, by device ordinal
}  // namespace

void noalloc_init(int device) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (device < 0) fail(HINV_EINVAL, "internal: bad device ordinal");
    if ((int)g_ptr.size() <= device) g_ptr.resize(device + 1, nullptr);
    if (g_ptr[device]) return;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        fail(HINV_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_ptr[device] = static_cast<double*>(p);
}

double* noalloc_scratch(int device) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (device < 0 || device >= (int)g_ptr.size() || !g_ptr[device])
        fail(HINV_ESTATE, "no-allocation scratch not set up on this device");
    return g_ptr[device];
}

}  // namespace hinv
