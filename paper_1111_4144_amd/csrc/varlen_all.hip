// varlen_all.hip -- the uneven-order batch path for real element types
// (float, double; orders 1..64), and the library-held scratch array of the
// allocation-free variant of that path.
#include <mutex>

#include "varlen_impl.hpp"
#include "ci_large.hpp"
#include "cholinv.h"

namespace ci {

// ---- library-held scratch (allocation-free entry point) ---------------------
// The bucketing plan and the sorted work list of one uneven batch of up to
// CI_NOALLOC_MAX_BATCH matrices.  Every device the library runs on holds its
// own copy for the life of the process.  In host code the name `scratch` is
// only a stand-in: its device address comes from hipGetSymbolAddress, taken
// once per device with that device current, and only that address is ever
// passed to a kernel.
constexpr size_t NOALLOC_SCRATCH_BYTES =
    varlen_plan_bytes() + ((size_t)CI_NOALLOC_MAX_BATCH * sizeof(int32_t) + 255) / 256 * 256;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[NOALLOC_MAX_DEVICES];

size_t noalloc_scratch_bytes() { return NOALLOC_SCRATCH_BYTES; }

hipError_t noalloc_scratch(void** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

size_t varlen_workspace(int64_t batch)
{
    return varlen_plan_bytes() + ((size_t)(batch > 0 ? batch : 0) * sizeof(int32_t) + 255) / 256 * 256;
}

hipError_t launch_varlen(int dtype, int64_t batch, const int32_t* n_dev, const int64_t* off_dev,
                         int n_max, const void* a, void* x, int method, int mixed, int ns_steps,
                         int fill, int32_t* info, void* work, hipStream_t s, int big_from)
{
    switch (dtype) {
    case DT_F32:
        return varlen_dispatch<float>(batch, n_dev, off_dev, n_max, a, x, method, mixed, ns_steps,
                                      fill, info, work, s, big_from);
    case DT_F64:
        return varlen_dispatch<double>(batch, n_dev, off_dev, n_max, a, x, method, mixed, ns_steps,
                                       fill, info, work, s, big_from);
    default:
        return hipErrorNotSupported;
    }
}

}  // namespace ci
