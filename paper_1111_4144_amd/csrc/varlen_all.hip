// varlen_all.hip -- the uneven-order batch path for real element types
// (float, double; orders 1..64).
#include "varlen_impl.hpp"
#include "ci_large.hpp"

namespace ci {

size_t varlen_workspace(int64_t batch)
{
    return varlen_plan_bytes() + ((size_t)(batch > 0 ? batch : 0) * sizeof(int32_t) + 255) / 256 * 256;
}

hipError_t launch_varlen(int dtype, int64_t batch, const int32_t* n_dev, const int64_t* off_dev,
                         int n_max, const void* a, void* x, int method, int mixed, int ns_steps,
                         int fill, int32_t* info, void* work, hipStream_t s)
{
    switch (dtype) {
    case DT_F32:
        return varlen_dispatch<float>(batch, n_dev, off_dev, n_max, a, x, method, mixed, ns_steps,
                                      fill, info, work, s);
    case DT_F64:
        return varlen_dispatch<double>(batch, n_dev, off_dev, n_max, a, x, method, mixed, ns_steps,
                                       fill, info, work, s);
    default:
        return hipErrorNotSupported;
    }
}

}  // namespace ci
