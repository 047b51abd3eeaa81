// bwd_all.hip -- backward kernels instantiated for every element type.
#include "bwd_impl.hpp"

namespace ci {

hipError_t launch_backward(int dtype, int n, const void* x, const void* g, void* ga,
                           int64_t batch, int64_t stride, hipStream_t s)
{
    switch (dtype) {
    case DT_F32: return bwd_run<float>(n, x, g, ga, batch, stride, s);
    case DT_F64: return bwd_run<double>(n, x, g, ga, batch, stride, s);
    case DT_C64: return bwd_run<cf>(n, x, g, ga, batch, stride, s);
    case DT_C128: return bwd_run<cd>(n, x, g, ga, batch, stride, s);
    default: return hipErrorNotSupported;
    }
}

}  // namespace ci
