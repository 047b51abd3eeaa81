// util.hip -- small utility kernels shared by the entry points.
#include "ci_large.hpp"
#include "ci_launch.hpp"

namespace ci {

__global__ void k_fill_i32(int32_t* p, int64_t count, int32_t v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

hipError_t fill_i32(int32_t* p, int64_t count, int32_t value, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, count,
                       value);
    return hipGetLastError();
}


}  // namespace ci
