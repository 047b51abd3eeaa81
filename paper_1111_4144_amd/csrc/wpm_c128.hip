// wpm_c128.hip -- LDS-resident group kernels (orders 17..64) for cd elements.
#include "wpm_impl.hpp"

namespace ci {

hipError_t launch_wpm_c128(int n, int op, int method, int mixed, const BatchArgs& p,
                            hipStream_t s)
{
    if (n <= 32) return wpm_run_ops<cd, 32>(n, op, method, mixed, p, s);
    if (n <= 64) return wpm_run_ops<cd, 64>(n, op, method, mixed, p, s);
    return hipErrorNotSupported;
}

}  // namespace ci
