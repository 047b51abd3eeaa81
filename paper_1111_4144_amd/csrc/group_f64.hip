// group_f64.hip -- register lane-group kernels (orders up to 16) for double elements.
#include "group_impl.hpp"

namespace ci {

hipError_t launch_group_f64(int n, int op, int method, int mixed, const BatchArgs& p,
                              hipStream_t s)
{
    if (n <= 16) return group_run_ops<double, 16, 16>(n, op, method, mixed, p, s);
    return launch_wpm_f64(n, op, method, mixed, p, s);
}

}  // namespace ci
