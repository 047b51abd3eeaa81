// group_f32.hip -- register lane-group kernels (orders up to 16) for float elements.
#include "group16_mfma.hpp"
#include "group_impl.hpp"

namespace ci {

hipError_t launch_group_f32(int n, int op, int method, int mixed, const BatchArgs& p,
                              hipStream_t s)
{
    if (n <= 16) {
        // four-lane groups by default (orders 9..16, mixed precision); an explicit
        // engine request (p.ns_engine set by the tuner) keeps the 16-lane groups
        if (op == OP_INV && n >= 9 && mixed && p.ns_engine < 0)
            return launch_quad16(DT_F32, n, op, method, mixed, p, s);
        const int eng = p.ns_engine >= 0 ? p.ns_engine : ns_engine();
        if (op == OP_INV && mixed && eng == NS_ENGINE_MFMA)
            return group16_mfma_run<float>(p, n, method, s);
        return group_run_ops<float, 16, 16>(n, op, method, mixed, p, s);
    }
    return launch_wpm_f32(n, op, method, mixed, p, s);
}

}  // namespace ci
