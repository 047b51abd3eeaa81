// group_c64.hip -- register lane-group kernels (orders up to 16) for cf elements.
#include "group16_mfma.hpp"
#include "group_impl.hpp"

namespace ci {

hipError_t launch_group_c64(int n, int op, int method, int mixed, const BatchArgs& p,
                              hipStream_t s)
{
    if (n <= 16) {
        // four-lane groups by default (orders 9..16); an explicit
        // engine request (p.ns_engine set by the tuner) keeps the 16-lane groups
        if (op == OP_INV && n >= 9 && p.ns_engine < 0)
            return launch_quad16(DT_C64, n, op, method, mixed, p, s);
        const int eng = p.ns_engine >= 0 ? p.ns_engine : ns_engine();
        if (op == OP_INV && mixed && eng == NS_ENGINE_MFMA)
            return group16_mfma_run<cf>(p, n, method, s);
        return group_run_ops<cf, 16, 16>(n, op, method, mixed, p, s);
    }
    return launch_wpm_c64(n, op, method, mixed, p, s);
}

}  // namespace ci
