// group8.hip -- eight lanes per matrix for FP64 elements (double and complex
// double), inversion of orders up to 16 in plain precision.
//
// Up to order 8 a lane owns one column (eight matrices per wave); above it a
// lane owns columns q and q + 8.  Broadcasts inside an eight-lane group are
// ds_swizzle moves.  Against the sixteen-lane kernel this halves the lanes per
// matrix and, up to order 8, the padding to order 16; against one lane per
// matrix it keeps a column, not a whole triangle, in a lane's registers.
#include "group_impl.hpp"

namespace ci {

template <class V>
static hipError_t group8_run(int n, int method, const BatchArgs& p, hipStream_t s)
{
    if (n <= 8) {
        if (method == 0) return group_run<V, 8, 8, OP_INV, 0, 0>(p, n, s);
        return group_run<V, 8, 8, OP_INV, 1, 0>(p, n, s);
    }
    if (method == 0) return group_run<V, 16, 8, OP_INV, 0, 0>(p, n, s);
    return group_run<V, 16, 8, OP_INV, 1, 0>(p, n, s);
}

hipError_t launch_group8(int dtype, int n, int op, int method, int mixed, const BatchArgs& p,
                         hipStream_t s)
{
    if (op != OP_INV || mixed || n < 1 || n > 16) return hipErrorNotSupported;
    if (dtype == DT_F64) return group8_run<double>(n, method, p, s);
    if (dtype == DT_C128) return group8_run<cd>(n, method, p, s);
    return hipErrorNotSupported;
}

}  // namespace ci
