// tpm_f32_hi.hip -- thread-per-matrix kernels for float elements, orders 9..TPM_NMAX_REAL.
#include "tpm_impl.hpp"

namespace ci {

hipError_t launch_tpm_f32_hi(int n, int op, int method, int mixed, const BatchArgs& p,
                                 hipStream_t s)
{
    if (n < 9 || n > TPM_NMAX_REAL) return hipErrorNotSupported;
    return tpm_run_range<float, 9>(n, op, method, mixed, p, s,
                                 std::make_integer_sequence<int, TPM_NMAX_REAL - 8>{});
}

}  // namespace ci
