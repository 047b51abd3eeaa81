// tpm_c128.hip -- thread-per-matrix kernels instantiated for cd elements.
#include "tpm_impl.hpp"

namespace ci {

hipError_t launch_tpm_c128(int n, int op, int method, int mixed, const BatchArgs& p, hipStream_t s)
{
    if (n < 1 || n > TPM_NMAX_CPLX) return hipErrorNotSupported;
    return tpm_run_range<cd, 1>(n, op, method, mixed, p, s,
                                 std::make_integer_sequence<int, TPM_NMAX_CPLX>{});
}

}  // namespace ci
