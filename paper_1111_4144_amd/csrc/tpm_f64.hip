// tpm_f64.hip -- thread-per-matrix kernels instantiated for double elements.
#include "tpm_impl.hpp"

namespace ci {

hipError_t launch_tpm_f64(int n, int op, int method, int mixed, const BatchArgs& p, hipStream_t s)
{
    if (n < 1 || n > TPM_NMAX_REAL) return hipErrorNotSupported;
    return tpm_run_dtype<double>(n, op, method, mixed, p, s,
                              std::make_integer_sequence<int, TPM_NMAX_REAL>{});
}

}  // namespace ci
