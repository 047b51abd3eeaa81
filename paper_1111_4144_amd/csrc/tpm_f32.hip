// tpm_f32.hip -- thread-per-matrix kernels for float elements, orders 1..8
// (9..16 are in tpm_f32_hi.hip, a separate translation unit so that the
// two compile in parallel).
#include "tpm_impl.hpp"

namespace ci {

hipError_t launch_tpm_f32_hi(int n, int op, int method, int mixed, const BatchArgs& p,
                                 hipStream_t s);

hipError_t launch_tpm_f32(int n, int op, int method, int mixed, const BatchArgs& p, hipStream_t s)
{
    if (n > 8) return launch_tpm_f32_hi(n, op, method, mixed, p, s);
    if (n < 1) return hipErrorNotSupported;
    return tpm_run_range<float, 1>(n, op, method, mixed, p, s, std::make_integer_sequence<int, 8>{});
}

}  // namespace ci
