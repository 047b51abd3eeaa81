// ci_nonherm.hpp -- launchers of the non-Hermitian inversion's products
// (internal to libcholinv).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ci {

// a = D D^* (upper triangle, real diagonal) for a batch of n x n matrices D
// (matrix b at d + b*sd, leading dimension n); a is dense, stride n*n.
hipError_t launch_gram(int dtype, const void* d, int64_t sd, void* a, int64_t batch, int n,
                       hipStream_t s);
// out = D^* X for a batch (X dense with stride n*n, out at out + b*so).
hipError_t launch_adjoint_product(int dtype, const void* d, int64_t sd, const void* x, void* out,
                                  int64_t so, int64_t batch, int n, hipStream_t s);

}  // namespace ci
