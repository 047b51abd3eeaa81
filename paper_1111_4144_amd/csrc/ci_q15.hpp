// ci_q15.hpp -- launcher of the fixed-point inversion (internal to libcholinv).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ci {

// Q15 inversion of `batch` complex Hermitian matrices of order n <= 16
// (int16 (re, im) pairs, matrix b at a + 2*b*stride, leading dimension n);
// variant 0 the Section IV.A route from R, 1 Section III.A, 2 Section III.B.
hipError_t launch_inv_q15(const int16_t* a, int64_t stride, int16_t* x, int32_t* xexp,
                          int32_t* sat, int32_t* info, int64_t batch, int n, hipStream_t s,
                          int variant = 0);

}  // namespace ci
