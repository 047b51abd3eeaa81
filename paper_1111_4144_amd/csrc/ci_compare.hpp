// ci_compare.hpp -- launcher of the Section III comparison methods (internal
// to libcholinv).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ci {

// variant 0: III.A (Cholesky), 1: III.A (LDL), 2: III.B, 3: Section IV
// (Cholesky), 4: Section IV (LDL); orders <= 16; a and
// x dense with leading dimension n, matrix b at a + b*sa and x + b*sx.
hipError_t launch_compare(int dtype, int variant, const void* a, int64_t sa, void* x, int64_t sx,
                          int32_t* info, int64_t batch, int n, hipStream_t s);

}  // namespace ci
