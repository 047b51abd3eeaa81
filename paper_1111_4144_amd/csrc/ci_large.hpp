// ci_large.hpp -- host-side launchers of the blocked large-order path, the
// variable-size batch path and small utilities (internal to libcholinv).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace ci {

enum { LG_FACTOR = 0, LG_INVERSE = 1 };

// info[0..count) = value, with a small kernel (capturable; no memset node).
hipError_t fill_i32(int32_t* p, int64_t count, int32_t value, hipStream_t s);

// Blocked path for one matrix of order n > 64.
size_t large_workspace(int dtype, int64_t n, int which, int mixed);
// cfg selects one of large_config_count() configurations (0 = built-in):
// the diagonal-block kernel, the inverse form and the split-K target.
int large_config_count();
hipError_t large_factor(int dtype, int64_t n, void* a, int64_t lda, int32_t* info, void* work,
                        hipStream_t s, int cfg = 0);
hipError_t large_inverse(int dtype, int64_t n, const void* a, int64_t lda, void* x, int64_t ldx,
                         int mixed, int ns_steps, int fill, int32_t* info, void* work,
                         hipStream_t s, int cfg = 0);

// Variable-size packed batch: device-side bucketing prologue + one persistent
// launch.
size_t varlen_workspace(int64_t batch);
// big_from: smallest order of the four-waves-per-matrix bucket (17, 25 or 33;
// other values mean 33).
hipError_t launch_varlen(int dtype, int64_t batch, const int32_t* n_dev, const int64_t* off_dev,
                         int n_max, const void* a, void* x, int method, int mixed, int ns_steps,
                         int fill, int32_t* info, void* work, hipStream_t s, int big_from = 33);

// Device address of the current device's library-held scratch array (taken
// once per device; the array holds the varlen plan of up to
// CI_NOALLOC_MAX_BATCH matrices), and its size in bytes.
hipError_t noalloc_scratch(void** out);
size_t noalloc_scratch_bytes();

}  // namespace ci
