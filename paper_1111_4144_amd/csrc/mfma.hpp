// mfma.hpp -- gfx950 MFMA 16x16x4 wrappers and their lane layout.
//
// Lane l = 0..63, g = l / 16, c = l % 16.  For D = A B + C with A 16 x 4 and
// B 4 x 16 per instruction: lane l supplies A[c][k_g] and B[k_g][c], where
// k_g is the k index that lane group g carries in this instruction (any
// assignment of the four k values to the four groups, the same for A and B).
// The four accumulator values of lane l are D[4 g + v][c] (v = 0..3) for the
// FP32 instruction and D[g + 4 v][c] for the FP64 one (measured on gfx950).
#pragma once

#include <hip/hip_runtime.h>

namespace ci {

typedef float gf4 __attribute__((ext_vector_type(4)));
typedef double gd4 __attribute__((ext_vector_type(4)));

template <class T> struct mfma_acc;
template <> struct mfma_acc<float> {
    using type = gf4;
    static __device__ __forceinline__ int row(int g, int v) { return 4 * g + v; }
};
template <> struct mfma_acc<double> {
    using type = gd4;
    static __device__ __forceinline__ int row(int g, int v) { return g + 4 * v; }
};

__device__ __forceinline__ gf4 mfma16(float a, float b, gf4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ gd4 mfma16(double a, double b, gd4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

}  // namespace ci
