// nonherm.hip -- the products around the inversion of a general square matrix
// through a Hermitian one (Section III.C): A = D D^* is Hermitian positive
// definite when D is nonsingular, so D^{-1} = D^* A^{-1} needs one Cholesky
// inversion and two products.  Orders are at most 64: one lane computes one
// entry; the lanes of a wave take consecutive columns, so the reads of D's
// rows (gram) and of X's rows (product) are shared or contiguous across it.
#include "ci_launch.hpp"
#include "ci_nonherm.hpp"
#include "ci_types.hpp"

namespace ci {

namespace {

constexpr int NH_THREADS = 256;

template <class V>
__global__ void __launch_bounds__(NH_THREADS)
k_gram(const V* __restrict__ d, int64_t sd, V* __restrict__ a, int64_t batch, int n)
{
    using R = typename vt<V>::real;
    const int64_t nn = (int64_t)n * n;
    const int64_t e = (int64_t)blockIdx.x * NH_THREADS + threadIdx.x;
    if (e >= batch * nn) return;
    const int64_t b = e / nn;
    const int q = (int)(e - b * nn), i = q / n, j = q - (q / n) * n;
    if (j < i) return;                     // the inversion reads the upper triangle only
    const V* di = d + b * sd + (int64_t)i * n;
    const V* dj = d + b * sd + (int64_t)j * n;
    V acc = mk<V>(R(0));
    for (int k = 0; k < n; ++k) madd(acc, di[k], cj(dj[k]));     // a_ij = sum_k d_ik d_jk^*
    a[e] = (i == j) ? realpart_only(acc) : acc;
}

template <class V>
__global__ void __launch_bounds__(NH_THREADS)
k_adjoint_product(const V* __restrict__ d, int64_t sd, const V* __restrict__ x,
                  V* __restrict__ out, int64_t so, int64_t batch, int n)
{
    using R = typename vt<V>::real;
    const int64_t nn = (int64_t)n * n;
    const int64_t e = (int64_t)blockIdx.x * NH_THREADS + threadIdx.x;
    if (e >= batch * nn) return;
    const int64_t b = e / nn;
    const int q = (int)(e - b * nn), i = q / n, j = q - (q / n) * n;
    const V* db = d + b * sd;
    const V* xb = x + b * nn;
    V acc = mk<V>(R(0));
    for (int k = 0; k < n; ++k)
        madd(acc, cj(db[(int64_t)k * n + i]), xb[(int64_t)k * n + j]);   // (D^* X)_ij
    out[b * so + q] = acc;
}

template <class V>
hipError_t gram_t(const void* d, int64_t sd, void* a, int64_t batch, int n, hipStream_t s)
{
    const int64_t total = batch * n * n;
    hipLaunchKernelGGL(k_gram<V>, dim3((unsigned)((total + NH_THREADS - 1) / NH_THREADS)),
                       dim3(NH_THREADS), 0, s, (const V*)d, sd, (V*)a, batch, n);
    return hipGetLastError();
}

template <class V>
hipError_t product_t(const void* d, int64_t sd, const void* x, void* out, int64_t so,
                     int64_t batch, int n, hipStream_t s)
{
    const int64_t total = batch * n * n;
    hipLaunchKernelGGL(k_adjoint_product<V>,
                       dim3((unsigned)((total + NH_THREADS - 1) / NH_THREADS)), dim3(NH_THREADS),
                       0, s, (const V*)d, sd, (const V*)x, (V*)out, so, batch, n);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_gram(int dtype, const void* d, int64_t sd, void* a, int64_t batch, int n,
                       hipStream_t s)
{
    switch (dtype) {
    case DT_F32: return gram_t<float>(d, sd, a, batch, n, s);
    case DT_F64: return gram_t<double>(d, sd, a, batch, n, s);
    case DT_C64: return gram_t<cf>(d, sd, a, batch, n, s);
    case DT_C128: return gram_t<cd>(d, sd, a, batch, n, s);
    default: return hipErrorNotSupported;
    }
}

hipError_t launch_adjoint_product(int dtype, const void* d, int64_t sd, const void* x, void* out,
                                  int64_t so, int64_t batch, int n, hipStream_t s)
{
    switch (dtype) {
    case DT_F32: return product_t<float>(d, sd, x, out, so, batch, n, s);
    case DT_F64: return product_t<double>(d, sd, x, out, so, batch, n, s);
    case DT_C64: return product_t<cf>(d, sd, x, out, so, batch, n, s);
    case DT_C128: return product_t<cd>(d, sd, x, out, so, batch, n, s);
    default: return hipErrorNotSupported;
    }
}

}  // namespace ci
