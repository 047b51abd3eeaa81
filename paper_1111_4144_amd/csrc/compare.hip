// compare.hip -- the two existing inversion methods the paper measures the
// proposed one against, on the GPU for side-by-side accuracy and timing:
//   Section III.A, equation solving: A x_i = e_i (eq. 15) for each column,
//     forward rows j >= i only, back-substitution for the upper half of the
//     column with the already finished columns supplying the rest by the
//     mirror (Cholesky or LDL factor);
//   Section III.B, triangular operations: M = R^{-1} column by column from
//     R m_i = e_i (eq. 18), then the upper half of X = M M^* (eq. 19);
// and, as the reference point of the comparison, the proposed Section IV
// back-substitution in this same framework (same factor code, same LDS
// layout, same reciprocal-then-multiply arithmetic), so that the three
// methods' errors and times differ only by their route from R to X.
// Orders up to 16, one lane per matrix, arithmetic in the element type.  The
// factor and X live in LDS (entry-major, the block's 8 lanes interleaved);
// III.B keeps M in X's place and overwrites it row by row in increasing
// column order, which never reads an overwritten entry.  X goes to the output
// once, at the end.
// Terms whose factor is an exact zero (entries known to vanish) are skipped;
// subtracting them would not change any result.
#include "ci_launch.hpp"
#include "ci_compare.hpp"
#include "ci_types.hpp"

namespace ci {

namespace {

constexpr int CL = 8;                       // lanes (matrices) per block
constexpr int CN = 16;                      // largest order
constexpr int CE = CN * (CN + 1) / 2;

__device__ __forceinline__ int cp(int i, int j) { return i * CN - (i * (i - 1)) / 2 + (j - i); }

template <class V> CI_D V cmul(V a, V b) { V acc = mk<V>(typename vt<V>::real(0)); madd(acc, a, b); return acc; }

// VARIANT 0: III.A with Cholesky, 1: III.A with LDL, 2: III.B (Cholesky),
// 3: Section IV with Cholesky, 4: Section IV with LDL
template <class V, int VARIANT>
__global__ void __launch_bounds__(CL)
k_compare(const V* __restrict__ a, int64_t sa, V* __restrict__ x, int64_t sx,
          int32_t* __restrict__ info, int64_t batch, int n)
{
    using R = typename vt<V>::real;
    __shared__ V Rs[CE * CL];
    __shared__ V Fs[CN * CL];
    __shared__ R Ds[CN * CL];
    __shared__ V Xs[CN * CN * CL];
    const int l = threadIdx.x;
    const int64_t b = (int64_t)blockIdx.x * CL + l;
    if (b >= batch) return;                 // lanes share no LDS entries
    const V* ab = a + b * sa;
    V* xb = x + b * sx;
#define RS(i, j) Rs[cp(i, j) * CL + l]
#define FS(k) Fs[(k) * CL + l]
#define DS(k) Ds[(k) * CL + l]
#define XS(i, j) Xs[((i) * CN + (j)) * CL + l]
    constexpr bool LDL = VARIANT == 1 || VARIANT == 4;
    int fail = 0;
    // ---- factor: eqs. 3-4, or 10-11 for LDL ----
    for (int i = 0; i < n && !fail; ++i) {
        R piv = re(ab[i * n + i]);
        for (int k = 0; k < i; ++k) {
            const V r = RS(k, i);
            const R m2 = re(cmul(cj(r), r));                       // |r_ki|^2
            piv -= LDL ? m2 * DS(k) : m2;
        }
        if (!(piv > R(0) && piv - piv == R(0))) { fail = i + 1; break; }
        const R dv = LDL ? piv : sqrt(piv);
        DS(i) = dv;
        RS(i, i) = mk<V>(LDL ? R(1) : dv);
        for (int j = i + 1; j < n; ++j) {
            V acc = ab[i * n + j];
            for (int k = 0; k < i; ++k) {
                const V t = LDL ? scal(cj(RS(k, i)), DS(k)) : cj(RS(k, i));
                acc = add(acc, neg(cmul(t, RS(k, j))));
            }
            RS(i, j) = scal(acc, R(1) / dv);
        }
    }
    if (fail) {
        for (int e = 0; e < n * n; ++e) xb[e] = nan_value<V>();
        if (info) info[b] = fail;
        return;
    }

    if constexpr (VARIANT <= 1) {
        // ---- III.A: columns from the last; forward rows j >= i (eq. 15) ----
        for (int i = n - 1; i >= 0; --i) {
            for (int j = i; j < n; ++j) {
                V acc = mk<V>(R(j == i ? 1 : 0));
                for (int k = i; k < j; ++k) acc = add(acc, neg(cmul(cj(RS(k, j)), FS(k))));
                FS(j) = LDL ? acc : scal(acc, R(1) / DS(j));
            }
            for (int j = i; j >= 0; --j) {
                // the forward solution of e_i vanishes above row i
                const V fj = (j == i) ? FS(j) : mk<V>(R(0));
                V acc = LDL ? scal(fj, R(1) / DS(j)) : fj;
                for (int k = j + 1; k < n; ++k) {
                    const V xh = (k <= i) ? XS(k, i) : cj(XS(i, k));
                    acc = add(acc, neg(cmul(RS(j, k), xh)));
                }
                V v = LDL ? acc : scal(acc, R(1) / DS(j));
                if (j == i) v = realpart_only(v);
                XS(j, i) = v;
            }
        }
    } else if constexpr (VARIANT >= 3) {
        // ---- Section IV: rows from the bottom, each row's diagonal last:
        // x_ij = (delta_ij s_i - sum_{k>i} r_ik xh_kj) s_i (LDL: without the
        // second s_i), s_i = 1/r_ii or 1/d_i ----
        for (int i = n - 1; i >= 0; --i) {
            const R si = R(1) / DS(i);
            for (int j = n - 1; j >= i; --j) {
                V acc = mk<V>(j == i ? si : R(0));
                for (int k = i + 1; k < n; ++k) {
                    const V xh = (k <= j) ? XS(k, j) : cj(XS(j, k));
                    acc = add(acc, neg(cmul(RS(i, k), xh)));
                }
                V v = LDL ? acc : scal(acc, si);
                if (j == i) v = realpart_only(v);
                XS(i, j) = v;
            }
        }
    } else {
        // ---- III.B: M = R^{-1} (eq. 18) into X's upper triangle ----
        for (int i = 0; i < n; ++i)
            for (int j = i; j >= 0; --j) {
                V acc = mk<V>(R(j == i ? 1 : 0));
                for (int k = j + 1; k <= i; ++k) acc = add(acc, neg(cmul(RS(j, k), XS(k, i))));
                XS(j, i) = scal(acc, R(1) / DS(j));
            }
        // X = M M^* (eq. 19), upper half, in place row by row
        for (int i = 0; i < n; ++i)
            for (int j = i; j < n; ++j) {
                V acc = mk<V>(R(0));
                for (int k = j; k < n; ++k) acc = add(acc, cmul(XS(i, k), cj(XS(j, k))));
                XS(i, j) = (i == j) ? realpart_only(acc) : acc;
            }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) xb[i * n + j] = (j >= i) ? XS(i, j) : cj(XS(j, i));
    if (info) info[b] = 0;
#undef RS
#undef FS
#undef DS
#undef XS
}

template <class V>
hipError_t compare_t(int variant, const void* a, int64_t sa, void* x, int64_t sx, int32_t* info,
                     int64_t batch, int n, hipStream_t s)
{
    const dim3 grid((unsigned)((batch + CL - 1) / CL)), block(CL);
    if (variant == 0)
        hipLaunchKernelGGL((k_compare<V, 0>), grid, block, 0, s, (const V*)a, sa, (V*)x, sx, info, batch, n);
    else if (variant == 1)
        hipLaunchKernelGGL((k_compare<V, 1>), grid, block, 0, s, (const V*)a, sa, (V*)x, sx, info, batch, n);
    else if (variant == 2)
        hipLaunchKernelGGL((k_compare<V, 2>), grid, block, 0, s, (const V*)a, sa, (V*)x, sx, info, batch, n);
    else if (variant == 3)
        hipLaunchKernelGGL((k_compare<V, 3>), grid, block, 0, s, (const V*)a, sa, (V*)x, sx, info, batch, n);
    else
        hipLaunchKernelGGL((k_compare<V, 4>), grid, block, 0, s, (const V*)a, sa, (V*)x, sx, info, batch, n);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_compare(int dtype, int variant, const void* a, int64_t sa, void* x, int64_t sx,
                          int32_t* info, int64_t batch, int n, hipStream_t s)
{
    if (batch <= 0 || n <= 0) return hipSuccess;
    if (n > CN || variant < 0 || variant > 4) return hipErrorNotSupported;
    switch (dtype) {
    case DT_F32: return compare_t<float>(variant, a, sa, x, sx, info, batch, n, s);
    case DT_F64: return compare_t<double>(variant, a, sa, x, sx, info, batch, n, s);
    case DT_C64: return compare_t<cf>(variant, a, sa, x, sx, info, batch, n, s);
    case DT_C128: return compare_t<cd>(variant, a, sa, x, sx, info, batch, n, s);
    default: return hipErrorNotSupported;
    }
}

}  // namespace ci
