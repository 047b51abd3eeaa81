// q15.hip -- fixed-point (Q15 storage, Q30 sums in int64) form of the
// proposed inversion: Cholesky by eqs. 3-4 with an exact integer square root
// and rounded integer division, then the Section IV.A back-substitution for
// the upper half of X with one power-of-two exponent per matrix, mirrored.
//
// Format (the paper names none): input q_ij (int16 re, im) stands for
// q_ij / 2^15; R entries are Q15, saturating at +-32767; the inverse is built
// as Y = X 2^F in int64 with F = 2 floor(log2 min r_ii) - ceil(log2 n) and Y
// parts saturating at +-(2^40 - 1); the output is int16 mantissas x_ij with
// X = x 2^xexp, the smallest shift that fits.  Every rounding is to nearest
// with halves away from zero.  Saturations are counted per matrix.
//
// The Section III comparison methods run in the same format (variant QV:
// 1 = III.A, 2 = III.B, Cholesky only): the same factor and output stage;
// the forward solution b of III.A (one column at a time) and M = R^{-1} of
// III.B are held as W = (.) 2^G in int64, G = floor(log2 min r_ii) + 13 -
// ceil(ceil(log2 n) / 2), saturating at +-(2^29 - 1) so that every sum of
// two-factor products stays below 2^63.  III.B forms X = M M^* in place over
// M: row i of X, left to right, needs only entries of M right of the one it
// replaces and rows below it.
//
// One lane per matrix.  The integer work is long (int64 products and
// divisions), so a lane keeps its factor and its Y in LDS, entry-major with
// the block's 16 lanes interleaved (conflict-free), and the block is small;
// its LDS is sized for order 8 or 16, whichever holds n.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ci_q15.hpp"

namespace ci {

namespace {

constexpr int QL = 16;                      // lanes (matrices) per block
constexpr int QN_MAX = 16;                  // largest order

// packed index of (i, j), i <= j, of the upper triangle of order QN
template <int QN>
__device__ __forceinline__ int qp(int i, int j) { return i * QN - (i * (i - 1)) / 2 + (j - i); }

// floor(sqrt(v)), 0 <= v < 2^31: a double estimate corrected to the exact floor
__device__ __forceinline__ int64_t q_sqrt_floor(int64_t v)
{
    int64_t r = (int64_t)sqrt((double)v);
    while (r * r > v) --r;
    while ((r + 1) * (r + 1) <= v) ++r;
    return r;
}

// num / den to nearest, halves away from zero (den > 0)
__device__ __forceinline__ int64_t q_div(int64_t num, int64_t den)
{
    const bool neg = num < 0;
    const int64_t m = neg ? -num : num;
    int64_t q = m / den;
    if (2 * (m - q * den) >= den) ++q;
    return neg ? -q : q;
}

__device__ __forceinline__ int64_t q_sat(int64_t v, int64_t lim, int& sat)
{
    if (v > lim) { ++sat; return lim; }
    if (v < -lim) { ++sat; return -lim; }
    return v;
}

// QN: the order the block's LDS is sized for (8 or 16; n <= QN), so that
// blocks of small orders take a quarter of the LDS and more of them reside.
// QV: 0 the Section IV.A back-substitution, 1 III.A, 2 III.B.
template <int QN, int QV>
__global__ void __launch_bounds__(QL)
k_inv_q15(const int16_t* __restrict__ a, int64_t stride, int16_t* __restrict__ x,
          int32_t* __restrict__ xexp, int32_t* __restrict__ sat_out, int32_t* __restrict__ info,
          int64_t batch, int n)
{
    constexpr int QE = QN * (QN + 1) / 2;   // packed upper entries
    constexpr int QW = (QV == 1) ? QN : 1;  // III.A's forward solution
    __shared__ int32_t Rr[QE * QL], Ri[QE * QL];
    __shared__ int64_t Yr[QE * QL], Yi[QE * QL];
    __shared__ int64_t Wr[QW * QL], Wi[QW * QL];
    const int l = threadIdx.x;
    const int64_t b = (int64_t)blockIdx.x * QL + l;
    if (b >= batch) return;                 // lanes share no LDS entries
    const int16_t* ab = a + b * stride * 2;
    int16_t* xb = x + b * stride * 2;
#define RR(i, j) Rr[qp<QN>(i, j) * QL + l]
#define RI(i, j) Ri[qp<QN>(i, j) * QL + l]
#define YR(i, j) Yr[qp<QN>(i, j) * QL + l]
#define YI(i, j) Yi[qp<QN>(i, j) * QL + l]
#define WR(j) Wr[(j) * QL + l]
#define WI(j) Wi[(j) * QL + l]
    constexpr int64_t QMAX = 32767, YLIM = ((int64_t)1 << 40) - 1, WLIM = ((int64_t)1 << 29) - 1;
    int sat = 0, fail = 0;

    // eqs. 3-4: R in Q15, sums in Q30
    for (int i = 0; i < n && !fail; ++i) {
        int64_t acc = (int64_t)ab[2 * (i * n + i)] * 32768;
        for (int k = 0; k < i; ++k) {
            const int64_t pr = RR(k, i), pi = RI(k, i);
            acc -= pr * pr + pi * pi;
        }
        if (acc <= 0) { fail = i + 1; break; }
        const int64_t d = q_sqrt_floor(acc);
        RR(i, i) = (int32_t)d;
        RI(i, i) = 0;
        for (int j = i + 1; j < n; ++j) {
            int64_t sr = (int64_t)ab[2 * (i * n + j)] * 32768;
            int64_t si = (int64_t)ab[2 * (i * n + j) + 1] * 32768;
            for (int k = 0; k < i; ++k) {
                const int64_t ur = RR(k, i), ui = RI(k, i), vr = RR(k, j), vi = RI(k, j);
                sr -= ur * vr + ui * vi;         // conj(r_ki) r_kj
                si -= ur * vi - ui * vr;
            }
            RR(i, j) = (int32_t)q_sat(q_div(sr, d), QMAX, sat);
            RI(i, j) = (int32_t)q_sat(q_div(si, d), QMAX, sat);
        }
    }
    if (fail) {
        for (int e = 0; e < 2 * n * n; ++e) xb[e] = 0;
        xexp[b] = 0;
        if (sat_out) sat_out[b] = sat;
        if (info) info[b] = fail;
        return;
    }

    int64_t rmin = QMAX;
    for (int i = 0; i < n; ++i) rmin = min(rmin, (int64_t)RR(i, i));
    int bb = 0;
    while ((rmin >> (bb + 1)) > 0) ++bb;
    int lg = 0;
    while ((1 << lg) < n) ++lg;
    const int F = 2 * bb - lg;

    const int G = bb + 13 - (lg + 1) / 2;
    if constexpr (QV == 1) {
        // III.A: columns i = n-1..0; forward R^* b = e_i (rows j >= i), then
        // backward R x = b (rows j = i..0) with xh_ki = conj(x_ik) for k > i
        const int64_t up = (int64_t)1 << (F + 15 - G);
        for (int i = n - 1; i >= 0; --i) {
            for (int j = i; j < n; ++j) {
                int64_t sr = (j == i) ? ((int64_t)1 << (G + 15)) : 0, si = 0;
                for (int k = i; k < j; ++k) {          // conj(r_kj) b_k
                    const int64_t rr = RR(k, j), ri = RI(k, j), wr = WR(k), wi = WI(k);
                    sr -= rr * wr + ri * wi;
                    si -= rr * wi - ri * wr;
                }
                const int64_t d = RR(j, j);
                WR(j) = q_sat(q_div(sr, d), WLIM, sat);
                WI(j) = q_sat(q_div(si, d), WLIM, sat);
            }
            for (int j = i; j >= 0; --j) {
                int64_t sr = (j == i) ? WR(j) * up : 0, si = (j == i) ? WI(j) * up : 0;
                for (int k = j + 1; k < n; ++k) {
                    int64_t hr, hi;
                    if (k <= i) { hr = YR(k, i); hi = YI(k, i); }
                    else        { hr = YR(i, k); hi = -YI(i, k); }
                    const int64_t rr = RR(j, k), ri = RI(j, k);
                    sr -= rr * hr - ri * hi;
                    si -= rr * hi + ri * hr;
                }
                const int64_t d = RR(j, j);
                YR(j, i) = q_sat(q_div(sr, d), YLIM, sat);
                YI(j, i) = (j == i) ? 0 : q_sat(q_div(si, d), YLIM, sat);
            }
        }
    } else if constexpr (QV == 2) {
        // III.B: M = R^{-1} 2^G in the Y slots, column by column (rows j = i..0)
        for (int i = 0; i < n; ++i) {
            YR(i, i) = q_sat(q_div((int64_t)1 << (G + 15), (int64_t)RR(i, i)), WLIM, sat);
            YI(i, i) = 0;
            for (int j = i - 1; j >= 0; --j) {
                int64_t sr = 0, si = 0;
                for (int k = j + 1; k <= i; ++k) {     // r_jk m_ki
                    const int64_t rr = RR(j, k), ri = RI(j, k), mr = YR(k, i), mi = YI(k, i);
                    sr -= rr * mr - ri * mi;
                    si -= rr * mi + ri * mr;
                }
                const int64_t d = RR(j, j);
                YR(j, i) = q_sat(q_div(sr, d), WLIM, sat);
                YI(j, i) = q_sat(q_div(si, d), WLIM, sat);
            }
        }
        // X = M M^* upper half, in place: x_ij = sum_{k >= j} m_ik conj(m_jk)
        const int64_t down = (int64_t)1 << (2 * G - F);
        for (int i = 0; i < n; ++i)
            for (int j = i; j < n; ++j) {
                int64_t sr = 0, si = 0;
                for (int k = j; k < n; ++k) {
                    const int64_t ar = YR(i, k), ai = YI(i, k), br = YR(j, k), bi = YI(j, k);
                    sr += ar * br + ai * bi;
                    si += ai * br - ar * bi;
                }
                YR(i, j) = q_sat(q_div(sr, down), YLIM, sat);
                YI(i, j) = (j == i) ? 0 : q_sat(q_div(si, down), YLIM, sat);
            }
    } else {
    // Section IV.A: rows bottom-up, each row's diagonal last
    for (int i = n - 1; i >= 0; --i) {
        const int64_t d = RR(i, i);
        const int64_t t = q_div((int64_t)1 << (F + 30), d);     // s_i 2^(F+15)
        for (int j = n - 1; j >= i; --j) {
            int64_t sr = (j == i) ? t : 0, si = 0;
            for (int k = i + 1; k < n; ++k) {
                int64_t hr, hi;
                if (k <= j) { hr = YR(k, j); hi = YI(k, j); }
                else        { hr = YR(j, k); hi = -YI(j, k); }
                const int64_t rr = RR(i, k), ri = RI(i, k);
                sr -= rr * hr - ri * hi;
                si -= rr * hi + ri * hr;
            }
            YR(i, j) = q_sat(q_div(sr, d), YLIM, sat);
            YI(i, j) = (j == i) ? 0 : q_sat(q_div(si, d), YLIM, sat);
        }
    }
    }

    int64_t m = 0;
    for (int i = 0; i < n; ++i)
        for (int j = i; j < n; ++j) {
            const int64_t vr = YR(i, j), vi = YI(i, j);
            m = max(m, max(vr < 0 ? -vr : vr, vi < 0 ? -vi : vi));
        }
    int s = 0;
    while (q_div(m, (int64_t)1 << s) > QMAX) ++s;
    for (int i = 0; i < n; ++i)
        for (int j = i; j < n; ++j) {
            const int16_t vr = (int16_t)q_div(YR(i, j), (int64_t)1 << s);
            const int16_t vi = (int16_t)q_div(YI(i, j), (int64_t)1 << s);
            xb[2 * (i * n + j)] = vr;
            xb[2 * (i * n + j) + 1] = vi;
            xb[2 * (j * n + i)] = vr;
            xb[2 * (j * n + i) + 1] = (int16_t)-vi;
        }
    xexp[b] = s - F;
    if (sat_out) sat_out[b] = sat;
    if (info) info[b] = 0;
#undef RR
#undef RI
#undef YR
#undef YI
#undef WR
#undef WI
}

}  // namespace

template <int QV>
static void launch_q15_variant(const int16_t* a, int64_t stride, int16_t* x, int32_t* xexp,
                               int32_t* sat, int32_t* info, int64_t batch, int n, hipStream_t s)
{
    const dim3 grid((unsigned)((batch + QL - 1) / QL)), block(QL);
    if (n <= 8)
        hipLaunchKernelGGL((k_inv_q15<8, QV>), grid, block, 0, s, a, stride, x, xexp, sat, info,
                           batch, n);
    else
        hipLaunchKernelGGL((k_inv_q15<16, QV>), grid, block, 0, s, a, stride, x, xexp, sat, info,
                           batch, n);
}

hipError_t launch_inv_q15(const int16_t* a, int64_t stride, int16_t* x, int32_t* xexp,
                          int32_t* sat, int32_t* info, int64_t batch, int n, hipStream_t s,
                          int variant)
{
    if (batch <= 0 || n <= 0) return hipSuccess;
    if (n > QN_MAX) return hipErrorNotSupported;
    switch (variant) {
    case 0: launch_q15_variant<0>(a, stride, x, xexp, sat, info, batch, n, s); break;
    case 1: launch_q15_variant<1>(a, stride, x, xexp, sat, info, batch, n, s); break;
    case 2: launch_q15_variant<2>(a, stride, x, xexp, sat, info, batch, n, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace ci
