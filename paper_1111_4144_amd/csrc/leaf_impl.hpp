// leaf_impl.hpp -- Cholesky of one NB x NB block and its inverse factor
// Y = R^{-1} with the updates on the matrix cores, one workgroup of four
// waves, the block in LDS: the diagonal blocks of the large-order
// factorisation.  Its MFMA tile and broadcast helpers also serve the uneven
// batch's one-wave kernel.
//
// Sub-blocks of LF_SB columns: wave 0 factors the diagonal sub-block in
// registers (one lane per column; row i of R reaches every lane by readlane
// from its owners; FP64 pivot accumulators in mixed precision) and inverts it
// the same way; then all waves apply it with MFMA 16x16x4 tiles: the
// sub-block's panel row R_{b,>b} = R_bb^{-T} A_{b,>b} and the upper part of
// A_{>b,>b} -= R_{b,>b}^T R_{b,>b}.  Last, the off-diagonal blocks of R^{-1},
// block rows bottom-up: Y_{a,>a} = -Y_aa (R_{a,>a} Y_{>a,>a}), as MFMA tiles.
// One workgroup barrier separates the phases (five per sub-block and four per
// inverse block row) instead of one per row.
#pragma once

#include "ci_types.hpp"
#include "mfma.hpp"

namespace ci {

constexpr int LF_SB = 16;
constexpr int LF_THREADS = 256;
template <class T, int NB> constexpr int lf_ld() { return NB + 16 / (int)sizeof(T); }   // padded row

template <class T>
__device__ __forceinline__ T lf_bcast(T v, int src)
{
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), src));
    } else {
        const uint64_t u = __builtin_bit_cast(uint64_t, v);
        const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)u, src);
        const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), src);
        return __builtin_bit_cast(T, ((uint64_t)hi << 32) | lo);
    }
}

// One 16 x 16 output tile: d += sum_k A(r, k) B(k, c) for k in [0, K), K a
// multiple of 4; lane (g, cc) supplies A(cc, k + g) and B(k + g, cc).
template <class T, class FA, class FB>
__device__ __forceinline__ void lf_tile(typename mfma_acc<T>::type& d, int K, int g, int cc, FA fa,
                                        FB fb)
{
    for (int k = 0; k < K; k += 4) d = mfma16(fa(cc, k + g), fb(k + g, cc), d);
}

// On entry Rm (row major, leading dimension lf_ld<T, NB>) holds the block's
// upper triangle (zero below, the identity beyond the first nl rows), Ym is
// zero, and in mixed precision dl[j] the FP64 pivot accumulator of column j.
// On return Rm holds R (upper) and Ym = R^{-1} (upper).  Every thread of the
// workgroup calls this together.  Returns, on wave 0, the 1-based index of
// the first failing pivot below nl (0 if none); other waves return 0.
template <class T, int NB, int MIXED>
__device__ int lf_factor_inverse(T* __restrict__ Rm, T* __restrict__ Ym, double* __restrict__ dl,
                                 int nl)
{
    constexpr int LD = lf_ld<T, NB>(), SB = LF_SB, NSB = NB / SB;
    using Acc = typename mfma_acc<T>::type;
    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
    const int g = lane / 16, cc = lane % 16;
    int fail = 0;

    for (int b = 0; b < NSB; ++b) {
        const int b0 = b * SB, b1 = b0 + SB, nr = NB - b1;
        // ---- wave 0: factor and invert the diagonal sub-block in registers
        if (wave == 0) {
            const int j = lane;                       // column b0 + j (lanes >= SB idle)
            T c[SB];
#pragma unroll
            for (int k = 0; k < SB; ++k)
                c[k] = (j < SB && k <= j) ? Rm[(b0 + k) * LD + b0 + j] : T(0);
            double dj = (MIXED && j < SB) ? dl[b0 + j] : 0.0;
            T sv[SB];                                 // 1/r_kk, uniform
#pragma unroll
            for (int i = 0; i < SB; ++i) {
                // the pivot reaches every lane first, so its square root needs
                // no broadcast after it
                const double piv = MIXED ? lf_bcast(dj, i) : (double)lf_bcast(c[i], i);
                T r_ii, s_i;
                if constexpr (sizeof(T) == 4) {
                    double r, y;
                    sqrt_rsqrt_est(piv, r, y);
                    r_ii = (T)r;
                    s_i = (T)y;
                } else {
                    const double r = sqrt(piv);
                    r_ii = (T)r;
                    s_i = (T)(1.0 / r);
                }
                const bool ok = piv > 0.0 && piv < __builtin_inf();
                if (!ok && !fail && b0 + i < nl) fail = b0 + i + 1;
                sv[i] = s_i;
                c[i] = (j > i) ? c[i] * s_i : ((j == i) ? r_ii : c[i]);
                if (MIXED && j > i) dj = fma(-(double)c[i], (double)c[i], dj);
#pragma unroll
                for (int k = i + 1; k < SB; ++k) c[k] -= lf_bcast(c[i], k) * c[i];
            }
            // Y_bb: column j bottom-up, y_kj = -s_k sum_{m > k} r_km y_mj, each
            // y_mj added to every row above it as soon as it is known (two
            // dependent operations per row instead of a serial sum)
            T y[SB], acc[SB];
#pragma unroll
            for (int k = 0; k < SB; ++k) acc[k] = T(0);
#pragma unroll
            for (int m = SB - 1; m >= 0; --m) {
                y[m] = (j > m) ? -sv[m] * acc[m] : ((j == m) ? sv[m] : T(0));
#pragma unroll
                for (int k = 0; k < m; ++k) acc[k] += lf_bcast(c[k], m) * y[m];
            }
            if (j < SB) {
#pragma unroll
                for (int k = 0; k < SB; ++k) {
                    if (k <= j) {
                        Rm[(b0 + k) * LD + b0 + j] = c[k];
                        Ym[(b0 + k) * LD + b0 + j] = y[k];
                    }
                }
            }
        }
        __syncthreads();
        if (nr == 0) break;
        // ---- panel row R_{b,>b} = Y_bb^T A_{b,>b} (tiles held in registers
        // until every wave has read A_{b,>b})
        constexpr int PT_MAX = (SB / 16) * ((NB - SB) / 16);
        constexpr int PT_PER = (PT_MAX + 3) / 4;
        const int ptn = nr / 16, pt = (SB / 16) * ptn;
        Acc pacc[PT_PER];
#pragma unroll
        for (int u = 0; u < PT_PER; ++u) {
            pacc[u] = Acc{0, 0, 0, 0};
            const int t = wave + 4 * u;
            if (t < pt) {
                const int tr = t / ptn, tc = t % ptn;
                lf_tile<T>(pacc[u], SB, g, cc,
                           [&](int r, int k) { return Ym[(b0 + k) * LD + b0 + 16 * tr + r]; },
                           [&](int k, int cl) { return Rm[(b0 + k) * LD + b1 + 16 * tc + cl]; });
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < PT_PER; ++u) {
            const int t = wave + 4 * u;
            if (t < pt) {
                const int tr = t / ptn, tc = t % ptn;
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    Rm[(b0 + 16 * tr + mfma_acc<T>::row(g, v)) * LD + b1 + 16 * tc + cc] = pacc[u][v];
            }
        }
        __syncthreads();
        // ---- FP64 pivots of the remaining columns, and the upper part of
        // A_{>b,>b} -= R_{b,>b}^T R_{b,>b}
        if (MIXED) {
            for (int jj = tid; jj < nr; jj += LF_THREADS) {
                double q = dl[b1 + jj];
#pragma unroll 8
                for (int k = 0; k < SB; ++k) {
                    const double v = (double)Rm[(b0 + k) * LD + b1 + jj];
                    q = fma(-v, v, q);
                }
                dl[b1 + jj] = q;
            }
        }
        const int st = ptn * (ptn + 1) / 2;
        for (int t = wave; t < st; t += 4) {
            int tr = 0, rem = t;
            while (rem >= ptn - tr) { rem -= ptn - tr; ++tr; }
            const int tc = tr + rem;
            Acc d = Acc{0, 0, 0, 0};
            lf_tile<T>(d, SB, g, cc,
                       [&](int r, int k) { return Rm[(b0 + k) * LD + b1 + 16 * tr + r]; },
                       [&](int k, int cl) { return Rm[(b0 + k) * LD + b1 + 16 * tc + cl]; });
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = b1 + 16 * tr + mfma_acc<T>::row(g, v), jc = b1 + 16 * tc + cc;
                if (jc >= i) Rm[i * LD + jc] -= d[v];
            }
        }
        __syncthreads();
    }
    // ---- off-diagonal blocks of Y = R^{-1}, block rows bottom-up
    for (int a = NSB - 2; a >= 0; --a) {
        const int a0 = a * SB, b1 = a0 + SB, nr = NB - b1, ptn = nr / 16, pt = (SB / 16) * ptn;
        constexpr int PT_PER = ((SB / 16) * ((NB - SB) / 16) + 3) / 4;
        Acc tacc[PT_PER];
        // T = R_{a,>a} Y_{>a,>a} (Y upper triangular: zero below its diagonal)
#pragma unroll
        for (int u = 0; u < PT_PER; ++u) {
            tacc[u] = Acc{0, 0, 0, 0};
            const int t = wave + 4 * u;
            if (t < pt) {
                const int tr = t / ptn, tc = t % ptn;
                lf_tile<T>(tacc[u], 16 * (tc + 1), g, cc,
                           [&](int r, int k) { return Rm[(a0 + 16 * tr + r) * LD + b1 + k]; },
                           [&](int k, int cl) { return Ym[(b1 + k) * LD + b1 + 16 * tc + cl]; });
            }
        }
        // T goes into Y_{a,>a} (still zero, read by nobody in this product)
#pragma unroll
        for (int u = 0; u < PT_PER; ++u) {
            const int t = wave + 4 * u;
            if (t < pt) {
                const int tr = t / ptn, tc = t % ptn;
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    Ym[(a0 + 16 * tr + mfma_acc<T>::row(g, v)) * LD + b1 + 16 * tc + cc] = tacc[u][v];
            }
        }
        __syncthreads();
        // Y_{a,>a} = -Y_aa T (Y_aa upper triangular)
#pragma unroll
        for (int u = 0; u < PT_PER; ++u) {
            tacc[u] = Acc{0, 0, 0, 0};
            const int t = wave + 4 * u;
            if (t < pt) {
                const int tr = t / ptn, tc = t % ptn;
                lf_tile<T>(tacc[u], SB, g, cc,
                           [&](int r, int k) { return Ym[(a0 + 16 * tr + r) * LD + a0 + k]; },
                           [&](int k, int cl) { return Ym[(a0 + k) * LD + b1 + 16 * tc + cl]; });
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < PT_PER; ++u) {
            const int t = wave + 4 * u;
            if (t < pt) {
                const int tr = t / ptn, tc = t % ptn;
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    Ym[(a0 + 16 * tr + mfma_acc<T>::row(g, v)) * LD + b1 + 16 * tc + cc] = -tacc[u][v];
            }
        }
        __syncthreads();
    }
    return fail;
}

}  // namespace ci
