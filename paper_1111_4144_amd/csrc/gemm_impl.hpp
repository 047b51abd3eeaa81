// gemm_impl.hpp -- MFMA GEMM tiles for the blocked large-order path (gfx950).
//
//   C = alpha * op(A) * op(B) + beta * C        (real float or double)
//
// op(A) is M x K: A row major M x K (transA = 0) or K x M (transA = 1);
// op(B) is K x N: B row major K x N (transB = 0) or N x K (transB = 1).
// Inputs may be stored in a narrower or wider type than the arithmetic type T
// (TA, TB): they are converted when staged into LDS (FP32 operands of an FP64
// product are exact).  uplo = 1 computes and writes only entries with
// column >= row (tiles entirely below the diagonal are skipped): the upper
// half of a symmetric product.
//
// Tiling: a workgroup of 256 lanes (4 waves, 2 x 2) owns a 128 x 128 tile of
// C; each wave a 64 x 64 sub-tile made of 4 x 4 MFMA blocks of 16 x 16
// (v_mfma_f32_16x16x4f32 / v_mfma_f64_16x16x4f64).  K advances by 16 per
// stage; the next stage's global loads are issued before the current stage's
// MFMAs (register double buffering), LDS holds one stage.
//
// The MFMA operand and accumulator layouts are those of mfma.hpp; lane group
// g takes k = 4 g .. 4 g + 3 of a stage over the four MFMA steps, so each
// lane reads 4 consecutive k values.
#pragma once

#include <stdint.h>

#include <hip/hip_runtime.h>

#include "mfma.hpp"

namespace ci {

struct GemmArgs {
    int M, N, K;
    double alpha, beta;
    const void* A;
    int64_t lda;
    int transA;
    const void* B;
    int64_t ldb;
    int transB;
    void* C;
    int64_t ldc;
    int uplo;
};

constexpr int GT_M = 128, GT_N = 128, GT_K = 16;
constexpr int G_THREADS = 256;

// LDS layouts: As[m][k] (k contiguous, row stride GT_K + PK) and Bs[n][k].
template <class T> constexpr int G_PK = 16 / (int)sizeof(T);   // pad 16 bytes per row

template <class T, class TA, class TB>
__global__ void __launch_bounds__(G_THREADS)
k_gemm(GemmArgs p)
{
    using Acc = typename mfma_acc<T>::type;
    constexpr int LDK = GT_K + G_PK<T>;
    __shared__ __align__(16) T As[GT_M * LDK];
    __shared__ __align__(16) T Bs[GT_N * LDK];

    const int tiles_n = (p.N + GT_N - 1) / GT_N;
    const int bm = blockIdx.x / tiles_n, bn = blockIdx.x % tiles_n;
    const int m0 = bm * GT_M, n0 = bn * GT_N;
    if (p.uplo && n0 + GT_N - 1 < m0) return;       // tile strictly below the diagonal

    const TA* A = static_cast<const TA*>(p.A);
    const TB* B = static_cast<const TB*>(p.B);
    const int tid = threadIdx.x;
    const int wave = tid / 64, lane = tid % 64;
    const int wm = wave / 2, wn = wave % 2;          // 2 x 2 waves, 64 x 64 each
    const int lg = lane / 16, lc = lane % 16;

    Acc acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = Acc{0, 0, 0, 0};

    // Staging: each thread moves 8 elements of A's tile and 8 of B's tile per
    // stage (128 x 16 = 2048 elements each).  Element e = tid + 256 r.
    T ra[8], rb[8];
    auto load_stage = [&](int k0) {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int e = tid + G_THREADS * r;
            // A: tile element (m, k) with the index order chosen so that
            // consecutive lanes read consecutive addresses of the source layout
            int m, k;
            if (p.transA) { m = e % GT_M; k = e / GT_M; } else { k = e % GT_K; m = e / GT_K; }
            const int gm = m0 + m, gk = k0 + k;
            T v = T(0);
            if (gm < p.M && gk < p.K)
                v = (T)(p.transA ? A[(int64_t)gk * p.lda + gm] : A[(int64_t)gm * p.lda + gk]);
            ra[r] = v;
            int n, kb;
            if (p.transB) { kb = e % GT_K; n = e / GT_K; } else { n = e % GT_N; kb = e / GT_N; }
            const int gn = n0 + n, gkb = k0 + kb;
            T w = T(0);
            if (gn < p.N && gkb < p.K)
                w = (T)(p.transB ? B[(int64_t)gn * p.ldb + gkb] : B[(int64_t)gkb * p.ldb + gn]);
            rb[r] = w;
        }
    };
    auto store_stage = [&]() {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int e = tid + G_THREADS * r;
            int m, k;
            if (p.transA) { m = e % GT_M; k = e / GT_M; } else { k = e % GT_K; m = e / GT_K; }
            As[m * LDK + k] = ra[r];
            int n, kb;
            if (p.transB) { kb = e % GT_K; n = e / GT_K; } else { n = e % GT_N; kb = e / GT_N; }
            Bs[n * LDK + kb] = rb[r];
        }
    };

    const int nk = (p.K + GT_K - 1) / GT_K;
    if (nk > 0) load_stage(0);
    for (int s = 0; s < nk; ++s) {
        __syncthreads();                 // previous stage's MFMA reads are done
        store_stage();
        __syncthreads();
        if (s + 1 < nk) load_stage((s + 1) * GT_K);   // in flight during the MFMAs
        // operands: lane group lg takes k = 4 lg .. 4 lg + 3
        T af[4][4], bf[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const T* pa = As + (wm * 64 + i * 16 + lc) * LDK + 4 * lg;
            const T* pb = Bs + (wn * 64 + i * 16 + lc) * LDK + 4 * lg;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                af[i][c] = pa[c];
                bf[i][c] = pb[c];
            }
        }
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = mfma16(af[i][c], bf[j][c], acc[i][j]);
    }

    // epilogue: lane holds D[row(lg, v)][lc] of block (i, j)
    T* C = static_cast<T*>(p.C);
    const T alpha = (T)p.alpha, beta = (T)p.beta;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gm = m0 + wm * 64 + i * 16 + mfma_acc<T>::row(lg, v);
                const int gn = n0 + wn * 64 + j * 16 + lc;
                if (gm < p.M && gn < p.N && (!p.uplo || gn >= gm)) {
                    T* c = C + (int64_t)gm * p.ldc + gn;
                    const T val = alpha * acc[i][j][v];
                    *c = (beta == T(0)) ? val : val + beta * (*c);
                }
            }
}

template <class T, class TA, class TB>
static hipError_t gemm_launch(const GemmArgs& p, hipStream_t s)
{
    if (p.M <= 0 || p.N <= 0) return hipSuccess;
    const int tiles = ((p.M + GT_M - 1) / GT_M) * ((p.N + GT_N - 1) / GT_N);
    hipLaunchKernelGGL((k_gemm<T, TA, TB>), dim3(tiles), dim3(G_THREADS), 0, s, p);
    return hipGetLastError();
}

}  // namespace ci
