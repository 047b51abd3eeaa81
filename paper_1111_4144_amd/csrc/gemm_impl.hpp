// gemm_impl.hpp -- MFMA GEMM tiles for the blocked large-order path (gfx950).
//
//   C = alpha * op(A) * op(B) + beta * C        (real float or double)
//
// op(A) is M x K: A row major M x K (transA = 0) or K x M (transA = 1);
// op(B) is K x N: B row major K x N (transB = 0) or N x K (transB = 1).
// Inputs may be stored in a narrower type than the arithmetic type T (TA, TB):
// they are converted when staged into LDS (FP32 operands of an FP64 product
// are exact).  uplo = 1 computes and writes only entries with column >= row:
// the upper half of a symmetric product; only tiles that meet it are launched.
//
// Tiling: a workgroup of 256 lanes (4 waves, 2 x 2) owns a 128 x 128 tile of
// C; each wave a 64 x 64 sub-tile made of 4 x 4 MFMA blocks of 16 x 16
// (v_mfma_f32_16x16x4f32 / v_mfma_f64_16x16x4f64).  K advances by BK per
// stage (32 for FP32, 16 for FP64).  Global loads are 16-byte vectors along
// each operand's contiguous dimension; an operand is kept in LDS in the same
// orientation as in memory ("ok": outer index o = m or n rows, k contiguous;
// "ko": k rows, o contiguous), so staging is a straight vector copy.  LDS is
// double buffered: the next stage's loads are in flight during the current
// stage's MFMAs and land in the other buffer, one barrier per stage.
//
// MFMA k mapping: in the 16-k chunk kk of a stage, MFMA step t takes
// k = 16 kk + 4 g + t in lane group g, for both operands (mfma.hpp).
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
    // split K: workgroups of split q take k in [q kc, (q + 1) kc) and write
    // C + q cstride (beta must be 0); splits = 1 is the plain product
    int splits = 1;
    int kc = 0;
    int64_t cstride = 0;
    // triangular operands: bit 0 = op(A) is zero left of the diagonal (row i
    // has no k < i), bit 1 = op(B) is zero above it (column j has no k < j);
    // each output tile then starts its K range at its first row / column
    int tri = 0;
};

constexpr int GT_M = 128, GT_N = 128;
constexpr int G_THREADS = 256;
template <class T> constexpr int G_BK = sizeof(T) == 4 ? 32 : 16;
template <class T> constexpr int G_PAD = 16 / (int)sizeof(T);          // 16 bytes per LDS row

// LDS elements of one operand buffer in either orientation
template <class T, bool KC> constexpr int g_lds_elems()
{
    return KC ? GT_M * (G_BK<T> + G_PAD<T>) : G_BK<T> * (GT_M + G_PAD<T>);
}
template <class T> constexpr size_t gemm_lds_bytes()
{
    constexpr int a = g_lds_elems<T, true>() > g_lds_elems<T, false>() ? g_lds_elems<T, true>()
                                                                       : g_lds_elems<T, false>();
    return (size_t)4 * a * sizeof(T);          // 2 operands x 2 buffers
}

// One operand: outer extent O (M or N), K, source pointer / leading dimension,
// KC = k contiguous in memory.  Staging registers hold NV vectors of VEC
// source elements per lane.
template <class T, class TS, bool KC>
struct GOperand {
    static constexpr int BK = G_BK<T>;
    static constexpr int VEC = 16 / (int)sizeof(TS);
    static constexpr int NV = GT_M * BK / VEC / G_THREADS;
    static constexpr int LDR = KC ? BK + G_PAD<T> : GT_M + G_PAD<T>;   // LDS row length
    static_assert(NV >= 1 && (GT_M * BK) % (VEC * G_THREADS) == 0, "tile / vector split");

    const TS* src;
    int64_t ld;
    int O, K, o0;
    bool vec_ok;       // base and leading dimension allow aligned 16-byte loads
    TS r[NV][VEC];

    __device__ void load(int k0, int tid)
    {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int e = tid + G_THREADS * v;
            int o, k;
            if constexpr (KC) { o = e / (BK / VEC); k = (e % (BK / VEC)) * VEC; }
            else { k = e / (GT_M / VEC); o = (e % (GT_M / VEC)) * VEC; }
            const int go = o0 + o, gk = k0 + k;
            const bool full = KC ? (go < O && gk + VEC <= K) : (gk < K && go + VEC <= O);
            if (vec_ok && full) {
                const TS* q = KC ? src + (int64_t)go * ld + gk : src + (int64_t)gk * ld + go;
                typedef TS vt16 __attribute__((ext_vector_type(VEC)));
                const vt16 w = *reinterpret_cast<const vt16*>(q);
#pragma unroll
                for (int c = 0; c < VEC; ++c) r[v][c] = w[c];
            } else {
#pragma unroll
                for (int c = 0; c < VEC; ++c) {
                    const int oo = KC ? go : go + c, kk = KC ? gk + c : gk;
                    r[v][c] = (oo < O && kk < K) ? src[KC ? (int64_t)oo * ld + kk
                                                         : (int64_t)kk * ld + oo]
                                                 : TS(0);
                }
            }
        }
    }

    __device__ void store(T* L, int tid) const
    {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int e = tid + G_THREADS * v;
            int o, k;
            if constexpr (KC) { o = e / (BK / VEC); k = (e % (BK / VEC)) * VEC; }
            else { k = e / (GT_M / VEC); o = (e % (GT_M / VEC)) * VEC; }
            T* q = KC ? L + o * LDR + k : L + k * LDR + o;
#pragma unroll
            for (int c = 0; c < VEC; ++c) q[c] = (T)r[v][c];
        }
    }

    // MFMA operand of outer index `row`, k = 16 kk + 4 g + t, t = 0..3
    static __device__ void frag(const T* L, int row, int kk, int g, T (&f)[4])
    {
        const int k = 16 * kk + 4 * g;
        if constexpr (KC) {
            const T* q = L + row * LDR + k;
#pragma unroll
            for (int t = 0; t < 4; ++t) f[t] = q[t];
        } else {
#pragma unroll
            for (int t = 0; t < 4; ++t) f[t] = L[(k + t) * LDR + row];
        }
    }
};

// Tile and K split of a workgroup: XCD-grouped (the hardware deals
// workgroups round-robin over 8 XCDs; consecutive indices on one XCD get
// neighbouring tiles), and for uplo only tiles that meet the upper triangle.
__device__ __forceinline__ void gemm_tile(int bid, int nblocks, int ntiles, int tiles_n, int uplo,
                                          int& bm, int& bn, int& split)
{
    int l = bid;
    if (nblocks % 8 == 0) l = (bid % 8) * (nblocks / 8) + bid / 8;
    split = l / ntiles;
    l -= split * ntiles;
    if (!uplo) {
        bm = l / tiles_n;
        bn = l % tiles_n;
        return;
    }
    int r = 0, rem = l;
    while (rem >= tiles_n - r) { rem -= tiles_n - r; ++r; }
    bm = r;
    bn = r + rem;
}

// Two workgroups per CU (two waves per SIMD): the LDS of two fits, and the
// FP64 accumulators alone take 128 registers, so the register budget must
// be bounded for the second workgroup to be resident.
template <class T, class TA, class TB, bool AKC, bool BKC>
__global__ void __launch_bounds__(G_THREADS) __attribute__((amdgpu_waves_per_eu(2)))
k_gemm(GemmArgs p)
{
    using Acc = typename mfma_acc<T>::type;
    constexpr int BK = G_BK<T>;
    extern __shared__ __align__(16) unsigned char g_smem[];
    constexpr int LA = g_lds_elems<T, AKC>(), LB = g_lds_elems<T, BKC>();
    T* const La0 = reinterpret_cast<T*>(g_smem);
    T* const Lb0 = La0 + 2 * LA;

    const int tiles_m = (p.M + GT_M - 1) / GT_M, tiles_n = (p.N + GT_N - 1) / GT_N;
    const int ntiles = p.uplo ? tiles_n * (tiles_n + 1) / 2 : tiles_m * tiles_n;
    int bm, bn, split;
    gemm_tile(blockIdx.x, gridDim.x, ntiles, tiles_n, p.uplo, bm, bn, split);
    const int m0 = bm * GT_M, n0 = bn * GT_N;
    int kb = split * p.kc;
    const int ke = min(p.K, kb + p.kc);
    if (p.tri & 1) kb = max(kb, m0);
    if (p.tri & 2) kb = max(kb, n0);
    const int K = max(0, ke - kb);
    const TA* Ap = static_cast<const TA*>(p.A) + (p.transA ? (int64_t)kb * p.lda : kb);
    const TB* Bp = static_cast<const TB*>(p.B) + (p.transB ? kb : (int64_t)kb * p.ldb);

    const int tid = threadIdx.x;
    const int wave = tid / 64, lane = tid % 64;
    const int wm = wave / 2, wn = wave % 2;
    const int lg = lane / 16, lc = lane % 16;

    using OA = GOperand<T, TA, AKC>;
    using OB = GOperand<T, TB, BKC>;
    OA opa;
    opa.src = Ap;
    opa.ld = p.lda; opa.O = p.M; opa.K = K; opa.o0 = m0;
    opa.vec_ok = ((uintptr_t)Ap % 16 == 0) && (p.lda % OA::VEC == 0);
    OB opb;
    opb.src = Bp;
    opb.ld = p.ldb; opb.O = p.N; opb.K = K; opb.o0 = n0;
    opb.vec_ok = ((uintptr_t)Bp % 16 == 0) && (p.ldb % OB::VEC == 0);

    Acc acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = Acc{0, 0, 0, 0};

    const int nk = (K + BK - 1) / BK;
    if (nk > 0) {
        opa.load(0, tid);
        opb.load(0, tid);
        opa.store(La0, tid);
        opb.store(Lb0, tid);
    }
    __syncthreads();
    for (int s = 0; s < nk; ++s) {
        const int cur = s & 1;
        const T* La = La0 + cur * LA;
        const T* Lb = Lb0 + cur * LB;
        if (s + 1 < nk) {
            opa.load((s + 1) * BK, tid);
            opb.load((s + 1) * BK, tid);
        }
#pragma unroll
        for (int kk = 0; kk < BK / 16; ++kk) {
            T af[4][4], bf[4][4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                OA::frag(La, wm * 64 + i * 16 + lc, kk, lg, af[i]);
                OB::frag(Lb, wn * 64 + i * 16 + lc, kk, lg, bf[i]);
            }
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[i][j] = mfma16(af[i][t], bf[j][t], acc[i][j]);
        }
        if (s + 1 < nk) {
            opa.store(La0 + (cur ^ 1) * LA, tid);
            opb.store(Lb0 + (cur ^ 1) * LB, tid);
        }
        __syncthreads();
    }

    // epilogue: lane holds D[row(lg, v)][lc] of block (i, j)
    T* C = static_cast<T*>(p.C) + split * p.cstride;
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

template <class T, class TA, class TB, bool AKC, bool BKC>
static hipError_t gemm_launch_t(const GemmArgs& p, int blocks, hipStream_t s)
{
    auto kern = k_gemm<T, TA, TB, AKC, BKC>;
    constexpr size_t smem = gemm_lds_bytes<T>();
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)kern,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(G_THREADS), smem, s, p);
    return hipGetLastError();
}

template <class T, class TA, class TB>
static hipError_t gemm_launch(const GemmArgs& p, hipStream_t s)
{
    if (p.M <= 0 || p.N <= 0) return hipSuccess;
    const int tm = (p.M + GT_M - 1) / GT_M, tn = (p.N + GT_N - 1) / GT_N;
    if (p.uplo && tm != tn) return hipErrorInvalidValue;
    if (p.splits < 1 || (p.splits > 1 && (p.kc <= 0 || p.beta != 0.0))) return hipErrorInvalidValue;
    GemmArgs q = p;
    if (q.splits == 1) q.kc = q.K;
    const int blocks = (p.uplo ? tn * (tn + 1) / 2 : tm * tn) * q.splits;
    // A is k-contiguous when not transposed; B is k-contiguous when transposed
    if (!q.transA && q.transB) return gemm_launch_t<T, TA, TB, true, true>(q, blocks, s);
    if (!q.transA && !q.transB) return gemm_launch_t<T, TA, TB, true, false>(q, blocks, s);
    if (q.transA && q.transB) return gemm_launch_t<T, TA, TB, false, true>(q, blocks, s);
    return gemm_launch_t<T, TA, TB, false, false>(q, blocks, s);
}

}  // namespace ci
