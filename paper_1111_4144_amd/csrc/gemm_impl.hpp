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
// Tiling: a workgroup of WM x WN waves owns a (64 WM) x (64 WN) tile of C
// (128 x 128 with 2 x 2 waves; 256 x 128 with 4 x 2 for long products, a
// quarter fewer operand bytes per flop); each wave a 64 x 64
// sub-tile made of 4 x 4 MFMA blocks of 16 x 16
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

// the small tile: 2 x 2 waves, 128 x 128
constexpr int GT_M = 128, GT_N = 128;
template <class T> constexpr int G_BK = sizeof(T) == 4 ? 32 : 16;
template <class T> constexpr int G_PAD = 16 / (int)sizeof(T);          // 16 bytes per LDS row

// LDS elements of one operand buffer of outer extent TO in either orientation
template <class T, bool KC, int TO> constexpr int g_lds_elems()
{
    return KC ? TO * (G_BK<T> + G_PAD<T>) : G_BK<T> * (TO + G_PAD<T>);
}
template <class T, int TO> constexpr int g_lds_max()
{
    return g_lds_elems<T, true, TO>() > g_lds_elems<T, false, TO>() ? g_lds_elems<T, true, TO>()
                                                                     : g_lds_elems<T, false, TO>();
}
// LDS of a (64 WM) x (64 WN) tile: 2 operands x 2 buffers
template <class T, int WM, int WN> constexpr size_t gemm_lds_bytes()
{
    return (size_t)2 * (g_lds_max<T, 64 * WM>() + g_lds_max<T, 64 * WN>()) * sizeof(T);
}

// One operand: outer extent O (M or N), K, source pointer / leading dimension,
// KC = k contiguous in memory, TO the tile's outer extent, NT the workgroup's
// lanes.  Staging registers hold NV vectors of VEC source elements per lane.
template <class T, class TS, bool KC, int TO, int NT>
struct GOperand {
    static constexpr int BK = G_BK<T>;
    static constexpr int VEC = 16 / (int)sizeof(TS);
    static constexpr int NV = TO * BK / VEC / NT;
    static constexpr int LDR = KC ? BK + G_PAD<T> : TO + G_PAD<T>;   // LDS row length
    static_assert(NV >= 1 && (TO * BK) % (VEC * NT) == 0, "tile / vector split");

    const TS* src;
    int64_t ld;
    int O, K, o0;
    bool vec_ok;       // base and leading dimension allow aligned 16-byte loads
    TS r[NV][VEC];

    __device__ void load(int k0, int tid)
    {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int e = tid + NT * v;
            int o, k;
            if constexpr (KC) { o = e / (BK / VEC); k = (e % (BK / VEC)) * VEC; }
            else { k = e / (TO / VEC); o = (e % (TO / VEC)) * VEC; }
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
            const int e = tid + NT * v;
            int o, k;
            if constexpr (KC) { o = e / (BK / VEC); k = (e % (BK / VEC)) * VEC; }
            else { k = e / (TO / VEC); o = (e % (TO / VEC)) * VEC; }
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

// Tiles of a TM x TN tiling that meet the upper triangle (column >= row):
// row tile r starts at column tile (r TM) / TN.
__device__ __host__ __forceinline__ int gemm_upper_tiles(int tiles_m, int tiles_n, int TM, int TN)
{
    int t = 0;
    for (int r = 0; r < tiles_m; ++r) {
        const int c0 = r * TM / TN;
        if (c0 < tiles_n) t += tiles_n - c0;
    }
    return t;
}

// Tile and K split of a workgroup: XCD-grouped (the hardware deals
// workgroups round-robin over 8 XCDs; consecutive indices on one XCD get
// neighbouring tiles), and for uplo only tiles that meet the upper triangle.
__device__ __forceinline__ void gemm_tile(int bid, int nblocks, int ntiles, int tiles_n, int uplo,
                                          int TM, int TN, int& bm, int& bn, int& split)
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
    while (rem >= tiles_n - r * TM / TN) { rem -= tiles_n - r * TM / TN; ++r; }
    bm = r;
    bn = r * TM / TN + rem;
}

// Occupancy: the 2 x 2 tile runs two workgroups per CU (two waves per SIMD:
// the LDS of two fits, and the FP64 accumulators alone take 128 registers,
// so the register budget is bounded for the second workgroup to be
// resident); the 4 x 2 tile one workgroup of eight waves (its LDS).
template <class T, class TA, class TB, bool AKC, bool BKC, int WM, int WN>
__global__ void __launch_bounds__(64 * WM * WN) __attribute__((amdgpu_waves_per_eu(2)))
k_gemm(GemmArgs p)
{
    using Acc = typename mfma_acc<T>::type;
    constexpr int BK = G_BK<T>;
    constexpr int TM = 64 * WM, TN = 64 * WN, NT = 64 * WM * WN;
    extern __shared__ __align__(16) unsigned char g_smem[];
    constexpr int LA = g_lds_elems<T, AKC, TM>(), LB = g_lds_elems<T, BKC, TN>();
    T* const La0 = reinterpret_cast<T*>(g_smem);
    T* const Lb0 = La0 + 2 * LA;

    const int tiles_m = (p.M + TM - 1) / TM, tiles_n = (p.N + TN - 1) / TN;
    const int ntiles = p.uplo ? gemm_upper_tiles(tiles_m, tiles_n, TM, TN) : tiles_m * tiles_n;
    int bm, bn, split;
    gemm_tile(blockIdx.x, gridDim.x, ntiles, tiles_n, p.uplo, TM, TN, bm, bn, split);
    const int m0 = bm * TM, n0 = bn * TN;
    int kb = split * p.kc;
    const int ke = min(p.K, kb + p.kc);
    if (p.tri & 1) kb = max(kb, m0);
    if (p.tri & 2) kb = max(kb, n0);
    const int K = max(0, ke - kb);
    const TA* Ap = static_cast<const TA*>(p.A) + (p.transA ? (int64_t)kb * p.lda : kb);
    const TB* Bp = static_cast<const TB*>(p.B) + (p.transB ? kb : (int64_t)kb * p.ldb);

    const int tid = threadIdx.x;
    const int wave = tid / 64, lane = tid % 64;
    const int wm = wave / WN, wn = wave % WN;
    const int lg = lane / 16, lc = lane % 16;

    using OA = GOperand<T, TA, AKC, TM, NT>;
    using OB = GOperand<T, TB, BKC, TN, NT>;
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

template <class T, class TA, class TB, bool AKC, bool BKC, int WM, int WN>
static hipError_t gemm_launch_t(const GemmArgs& p, hipStream_t s)
{
    auto kern = k_gemm<T, TA, TB, AKC, BKC, WM, WN>;
    constexpr size_t smem = gemm_lds_bytes<T, WM, WN>();
    constexpr int TM = 64 * WM, TN = 64 * WN;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)kern,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
        if (e != hipSuccess) return e;
        attr = true;
    }
    const int tm = (p.M + TM - 1) / TM, tn = (p.N + TN - 1) / TN;
    const int blocks = (p.uplo ? gemm_upper_tiles(tm, tn, TM, TN) : tm * tn) * p.splits;
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(64 * WM * WN), smem, s, p);
    return hipGetLastError();
}

// Whether a product takes the 256 x 128 tile: a plain (not split) product
// with at least one such tile per compute unit and a long K range, when the
// large-order configuration asks for it (set per thread; off by default:
// measured at N = 8192 it gained 4% on the refinement's FP64 residual and
// lost 3-7% on X = M M^T).
static thread_local bool g_gemm_big = false;
inline bool gemm_big_tile(const GemmArgs& p)
{
    if (!g_gemm_big || p.splits > 1 || p.K < 512) return false;
    const int tm = (p.M + 255) / 256, tn = (p.N + 127) / 128;
    const int tiles = p.uplo ? gemm_upper_tiles(tm, tn, 256, 128) : tm * tn;
    return tiles >= 256;
}

template <class T, class TA, class TB, int WM, int WN>
static hipError_t gemm_launch_w(const GemmArgs& q, hipStream_t s)
{
    // A is k-contiguous when not transposed; B is k-contiguous when transposed
    if (!q.transA && q.transB) return gemm_launch_t<T, TA, TB, true, true, WM, WN>(q, s);
    if (!q.transA && !q.transB) return gemm_launch_t<T, TA, TB, true, false, WM, WN>(q, s);
    if (q.transA && q.transB) return gemm_launch_t<T, TA, TB, false, true, WM, WN>(q, s);
    return gemm_launch_t<T, TA, TB, false, false, WM, WN>(q, s);
}

template <class T, class TA, class TB>
static hipError_t gemm_launch(const GemmArgs& p, hipStream_t s)
{
    if (p.M <= 0 || p.N <= 0) return hipSuccess;
    if (p.uplo && p.M != p.N) return hipErrorInvalidValue;
    if (p.splits < 1 || (p.splits > 1 && (p.kc <= 0 || p.beta != 0.0))) return hipErrorInvalidValue;
    GemmArgs q = p;
    if (q.splits == 1) q.kc = q.K;
    if (gemm_big_tile(q)) return gemm_launch_w<T, TA, TB, 4, 2>(q, s);
    return gemm_launch_w<T, TA, TB, 2, 2>(q, s);
}

}  // namespace ci
