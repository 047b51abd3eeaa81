// large.hip -- X = A^{-1} for one real symmetric positive-definite matrix of
// large order, blocked with MFMA GEMM tiles.
//
// Factorisation (Section II eqs. 3-4, right-looking, panels of nb rows):
//   for each diagonal block I:
//     R_II = chol(A_II) and R_II^{-1}          one workgroup, LDS resident
//     R_I,>I = R_II^{-T} A_I,>I                 GEMM with the explicit inverse
//     A_>I,>I -= R_I,>I^T R_I,>I                 upper-only GEMM (SYRK)
// Inversion, default: M = R^{-1} by block columns (zero blocks skipped), then
// the upper half of X = M M^T in one product (lg_trtri, lg_lauum).
// Inversion, alternative (Section IV in block form, block rows bottom-up;
// CHOLINV_LARGE_INVERSE=blocked_iv).  Row block I of
// R X = B, with B lower triangular and its upper triangle S = diag(1/r_ii)
// known, gives for J > I:  X_I,J = -R_II^{-1} (R_I,>I X-hat_>I,J) (B_I,J = 0),
// and for the diagonal block the scalar recurrence of the small kernels with
// the extra term W = R_I,>I X-hat_>I,I = R_I,>I X_I,>I^T:
//     x_ij = s_i (delta_ij s_i - w_ij - sum_{k>i, k in I} r_ik xh_kj).
// Only the upper half of X is computed; the lower half is the mirror.
//
// Mixed precision: FP32 data and MFMA products; the diagonal pivots keep an
// FP64 accumulator d_j = a_jj - sum_k r_kj^2 (updated per panel from the FP32
// R entries, whose squares are exact in FP64); then Newton-Schulz steps
// X <- X + X (I - A X) with the residual I - A X as an FP64 MFMA GEMM on the
// exact FP32 inputs and the update as an FP32 GEMM.
#include <algorithm>
#include <cstdlib>
#include <cstring>

#include "ci_large.hpp"
#include "ci_launch.hpp"
#include "ci_types.hpp"
#include "gemm_impl.hpp"
#include "leaf_impl.hpp"

namespace ci {

template <class T> constexpr int LG_NB = sizeof(T) == 4 ? 128 : 64;   // panel width
template <class T> constexpr int LG_P = 16 / (int)sizeof(T);
template <class T> constexpr int LG_LD = LG_NB<T> + LG_P<T>;
constexpr int LG_SPLIT_MAX = 8;

// sum over packets p in [p0, p1) of sum_c a_p[c] b_p[c]; fa / fb fetch the P
// entries of packet p.  Four packets are fetched before their products so
// that several LDS loads are in flight; P independent partial sums.
template <class T, class FA, class FB>
__device__ __forceinline__ T lg_dot(int p0, int p1, FA fa, FB fb)
{
    constexpr int P = LG_P<T>;
    T part[P];
#pragma unroll
    for (int c = 0; c < P; ++c) part[c] = T(0);
    int p = p0;
    for (; p + 4 <= p1; p += 4) {
        T a[4][P], b[4][P];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            fa(p + q, a[q]);
            fb(p + q, b[q]);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int c = 0; c < P; ++c) part[c] += a[q][c] * b[q][c];
    }
    for (; p < p1; ++p) {
        T a[P], b[P];
        fa(p, a);
        fb(p, b);
#pragma unroll
        for (int c = 0; c < P; ++c) part[c] += a[c] * b[c];
    }
    T r = part[0];
#pragma unroll
    for (int c = 1; c < P; ++c) r += part[c];
    return r;
}

// contiguous packet of P entries from LDS (16 bytes, aligned)
template <class T>
__device__ __forceinline__ void lg_ldv(const T* q, T (&v)[LG_P<T>])
{
    typedef T v16 __attribute__((ext_vector_type(LG_P<T>)));
    const v16 w = *reinterpret_cast<const v16*>(q);
#pragma unroll
    for (int c = 0; c < LG_P<T>; ++c) v[c] = w[c];
}

// ---- diagonal block: Cholesky (Crout, FP64 pivots when mixed) + R^{-1} --------
// LG_TPC adjacent lanes share column j: lane h of the column takes the
// packets p = h, h + LG_TPC, ... of every inner product, and the partial sums
// are combined with lane shuffles, so the serial steps are spread over
// LG_TPC times more waves.
constexpr int LG_TPC = 4;
template <class T> constexpr int LG_SB = 32;          // sub-block of the diagonal factor

template <class T>
__device__ __forceinline__ T lg_colsum(T v)
{
    return quad_sum<LG_TPC>(v);
}

// LDS of the diagonal factor kernel: R and Y (NB x LD each), 1/r_ii and r_ii,
// then the FP64 pivot accumulators of the panel.
template <class T> constexpr size_t lg_diag_dl_offset()
{
    return ((size_t)(2 * LG_NB<T> * LG_LD<T> + 2 * LG_NB<T>) * sizeof(T) + 15) / 16 * 16;
}
template <class T> constexpr size_t lg_diag_smem() { return lg_diag_dl_offset<T>() + LG_NB<T> * 8; }

template <class T, int MIXED>
__global__ void __launch_bounds__(LG_NB<T> * LG_TPC)
k_lg_diag_factor(T* __restrict__ W, int64_t ldw, int r0, int nl, const double* __restrict__ dacc,
                 T* __restrict__ rinv, int32_t* __restrict__ info)
{
    constexpr int NB = LG_NB<T>, LD = LG_LD<T>, P = LG_P<T>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* Rm = reinterpret_cast<T*>(smem_raw);
    T* Ym = Rm + NB * LD;
    T* sv = Ym + NB * LD;                          // 1/r_ii
    T* rd = sv + NB;                               // r_ii
    double* dl = reinterpret_cast<double*>(smem_raw + lg_diag_dl_offset<T>());   // FP64 pivots
    const int j = threadIdx.x / LG_TPC, h = threadIdx.x % LG_TPC;
    T* Wb = W + (int64_t)r0 * ldw + r0;
    for (int k = h; k < NB; k += LG_TPC) {
        T v = (k == j) ? T(1) : T(0);
        if (j < nl && k < nl && k <= j) v = Wb[(int64_t)k * ldw + j];
        Rm[j * LD + k] = (k <= j) ? v : T(0);
        Ym[j * LD + k] = T(0);
    }
    if (MIXED && h == 0) dl[j] = (j < nl) ? dacc[r0 + j] : 1.0;
    __syncthreads();
    int fail = 0;
    // Sub-blocks of LG_SB columns: rows of a sub-block by the Crout recurrence
    // over the sub-block's own earlier rows only, then the finished sub-block
    // applied to the rest of the block as one rank-LG_SB update (parallel over
    // all lanes), with the FP64 pivot accumulators updated the same way.
    // Every lane forms the pivot of row i itself (column i's squares ride
    // along in the same packet loop), so one barrier per row suffices; row
    // i's diagonal goes to rd[] and into R only after the loop (column i is
    // read by every lane during step i).
    constexpr int SB = LG_SB<T>;
    for (int b0 = 0; b0 < NB; b0 += SB) {
        for (int i = b0; i < b0 + SB; ++i) {
            const T* ci = Rm + i * LD;
            const T* cj = Rm + j * LD;
            const int p0 = b0 / P, full = i / P;
            T dot = T(0), sii = T(0);
            double s64 = 0.0;
            for (int p = p0 + h; p < full; p += LG_TPC) {
                T u[P], w[P];
                lg_ldv(ci + p * P, u);
                lg_ldv(cj + p * P, w);
#pragma unroll
                for (int c = 0; c < P; ++c) {
                    dot += u[c] * w[c];
                    if (MIXED) s64 = fma((double)u[c], (double)u[c], s64);
                    else sii += u[c] * u[c];
                }
            }
            if (h == 0) {
                for (int k = full * P; k < i; ++k) {
                    const T u = ci[k];
                    dot += u * cj[k];
                    if (MIXED) s64 = fma((double)u, (double)u, s64);
                    else sii += u * u;
                }
            }
            dot = lg_colsum(dot);
            const T acc = cj[i] - dot;
            double piv;
            if (MIXED) piv = dl[i] - lg_colsum(s64);
            else piv = (double)(ci[i] - lg_colsum(sii));
            const bool ok = piv > 0.0 && piv < __builtin_inf();
            if (!ok && !fail && i < nl) fail = i + 1;
            T rii, si;
            if constexpr (sizeof(T) == 4) {
                double r, y;
                sqrt_rsqrt_est(piv, r, y);       // FP32 results
                rii = (T)r;
                si = (T)y;
            } else {
                const double r = sqrt(piv);
                rii = (T)r;
                si = (T)(1.0 / r);
            }
            if (h == 0) {
                if (j > i) Rm[j * LD + i] = acc * si;
                if (j == i) {
                    sv[i] = si;
                    rd[i] = rii;
                }
            }
            __syncthreads();
        }
        const int b1 = b0 + SB;
        if (b1 < NB && j >= b1) {
            // a_kj -= sum_{m in sub-block} r_mk r_mj, b1 <= k <= j (this lane's rows)
            const T* cj = Rm + j * LD;
            T wj[SB];
#pragma unroll
            for (int m = 0; m < SB; m += P) lg_ldv(cj + b0 + m, *reinterpret_cast<T(*)[P]>(wj + m));
            for (int k = b1 + h; k <= j; k += LG_TPC) {
                const T* ck = Rm + k * LD + b0;
                T part = T(0);
#pragma unroll
                for (int m = 0; m < SB; m += P) {
                    T u[P];
                    lg_ldv(ck + m, u);
#pragma unroll
                    for (int c = 0; c < P; ++c) part += u[c] * wj[m + c];
                }
                Rm[j * LD + k] -= part;
            }
            if (MIXED && h == 0) {
                double q = 0.0;
#pragma unroll
                for (int m = 0; m < SB; ++m) q = fma((double)wj[m], (double)wj[m], q);
                dl[j] -= q;
            }
        }
        __syncthreads();
    }
    if (h == 0) Rm[j * LD + j] = rd[j];
    __syncthreads();
    if (j < nl)
        for (int k = h; k <= j; k += LG_TPC) Wb[(int64_t)k * ldw + j] = Rm[j * LD + k];
    // Y = R^{-1} by sub-blocks.  Diagonal sub-blocks first, all at once: in
    // column j, y_jj = 1/r_jj and y_ij = -(1/r_ii) sum_{k=i+1..j} r_ik y_kj for
    // i down to the sub-block's first row (entries not computed yet are zero,
    // and R is zero below its diagonal, so the packets may start below i+1;
    // the lanes of column j are adjacent in one wave, and a wavefront-scope
    // fence orders lane 0's write of y_ij before every lane's later reads).  Then block rows bottom-up:
    // Y_{I,>I} = -Y_II (R_{I,>I} Y_{>I,>I}), each a parallel stage.
    if (h == 0) Ym[j * LD + j] = sv[j];
    {
        const int bj = (j / SB) * SB;
        for (int i = j - 1; i >= bj; --i) {
            T dot = T(0);
            for (int p = (i + 1) / P + h; p <= j / P; p += LG_TPC) {
                T w[P];
                lg_ldv(Ym + j * LD + p * P, w);
#pragma unroll
                for (int c = 0; c < P; ++c) dot += Rm[(p * P + c) * LD + i] * w[c];
            }
            dot = lg_colsum(dot);
            if (h == 0) Ym[j * LD + i] = -sv[i] * dot;
            // the next row's sums read y_ij: lane 0's write precedes them (the
            // lanes of a column are in one wave)
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
    __syncthreads();
    constexpr int NT = NB * LG_TPC;
    constexpr int PER = (SB * (NB - SB) + NT - 1) / NT;
    for (int a0 = NB - 2 * SB; a0 >= 0; a0 -= SB) {
        const int b1 = a0 + SB, cnt = SB * (NB - b1);
        // t_ij = sum_{k=b1..j} r_ik y_kj into the (still zero) Y_{I,>I} block
        for (int e = threadIdx.x; e < cnt; e += NT) {
            const int i = a0 + e % SB, jj = b1 + e / SB;
            T t = T(0);
            for (int k = b1; k <= jj; ++k) t += Rm[k * LD + i] * Ym[jj * LD + k];
            Ym[jj * LD + i] = t;
        }
        __syncthreads();
        // y_ij = -sum_{m=i..b1-1} (Y_II)_im t_mj
        T val[PER];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = threadIdx.x + q * NT;
            val[q] = T(0);
            if (e < cnt) {
                const int i = a0 + e % SB, jj = b1 + e / SB;
                T acc = T(0);
                for (int m = i; m < b1; ++m) acc += Ym[m * LD + i] * Ym[jj * LD + m];
                val[q] = -acc;
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = threadIdx.x + q * NT;
            if (e < cnt) Ym[(b1 + e / SB) * LD + a0 + e % SB] = val[q];
        }
        __syncthreads();
    }
    for (int i = h; i < NB; i += LG_TPC) rinv[(int64_t)i * NB + j] = (i <= j) ? Ym[j * LD + i] : T(0);
    if (threadIdx.x == 0 && fail && info && info[0] == 0) info[0] = r0 + fail;
}

// ---- diagonal block, sub-blocked on the matrix cores (leaf_impl.hpp) -------------
template <class T> constexpr int LF_LD = lf_ld<T, LG_NB<T>>();
template <class T> constexpr size_t lf_smem()
{
    return (size_t)2 * LG_NB<T> * LF_LD<T> * sizeof(T) + LG_NB<T> * sizeof(double);
}

template <class T, int MIXED>
__global__ void __launch_bounds__(LF_THREADS)
k_lg_leaf(T* __restrict__ W, int64_t ldw, int r0, int nl, const double* __restrict__ dacc,
          T* __restrict__ rinv, int32_t* __restrict__ info)
{
    constexpr int NB = LG_NB<T>, LD = LF_LD<T>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* Rm = reinterpret_cast<T*>(smem_raw);              // R, row major, upper
    T* Ym = Rm + NB * LD;                                // R^{-1}, row major, upper
    double* dl = reinterpret_cast<double*>(Ym + NB * LD); // FP64 pivot accumulators
    const int tid = threadIdx.x;
    T* Wb = W + (int64_t)r0 * ldw + r0;
    // the block's upper triangle (identity beyond nl); Y starts at zero.  All
    // of a lane's loads are issued before its first LDS store, so the global
    // latency is paid once, not once per element.
    {
        constexpr int PER = NB * NB / LF_THREADS;
        T v[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = tid + LF_THREADS * u, k = e / NB, j = e % NB;
            v[u] = (k == j) ? T(1) : T(0);
            if (j < nl && k < nl && k <= j) v[u] = Wb[(int64_t)k * ldw + j];
        }
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = tid + LF_THREADS * u, k = e / NB, j = e % NB;
            Rm[k * LD + j] = (k <= j) ? v[u] : T(0);
            Ym[k * LD + j] = T(0);
        }
    }
    if (MIXED)
        for (int j = tid; j < NB; j += LF_THREADS) dl[j] = (j < nl) ? dacc[r0 + j] : 1.0;
    __syncthreads();
    const int fail = lf_factor_inverse<T, NB, MIXED>(Rm, Ym, dl, nl);
    // ---- R back to W (upper triangle of the block), R^{-1} to rinv
    for (int e = tid; e < NB * NB; e += LF_THREADS) {
        const int k = e / NB, j = e % NB;
        if (k <= j && j < nl) Wb[(int64_t)k * ldw + j] = Rm[k * LD + j];
        rinv[(int64_t)k * NB + j] = (k <= j) ? Ym[k * LD + j] : T(0);
    }
    if (tid == 0 && fail && info && info[0] == 0) info[0] = r0 + fail;
}

// ---- FP64 pivot accumulators: d_j -= sum_{k in panel} r_kj^2, j >= c0 ----------
// 64-lane blocks over the columns; rows in batches of 8 independent loads.
template <class T>
__global__ void __launch_bounds__(64)
k_lg_dacc(const T* __restrict__ W, int64_t ldw, int r0, int nl, int c0, int n,
          double* __restrict__ dacc)
{
    const int j = c0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const T* col = W + (int64_t)r0 * ldw + j;
    double s = dacc[j];
    int k = 0;
    for (; k + 8 <= nl; k += 8) {
        T v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = col[(int64_t)(k + q) * ldw];
#pragma unroll
        for (int q = 0; q < 8; ++q) s = fma(-(double)v[q], (double)v[q], s);
    }
    for (; k < nl; ++k) {
        const double v = (double)col[(int64_t)k * ldw];
        s = fma(-v, v, s);
    }
    dacc[j] = s;
}

template <class TI>
__global__ void k_lg_dacc_init(const TI* __restrict__ a, int64_t lda, int n, double* __restrict__ dacc)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) dacc[j] = (double)a[(int64_t)j * lda + j];
}

// ---- diagonal block of X: the Section IV recurrence with the W term ------------
template <class T>
__global__ void __launch_bounds__(LG_NB<T>)
k_lg_diag_inverse(const T* __restrict__ W, int64_t ldw, int r0, int nl,
                  const T* __restrict__ wblk, int has_w, T* __restrict__ X, int64_t ldx)
{
    constexpr int NB = LG_NB<T>, LD = LG_LD<T>, P = LG_P<T>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* Rm = reinterpret_cast<T*>(smem_raw);
    T* Xm = Rm + NB * LD;
    T* sv = Xm + NB * LD;
    const int j = threadIdx.x;
    const T* Wb = W + (int64_t)r0 * ldw + r0;
    // R row major here (Rm[k * LD + j] = r_kj): the dot products below run
    // along rows of R and columns of X, both contiguous
    for (int k = 0; k < NB; ++k) {
        T v = T(0);
        if (j < nl && k < nl && k <= j) v = Wb[(int64_t)k * ldw + j];
        if (j >= nl && k == j) v = T(1);
        Rm[k * LD + j] = v;
        Xm[j * LD + k] = T(0);
    }
    __syncthreads();
    sv[j] = T(1) / Rm[j * LD + j];
    __syncthreads();
    const int pend = (nl + P - 1) / P;
    // w_ij of this column, fetched one step ahead so that no global load
    // latency sits inside the serial loop
    T w_next = (has_w && j < nl && nl > 0) ? wblk[(int64_t)(nl - 1) * NB + j] : T(0);
    for (int i = nl - 1; i >= 0; --i) {
        const T si = sv[i];
        const T w_cur = w_next;
        if (has_w && j < nl && i > 0) w_next = wblk[(int64_t)(i - 1) * NB + j];
        if (j > i && j < nl) {
            const T dot = lg_dot<T>((i + 1) / P, pend,
                                    [&](int p, T (&v)[P]) { lg_ldv(Rm + i * LD + p * P, v); },
                                    [&](int p, T (&v)[P]) { lg_ldv(Xm + j * LD + p * P, v); });
            const T xij = si * (-w_cur - dot);
            Xm[j * LD + i] = xij;
            Xm[i * LD + j] = xij;
        }
        __syncthreads();
        if (j == i) {
            const T dot = lg_dot<T>((i + 1) / P, pend,
                                    [&](int p, T (&v)[P]) { lg_ldv(Rm + i * LD + p * P, v); },
                                    [&](int p, T (&v)[P]) { lg_ldv(Xm + i * LD + p * P, v); });
            Xm[i * LD + i] = si * (si - w_cur - dot);
        }
        __syncthreads();
    }
    if (j < nl)
        for (int k = 0; k < nl; ++k) X[(int64_t)(r0 + k) * ldx + r0 + j] = Xm[j * LD + k];
}

// ---- split-K reduction: C = alpha * sum_s P_s (+ beta C) ------------------------
template <class T>
__global__ void k_lg_reduce(const T* __restrict__ part, int splits, int64_t pstride, int m, int n,
                            int64_t ldp, T alpha, T* __restrict__ C, int64_t ldc)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)m * n) return;
    const int i = (int)(e / n), jj = (int)(e % n);
    T s = T(0);
    for (int k = 0; k < splits; ++k) s += part[k * pstride + (int64_t)i * ldp + jj];
    C[(int64_t)i * ldc + jj] = alpha * s;
}

// ---- transposed copy dst[j][i] = src[i][j] (32 x 32 tiles through LDS) ------------
template <class TS, class TD>
__global__ void k_lg_transpose(const TS* __restrict__ src, int64_t lds, TD* __restrict__ dst,
                               int64_t ldd, int rows, int cols)
{
    __shared__ TD t[32][33];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    for (int r = threadIdx.y; r < 32; r += blockDim.y) {
        const int i = by + r, jj = bx + threadIdx.x;
        if (i < rows && jj < cols) t[r][threadIdx.x] = (TD)src[(int64_t)i * lds + jj];
    }
    __syncthreads();
    for (int r = threadIdx.y; r < 32; r += blockDim.y) {
        const int jj = bx + r, i = by + threadIdx.x;
        if (i < rows && jj < cols) dst[(int64_t)jj * ldd + i] = t[threadIdx.x][r];
    }
}

// ---- symmetric matrix from its upper triangle: dst = upper(src) + mirror ---------
template <class TS, class TD>
__global__ void k_lg_symmetrize(const TS* __restrict__ src, int64_t lds, TD* __restrict__ dst,
                                int64_t ldd, int n)
{
    __shared__ TD t[32][33];
    const int bi = blockIdx.y, bj = blockIdx.x;
    if (bj < bi) return;
    const int i0 = bi * 32, j0 = bj * 32;
    for (int r = threadIdx.y; r < 32; r += blockDim.y) {
        const int i = i0 + r, jj = j0 + threadIdx.x;
        TD v = TD(0);
        if (i < n && jj < n && jj >= i) v = (TD)src[(int64_t)i * lds + jj];
        t[r][threadIdx.x] = v;
        if (i < n && jj < n && jj >= i) dst[(int64_t)i * ldd + jj] = v;
    }
    __syncthreads();
    // mirror: dst[jj][i] = upper value (i < jj)
    for (int r = threadIdx.y; r < 32; r += blockDim.y) {
        const int jj = j0 + r, i = i0 + threadIdx.x;
        if (i < n && jj < n && jj > i) dst[(int64_t)jj * ldd + i] = t[threadIdx.x][r];
    }
}

// upper_only: 0 whole matrix, 1 upper triangle, 2 upper triangle and zeros below
template <class TS, class TD>
__global__ void k_lg_copy(const TS* __restrict__ src, int64_t lds, TD* __restrict__ dst, int64_t ldd,
                          int rows, int cols, int upper_only)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)rows * cols) return;
    const int i = (int)(e / cols), jj = (int)(e % cols);
    if (upper_only && jj < i) {
        if (upper_only == 2) dst[(int64_t)i * ldd + jj] = TD(0);
        return;
    }
    dst[(int64_t)i * ldd + jj] = (TD)src[(int64_t)i * lds + jj];
}

template <class T>
__global__ void k_lg_identity(T* __restrict__ e, int64_t lde, int n)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)n * n) return;
    const int i = (int)(k / n), jj = (int)(k % n);
    e[(int64_t)i * lde + jj] = (i == jj) ? T(1) : T(0);
}

template <class T>
__global__ void k_lg_nan_if(const int32_t* __restrict__ info, T* __restrict__ x, int64_t ldx, int n)
{
    if (!info || info[0] == 0) return;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)n * n) return;
    x[(k / n) * ldx + (k % n)] = (T)__builtin_nan("");
}

// ---- host orchestration ---------------------------------------------------------
static unsigned blocks_for(int64_t count, int t = 256) { return (unsigned)((count + t - 1) / t); }

template <class T>
struct LgWork {
    // byte offsets inside the caller's workspace
    size_t wmat, rinv, ctmp, wblk, part, dacc, emat, xtmp, total;
    int64_t part_elems;
    LgWork(int64_t n, int mixed)
    {
        const int nb = LG_NB<T>;
        const int64_t nblk = (n + nb - 1) / nb;
        size_t o = 0;
        auto take = [&](size_t bytes) { size_t r = o; o += (bytes + 255) / 256 * 256; return r; };
        wmat = take((size_t)n * n * sizeof(T));
        rinv = take((size_t)nblk * nb * nb * sizeof(T));
        ctmp = take((size_t)nb * n * sizeof(T));
        wblk = take((size_t)nb * nb * sizeof(T));
        part_elems = (int64_t)LG_SPLIT_MAX * nb * n;
        part = take((size_t)part_elems * sizeof(T));
        dacc = take((size_t)n * sizeof(double));
        emat = mixed ? take((size_t)n * n * sizeof(double)) : 0;
        xtmp = mixed ? take((size_t)n * n * sizeof(T)) : 0;
        total = o;
    }
};

template <class T, class TA, class TB>
static hipError_t gemm(int M, int N, int K, double alpha, const TA* A, int64_t lda, int ta,
                       const TB* B, int64_t ldb, int tb, double beta, T* C, int64_t ldc, int uplo,
                       hipStream_t s, int tri = 0)
{
    GemmArgs g{M, N, K, alpha, beta, A, lda, ta, B, ldb, tb, C, ldc, uplo};
    g.tri = tri;
    return gemm_launch<T, TA, TB>(g, s);
}

// C (m x n) = alpha * A B with K split over partial products so that about
// g_splitk_target workgroups run, each split at least kmin deep, the partials
// within the workspace's capacity `cap` (elements)
// The target workgroup count is the tuned configuration's (512 by default).
static thread_local int g_splitk_target = 512;

template <class T>
static hipError_t gemm_splitk(int M, int N, int K, double alpha, const T* A, int64_t lda, int ta,
                              const T* B, int64_t ldb, int tb, T* C, int64_t ldc, T* part,
                              int64_t cap, hipStream_t s, int tri = 0, int kmin = 64)
{
    const int tiles = ((M + GT_M - 1) / GT_M) * ((N + GT_N - 1) / GT_N);
    int splits = (g_splitk_target + tiles - 1) / tiles;
    splits = std::min<int64_t>(splits, std::max(1, K / kmin));
    splits = (int)std::min<int64_t>(splits, cap / ((int64_t)M * N));
    if (splits <= 1)
        return gemm<T, T, T>(M, N, K, alpha, A, lda, ta, B, ldb, tb, 0.0, C, ldc, 0, s, tri);
    constexpr int BK = G_BK<T>;
    const int kc = ((K + splits - 1) / splits + BK - 1) / BK * BK;   // whole stages
    splits = (K + kc - 1) / kc;            // every split has kc > 0 terms
    const int64_t pstride = (int64_t)M * N;
    GemmArgs g{M, N, K, 1.0, 0.0, A, lda, ta, B, ldb, tb, part, (int64_t)N, 0};
    g.splits = splits;
    g.kc = kc;
    g.cstride = pstride;
    g.tri = tri;
    hipError_t e = gemm_launch<T, T, T>(g, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_lg_reduce<T>, dim3(blocks_for((int64_t)M * N)), dim3(256), 0, s, part,
                       splits, pstride, M, N, (int64_t)N, (T)alpha, C, ldc);
    return hipGetLastError();
}

// Configurations of the large-order path the tuner chooses between:
//   diag    0 = diagonal blocks sub-blocked on MFMA (k_lg_leaf), 1 = the
//           Crout recurrence with one barrier per row (k_lg_diag_factor)
//   inv     0 = blocked triangular inverse + X = M M^T, 1 = the Section IV
//           recurrence in block form
//   splitk  target workgroups of the split-K products
//   big     1 = long unsplit products take the 256 x 128 tile, 0 = 128 x 128 only
struct LgCfg { int diag, inv, splitk, big; };
static const LgCfg LG_CFGS[] = {{0, 0, 512, 0}, {0, 0, 256, 0}, {0, 0, 1024, 0},
                                {1, 0, 512, 0}, {0, 1, 512, 0}, {0, 0, 512, 1}};
constexpr int LG_NCFG = sizeof(LG_CFGS) / sizeof(LG_CFGS[0]);
static thread_local LgCfg g_cfg = LG_CFGS[0];

int large_config_count() { return LG_NCFG; }
static int lg_diag_engine() { return g_cfg.diag; }

template <class T, int MIXED>
static hipError_t lg_factor(T* W, int64_t n, double* dacc, T* rinv, T* part, int64_t part_cap,
                            int32_t* info, hipStream_t s)
{
    constexpr int NB = LG_NB<T>;
    const size_t smem = lg_diag_smem<T>(), smem_leaf = lf_smem<T>();
    const bool leaf = lg_diag_engine() == 0;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)k_lg_diag_factor<T, MIXED>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
        if (e != hipSuccess) return e;
        e = hipFuncSetAttribute((const void*)k_lg_leaf<T, MIXED>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem_leaf);
        if (e != hipSuccess) return e;
        attr = true;
    }
    for (int64_t r0 = 0; r0 < n; r0 += NB) {
        const int nl = (int)std::min<int64_t>(NB, n - r0);
        const int64_t c0 = r0 + nl, mr = n - c0;
        T* rv = rinv + (r0 / NB) * NB * NB;
        if (leaf)
            hipLaunchKernelGGL((k_lg_leaf<T, MIXED>), dim3(1), dim3(LF_THREADS), smem_leaf, s, W, n,
                               (int)r0, nl, dacc, rv, info);
        else
            hipLaunchKernelGGL((k_lg_diag_factor<T, MIXED>), dim3(1), dim3(NB * LG_TPC), smem, s, W, n,
                               (int)r0, nl, dacc, rv, info);
        if (mr <= 0) break;
        // R_I,>I = R_II^{-T} A_I,>I over one tile row: K split (32 deep) so that
        // the GPU fills; the partials are reduced into place after every split
        // has read A_I,>I (without a split, one M tile spans the panel, so the
        // product is also safe in place)
        hipError_t e = gemm_splitk<T>(nl, (int)mr, nl, 1.0, rv, NB, 1, W + r0 * n + c0, n, 0,
                                      W + r0 * n + c0, n, part, part_cap, s, 0, 32);
        if (e != hipSuccess) return e;
        if (MIXED)
            hipLaunchKernelGGL(k_lg_dacc<T>, dim3(blocks_for(mr, 64)), dim3(64), 0, s, W, n, (int)r0,
                               nl, (int)c0, (int)n, dacc);
        // A_>I,>I -= R_I,>I^T R_I,>I  (upper half)
        e = gemm<T, T, T>((int)mr, (int)mr, nl, -1.0, W + r0 * n + c0, n, 1, W + r0 * n + c0, n, 0,
                          1.0, W + c0 * n + c0, n, 1, s);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

template <class T>
static hipError_t lg_inverse_from_r(const T* W, int64_t n, const T* rinv, T* X, int64_t ldx,
                                    T* ctmp, T* wblk, T* part, int64_t part_cap, hipStream_t s)
{
    constexpr int NB = LG_NB<T>;
    const size_t smem = (size_t)(2 * NB * LG_LD<T> + NB + 4) * sizeof(T);
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)k_lg_diag_inverse<T>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
        if (e != hipSuccess) return e;
        attr = true;
    }
    const int64_t nblk = (n + NB - 1) / NB;
    for (int64_t I = nblk - 1; I >= 0; --I) {
        const int64_t r0 = I * NB;
        const int nl = (int)std::min<int64_t>(NB, n - r0);
        const int64_t c0 = r0 + nl, mr = n - c0;
        const T* rv = rinv + I * NB * NB;
        if (mr > 0) {
            // C = R_I,>I X_>I,>I
            hipError_t e = gemm_splitk<T>(nl, (int)mr, (int)mr, 1.0, W + r0 * n + c0, n, 0,
                                          X + c0 * ldx + c0, ldx, 0, ctmp, mr, part, part_cap, s);
            if (e != hipSuccess) return e;
            // X_I,>I = -R_II^{-1} C
            e = gemm<T, T, T>(nl, (int)mr, nl, -1.0, rv, NB, 0, ctmp, mr, 0, 0.0,
                              X + r0 * ldx + c0, ldx, 0, s);
            if (e != hipSuccess) return e;
            // X_>I,I = X_I,>I^T
            hipLaunchKernelGGL((k_lg_transpose<T, T>), dim3((unsigned)((mr + 31) / 32), (unsigned)((nl + 31) / 32)),
                               dim3(32, 8), 0, s, X + r0 * ldx + c0, ldx, X + c0 * ldx + r0, ldx,
                               nl, (int)mr);
            // W = R_I,>I X_I,>I^T
            e = gemm_splitk<T>(nl, nl, (int)mr, 1.0, W + r0 * n + c0, n, 0, X + r0 * ldx + c0, ldx,
                               1, wblk, NB, part, part_cap, s);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL((k_lg_diag_inverse<T>), dim3(1), dim3(NB), smem, s, W, n, (int)r0, nl,
                           wblk, mr > 0 ? 1 : 0, X, ldx);
    }
    return hipGetLastError();
}

// diagonal block of M = R^{-1}: the upper triangle from the panel inverse,
// zeros below (the triangular GEMMs read whole diagonal tiles)
template <class T>
__global__ void k_lg_put_diag(const T* __restrict__ rv, T* __restrict__ W, int64_t ldw, int jb)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    constexpr int NB = LG_NB<T>;
    if (e >= jb * jb) return;
    const int i = e / jb, jj = e % jb;
    W[(int64_t)i * ldw + jj] = (jj >= i) ? rv[(int64_t)i * NB + jj] : T(0);
}

// M = R^{-1} in place over R in W (blocked triangular inverse, block columns
// left to right; the zero blocks below the diagonal are never touched):
//   M_{<J,J} = -(M_{<J,<J} R_{<J,J}) M_JJ,   M_JJ = R_JJ^{-1} (from the factor)
template <class T>
static hipError_t lg_trtri(T* W, int64_t n, const T* rinv, T* ctmp, T* part, int64_t cap,
                           hipStream_t s)
{
    constexpr int NB = LG_NB<T>;
    for (int64_t j0 = 0; j0 < n; j0 += NB) {
        const int jb = (int)std::min<int64_t>(NB, n - j0);
        const T* rv = rinv + (j0 / NB) * NB * NB;
        if (j0 > 0) {
            // ctmp (j0 x jb) = M_{<J,<J} R_{<J,J}; M is upper triangular by tiles
            hipError_t e = gemm_splitk<T>((int)j0, jb, (int)j0, 1.0, W, n, 0, W + j0, n, 0, ctmp,
                                          jb, part, cap, s, /*tri=*/1);
            if (e != hipSuccess) return e;
            e = gemm<T, T, T>((int)j0, jb, jb, -1.0, ctmp, jb, 0, rv, NB, 0, 0.0, W + j0, n, 0, s);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(k_lg_put_diag<T>, dim3(blocks_for((int64_t)jb * jb)), dim3(256), 0, s, rv,
                           W + j0 * n + j0, n, jb);
    }
    return hipGetLastError();
}

// X = M M^T (upper half, then mirrored): x_ij = sum_{k >= j} m_ik m_jk, one
// launch over the upper tiles, each starting its K range at its first column
template <class T>
static hipError_t lg_lauum(const T* W, int64_t n, T* X, int64_t ldx, hipStream_t s)
{
    hipError_t e = gemm<T, T, T>((int)n, (int)n, (int)n, 1.0, W, n, 0, W, n, 1, 0.0, X, ldx, 1, s,
                                 /*tri=*/2);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_lg_symmetrize<T, T>), dim3((unsigned)((n + 31) / 32), (unsigned)((n + 31) / 32)),
                       dim3(32, 8), 0, s, X, ldx, X, ldx, (int)n);
    return hipGetLastError();
}

// Inverse from the factor: TRTRI + M M^T (default), or the Section IV
// recurrence in block form (configuration inv = 1).
static int lg_use_blocked_iv() { return g_cfg.inv; }

template <class T, int MIXED>
static hipError_t lg_inverse(int64_t n, const T* a, int64_t lda, T* x, int64_t ldx, int ns_steps,
                             int32_t* info, void* work, hipStream_t s)
{
    LgWork<T> L(n, MIXED);
    char* w = static_cast<char*>(work);
    T* W = reinterpret_cast<T*>(w + L.wmat);
    T* rinv = reinterpret_cast<T*>(w + L.rinv);
    T* ctmp = reinterpret_cast<T*>(w + L.ctmp);
    T* wblk = reinterpret_cast<T*>(w + L.wblk);
    T* part = reinterpret_cast<T*>(w + L.part);
    double* dacc = reinterpret_cast<double*>(w + L.dacc);
    if (info) {
        hipError_t e0 = fill_i32(info, 1, 0, s);
        if (e0 != hipSuccess) return e0;
    }
    // upper triangle of A; zeros below (the triangular products read whole tiles)
    hipLaunchKernelGGL((k_lg_copy<T, T>), dim3(blocks_for(n * n)), dim3(256), 0, s, a, lda, W, n,
                       (int)n, (int)n, 2);
    if (MIXED)
        hipLaunchKernelGGL(k_lg_dacc_init<T>, dim3(blocks_for(n)), dim3(256), 0, s, a, lda, (int)n,
                           dacc);
    hipError_t e = lg_factor<T, MIXED>(W, n, dacc, rinv, part, L.part_elems, info, s);
    if (e != hipSuccess) return e;
    if (lg_use_blocked_iv()) {
        e = lg_inverse_from_r<T>(W, n, rinv, x, ldx, ctmp, wblk, part, L.part_elems, s);
    } else {
        e = lg_trtri<T>(W, n, rinv, ctmp, part, L.part_elems, s);
        if (e == hipSuccess) e = lg_lauum<T>(W, n, x, ldx, s);
    }
    if (e != hipSuccess) return e;
    if (MIXED && ns_steps > 0) {
        double* E = reinterpret_cast<double*>(w + L.emat);
        T* X1 = reinterpret_cast<T*>(w + L.xtmp);
        // full symmetric A (the factor in W is no longer needed)
        hipLaunchKernelGGL((k_lg_symmetrize<T, T>), dim3((unsigned)((n + 31) / 32), (unsigned)((n + 31) / 32)),
                           dim3(32, 8), 0, s, a, lda, W, n, (int)n);
        for (int st = 0; st < ns_steps; ++st) {
            // E = I - A X in FP64 (FP32 operands, exact products)
            hipLaunchKernelGGL(k_lg_identity<double>, dim3(blocks_for(n * n)), dim3(256), 0, s, E, n,
                               (int)n);
            e = gemm<double, T, T>((int)n, (int)n, (int)n, -1.0, W, n, 0, x, ldx, 0, 1.0, E, n, 0, s);
            if (e != hipSuccess) return e;
            // X1 = X + X E (upper half, FP32), then X = sym(X1)
            hipLaunchKernelGGL((k_lg_copy<T, T>), dim3(blocks_for(n * n)), dim3(256), 0, s, x, ldx, X1,
                               n, (int)n, (int)n, 1);
            e = gemm<T, T, double>((int)n, (int)n, (int)n, 1.0, x, ldx, 0, E, n, 0, 1.0, X1, n, 1, s);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL((k_lg_symmetrize<T, T>), dim3((unsigned)((n + 31) / 32), (unsigned)((n + 31) / 32)),
                               dim3(32, 8), 0, s, X1, n, x, ldx, (int)n);
        }
    }
    if (info)
        hipLaunchKernelGGL(k_lg_nan_if<T>, dim3(blocks_for(n * n)), dim3(256), 0, s, info, x, ldx,
                           (int)n);
    return hipGetLastError();
}

// ---- entry points ---------------------------------------------------------------
size_t large_workspace(int dtype, int64_t n, int which, int mixed)
{
    (void)which;
    if (dtype == DT_F32) return LgWork<float>(n, mixed).total;
    if (dtype == DT_F64) return LgWork<double>(n, 0).total;
    return 0;
}

// Selects configuration `cfg` (0..large_config_count()-1) for the calls that
// follow on this host thread.
static void lg_select(int cfg)
{
    g_cfg = LG_CFGS[(cfg >= 0 && cfg < LG_NCFG) ? cfg : 0];
    g_splitk_target = g_cfg.splitk;
    g_gemm_big = g_cfg.big != 0;
}

hipError_t large_factor(int dtype, int64_t n, void* a, int64_t lda, int32_t* info, void* work,
                        hipStream_t s, int cfg)
{
    lg_select(cfg);
    // in place on a (leading dimension lda must equal n for the blocked path)
    if (lda != n) return hipErrorNotSupported;
    if (info) {
        hipError_t e0 = fill_i32(info, 1, 0, s);
        if (e0 != hipSuccess) return e0;
    }
    if (dtype == DT_F32) {
        LgWork<float> L(n, 0);
        char* w = static_cast<char*>(work);
        return lg_factor<float, 0>(static_cast<float*>(a), n, reinterpret_cast<double*>(w + L.dacc),
                                   reinterpret_cast<float*>(w + L.rinv),
                                   reinterpret_cast<float*>(w + L.part), L.part_elems, info, s);
    }
    if (dtype == DT_F64) {
        LgWork<double> L(n, 0);
        char* w = static_cast<char*>(work);
        return lg_factor<double, 0>(static_cast<double*>(a), n,
                                    reinterpret_cast<double*>(w + L.dacc),
                                    reinterpret_cast<double*>(w + L.rinv),
                                    reinterpret_cast<double*>(w + L.part), L.part_elems, info, s);
    }
    return hipErrorNotSupported;
}

hipError_t large_inverse(int dtype, int64_t n, const void* a, int64_t lda, void* x, int64_t ldx,
                         int mixed, int ns_steps, int fill, int32_t* info, void* work, hipStream_t s,
                         int cfg)
{
    (void)fill;   // the blocked path always writes both halves (the GEMMs read them)
    lg_select(cfg);
    if (dtype == DT_F32) {
        if (mixed)
            return lg_inverse<float, 1>(n, static_cast<const float*>(a), lda, static_cast<float*>(x),
                                        ldx, ns_steps, info, work, s);
        return lg_inverse<float, 0>(n, static_cast<const float*>(a), lda, static_cast<float*>(x), ldx,
                                    0, info, work, s);
    }
    if (dtype == DT_F64 && !mixed)
        return lg_inverse<double, 0>(n, static_cast<const double*>(a), lda, static_cast<double*>(x),
                                     ldx, 0, info, work, s);
    return hipErrorNotSupported;
}

}  // namespace ci
