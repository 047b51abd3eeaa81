// group16_mfma.hpp -- mixed-precision inversion of batches of order <= 16
// (float or complex float): factorisation and Section IV back-substitution on
// 16-lane groups, Newton-Schulz refinement on the matrix cores.
//
// One wave owns four matrices (one per 16-lane group).  A is staged through
// LDS (rows padded to 17 entries), made Hermitian there from its upper
// triangle, and each lane takes its column into registers for group_core.
// The X-hat columns go back to LDS, and each refinement step of each matrix
// then runs as whole-wave MFMA 16 x 16 x 4 products:
//   E = I - A X   in FP64 (v_mfma_f64_16x16x4f64 on exactly converted FP32
//                 values: every product is exact, the sums are FP64),
//   F = X E       in FP32 (v_mfma_f32_16x16x4f32, E rounded to FP32),
//   X <- X + F    upper half, diagonal real, lower half the conjugate mirror.
// Complex products take three real products (Ar Xr, Ai Xi and
// (Ar + Ai)(Xr + Xi)).  The residual accumulator lands in the
// FP64 layout (lane holds E[g + 4 v][c]), which is directly the B operand of
// the update when step v takes k = g + 4 v.
#pragma once

#include "group_impl.hpp"
#include "mfma.hpp"

namespace ci {

constexpr int G16_LD = 17;                 // padded LDS row (entries)
constexpr int G16_MAT = 16 * G16_LD;       // entries per staged matrix
constexpr int G16_MPW = 4;                 // matrices per wave

CI_D float g16_re(float v) { return v; }
CI_D float g16_re(cf v) { return v.re; }
CI_D float g16_im(float) { return 0.f; }
CI_D float g16_im(cf v) { return v.im; }

template <class V>
CI_D V g16_make(float r, float i)
{
    if constexpr (vt<V>::cplx) return V{r, i};
    else return r;
}

// Orders the LDS accesses of one wave across its lanes (a workgroup of one
// wave needs no workgroup barrier): a wavefront-scope release fence, a wave
// barrier that no instruction is moved across, and an acquire fence.
CI_D void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One Newton-Schulz step on the staged matrix A (Hermitian, full) and X
// (Hermitian, full), in place on X.  Whole wave.
template <class V>
CI_D void g16_ns_step(const V* __restrict__ As, V* __restrict__ Xs, int lane)
{
    constexpr bool C = vt<V>::cplx;
    const int g = lane / 16, c = lane % 16;
    // complex products with three real products each:
    //   Re(A X) = P1 - P2, Im(A X) = P3 - P1 - P2,
    //   P1 = Ar Xr, P2 = Ai Xi, P3 = (Ar + Ai)(Xr + Xi)
    // (the operand sums are exact or FP64-rounded for the residual; for the
    // update they round in FP32 inside a correction of size ~kappa u)
    gd4 p1 = {0, 0, 0, 0}, p2 = {0, 0, 0, 0}, p3 = {0, 0, 0, 0};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int k = 4 * t + g;
        const V av = As[c * G16_LD + k];       // A[c][k]
        const V xv = Xs[k * G16_LD + c];       // X[k][c]
        const double ar = g16_re(av), xr = g16_re(xv);
        p1 = mfma16(ar, xr, p1);
        if constexpr (C) {
            const double ai = g16_im(av), xi = g16_im(xv);
            p2 = mfma16(ai, xi, p2);
            p3 = mfma16(ar + ai, xr + xi, p3);
        }
    }
    // E = I - A X; lane holds rows g + 4 v of column c
    float e_r[4], e_i[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const double axr = C ? p1[v] - p2[v] : p1[v];
        e_r[v] = (float)(((g + 4 * v) == c ? 1.0 : 0.0) - axr);
        e_i[v] = C ? (float)(-(p3[v] - p1[v] - p2[v])) : 0.f;
    }
    gf4 q1 = {0, 0, 0, 0}, q2 = {0, 0, 0, 0}, q3 = {0, 0, 0, 0};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int k = g + 4 * t;
        const V xv = Xs[c * G16_LD + k];       // X[c][k]
        const float xr = g16_re(xv);
        q1 = mfma16(xr, e_r[t], q1);
        if constexpr (C) {
            const float xi = g16_im(xv);
            q2 = mfma16(xi, e_i[t], q2);
            q3 = mfma16(xr + xi, e_r[t] + e_i[t], q3);
        }
    }
    gf4 fr, fi;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        fr[v] = C ? q1[v] - q2[v] : q1[v];
        fi[v] = C ? q3[v] - q1[v] - q2[v] : 0.f;
    }
    // F lands as rows 4 g + v of column c: X + F on the upper half
    V xn[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int i = 4 * g + v;
        const V xo = Xs[i * G16_LD + c];
        xn[v] = g16_make<V>(g16_re(xo) + fr[v], C ? g16_im(xo) + fi[v] : 0.f);
    }
    // Every lane's reads of X above precede any lane's writes below, and the
    // writes precede later reads (the next step, the store): both orders are
    // made explicit at wavefront scope.
    wave_sync();
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int i = 4 * g + v;
        if (i == c) Xs[i * G16_LD + c] = realpart_only(xn[v]);
        if (i < c) {
            Xs[i * G16_LD + c] = xn[v];
            Xs[c * G16_LD + i] = cj(xn[v]);
        }
    }
    wave_sync();
}

#ifndef CI_G16_WAVES
#define CI_G16_WAVES 1
#endif

// Occupancy target: CI_G16_WAVES waves per SIMD bounds the registers the
// scheduler may use (the factorisation's broadcasts are latency-bound and
// need several waves to hide).
template <class V, int METHOD>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(CI_G16_WAVES)))
k_group16_mfma(const V* __restrict__ a, V* __restrict__ x, int64_t batch, int n, int64_t lda,
               int64_t sa, int64_t ldx, int64_t sx, int ns_steps, int fill,
               int32_t* __restrict__ info)
{
    using R = typename vt<V>::real;
    constexpr int NB = 16, G = 16;
    __shared__ __align__(16) V As[G16_MPW * G16_MAT];
    __shared__ __align__(16) V Xs[G16_MPW * G16_MAT];
    __shared__ int s_fail[G16_MPW];
    const int lane = threadIdx.x;
    const int grp = lane / G, q = lane % G;
    const int64_t b0 = (int64_t)blockIdx.x * G16_MPW;

    // ---- stage A (identity beyond n and for matrices past the batch); all
    // sixteen loads of a lane are issued before the first LDS store ----
    {
        V ar[16];
#pragma unroll
        for (int qq = 0; qq < 16; ++qq) {
            const int e = lane + 64 * qq;
            const int m = e / 256, i = (e / 16) % 16, j = e % 16;
            const int64_t b = b0 + m;
            ar[qq] = mk<V>(R(i == j ? 1 : 0));
            if (b < batch && i < n && j < n) ar[qq] = a[b * sa + (int64_t)i * lda + j];
        }
#pragma unroll
        for (int qq = 0; qq < 16; ++qq) {
            const int e = lane + 64 * qq;
            const int m = e / 256, i = (e / 16) % 16, j = e % 16;
            As[m * G16_MAT + i * G16_LD + j] = ar[qq];
        }
    }
    __syncthreads();

    // ---- column q of A from its upper triangle; complete the Hermitian A ----
    V* Am = As + grp * G16_MAT;
    V M[1][NB];
    double piv[1];
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        const V up = Am[k * G16_LD + q];          // a_kq, k <= q (upper triangle)
        M[0][k] = (k < q) ? up : ((k == q) ? realpart_only(up) : mk<V>(R(0)));
        if (k == q) piv[0] = (double)re(up);
    }
    // lane q rewrites only the strict lower part of its column (from row q of
    // the upper triangle) and its own diagonal: no entry another lane reads
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        if (k > q) Am[k * G16_LD + q] = cj(Am[q * G16_LD + k]);
        if (k == q) Am[k * G16_LD + q] = realpart_only(Am[k * G16_LD + q]);
    }

    R dall[NB];
    const int fail = group_core<V, NB, G, OP_INV, METHOD, 1>(M, piv, dall, q);
    V* Xm = Xs + grp * G16_MAT;
#pragma unroll
    for (int k = 0; k < NB; ++k) Xm[k * G16_LD + q] = M[0][k];
    if (q == 0) s_fail[grp] = fail;
    __syncthreads();

    // ---- Newton-Schulz on the matrix cores, one matrix at a time ----
    for (int st = 0; st < ns_steps; ++st)
        for (int m = 0; m < G16_MPW; ++m) g16_ns_step<V>(As + m * G16_MAT, Xs + m * G16_MAT, lane);

    // ---- store (NaN for a failed factorisation) ----
#pragma unroll
    for (int e = lane; e < G16_MPW * 256; e += 64) {
        const int m = e / 256, i = (e / 16) % 16, j = e % 16;
        const int64_t b = b0 + m;
        if (b < batch && i < n && j < n && (fill || i <= j)) {
            const V v = s_fail[m] ? nan_value<V>() : Xs[m * G16_MAT + i * G16_LD + j];
            x[b * sx + (int64_t)i * ldx + j] = v;
        }
    }
    if (q == 0 && info && b0 + grp < batch) info[b0 + grp] = fail;
}

template <class V>
static hipError_t group16_mfma_run(const BatchArgs& p, int n, int method, hipStream_t s)
{
    const int64_t blocks = (p.batch + G16_MPW - 1) / G16_MPW;
    if (method == 0)
        hipLaunchKernelGGL((k_group16_mfma<V, 0>), dim3((unsigned)blocks), dim3(64), 0, s,
                           (const V*)p.a, (V*)p.x, p.batch, n, p.lda, p.sa, p.ldx, p.sx,
                           p.ns_steps, p.fill, p.info);
    else
        hipLaunchKernelGGL((k_group16_mfma<V, 1>), dim3((unsigned)blocks), dim3(64), 0, s,
                           (const V*)p.a, (V*)p.x, p.batch, n, p.lda, p.sa, p.ldx, p.sx,
                           p.ns_steps, p.fill, p.info);
    return hipGetLastError();
}

}  // namespace ci
