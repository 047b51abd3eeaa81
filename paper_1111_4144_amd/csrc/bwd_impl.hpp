// bwd_impl.hpp -- adjoint of X = A^{-1}: gA = -X Gh X, Gh = (G + G^H)/2, for
// batches of small matrices.  Included by one translation unit per type.
//
// With L = Re<G, X> and Hermitian perturbations dA, d(A^{-1}) = -X dA X gives
// dL = Re<-X Gh X, dA>; gA is Hermitian.  The forward's X (full Hermitian)
// is reused, so the backward costs two products and one HBM pass (X, G in;
// gA out).
//
// Orders <= 16: a group of G lanes per matrix in registers, columns dealt
// cyclically (column j = s*G + q on lane q, slot s).  T = Gh X column by
// column: T[:, j] = sum_k Gh[:, k] x_kj with column k of Gh broadcast from its
// owner; then gA[:, j] = -sum_k X[:, k] t_kj the same way.
// Orders 17..64: one lane per column, Gh / X / T column-major in LDS, every
// entry a 16-byte-packet inner product: t_ij = Gh[:, i]^H X[:, j] and
// gA_ij = -X[:, i]^H T[:, j] (Gh and X are Hermitian).
#pragma once

#include "group_impl.hpp"
#include "mfma.hpp"
#include "tpm_impl.hpp"
#include "wpm_impl.hpp"

namespace ci {

template <class V, int NB, int G>
__global__ void __launch_bounds__(GROUP_BLOCK)
k_bwd_group(const V* __restrict__ x, const V* __restrict__ g, V* __restrict__ ga, int64_t batch,
            int n, int64_t stride)
{
    using R = typename vt<V>::real;
    constexpr int S = (NB + G - 1) / G;
    constexpr int MPB = GROUP_BLOCK / G;
    const int q = threadIdx.x % G;
    const int64_t b = (int64_t)blockIdx.x * MPB + threadIdx.x / G;
    const bool valid = b < batch;
    const V* xb = x + (valid ? b : 0) * stride;
    const V* gb = g + (valid ? b : 0) * stride;
    V* ob = ga + (valid ? b : 0) * stride;

    V Xc[S][NB], Hc[S][NB];     // columns of X and Gh (zero beyond n)
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int j = s * G + q;
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            V xv = mk<V>(R(0)), hv = mk<V>(R(0));
            if (valid && j < n && k < n) {
                xv = xb[k * n + j];
                const V gkj = gb[k * n + j], gjk = gb[j * n + k];
                hv = scal(add(gkj, cj(gjk)), R(0.5));
            }
            Xc[s][k] = xv;
            Hc[s][k] = hv;
        }
    }
    // T = Gh X: t_ij = sum_k Gh_ik x_kj, Gh_ik from the owner of column k
    V T[S][NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
#pragma unroll
        for (int s = 0; s < S; ++s) T[s][i] = mk<V>(R(0));
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            // the empty asm on the accumulator keeps each product next to its
            // broadcast (otherwise every broadcast is hoisted and stays live)
            const V hik = bc<G>(Hc[k / G][i], k % G);
#pragma unroll
            for (int s = 0; s < S; ++s) {
                madd(T[s][i], hik, Xc[s][k]);
                opaque(T[s][i]);
            }
        }
    }
    // gA = -X T: ga_ij = -sum_k x_ik t_kj, x_ik from the owner of column k
    V O[S][NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
#pragma unroll
        for (int s = 0; s < S; ++s) O[s][i] = mk<V>(R(0));
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            const V xik = bc<G>(Xc[k / G][i], k % G);
#pragma unroll
            for (int s = 0; s < S; ++s) {
                msub(O[s][i], xik, T[s][k]);
                opaque(O[s][i]);
            }
        }
    }
    // upper half of column j and its conjugate mirror (exactly Hermitian)
    if (valid) {
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int j = s * G + q;
            if (j < n) {
#pragma unroll
                for (int i = 0; i < NB; ++i) {
                    if (i < n && i <= j) {
                        const V v = (i == j) ? realpart_only(O[s][i]) : O[s][i];
                        ob[i * n + j] = v;
                        if (i < j) ob[j * n + i] = cj(v);
                    }
                }
            }
        }
    }
}

template <class V, int NB>
__global__ void __launch_bounds__(64)
k_bwd_lds(const V* __restrict__ x, const V* __restrict__ g, V* __restrict__ ga, int64_t batch,
          int n, int64_t stride)
{
    using R = typename vt<V>::real;
    constexpr int MPB = 64 / NB;
    constexpr int P = WPM_P<V>;
    constexpr int LD = WPM_LD<V, NB>;
    constexpr int REG = NB * LD;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int grp = threadIdx.x / NB;
    const int j = threadIdx.x % NB;
    const int64_t b = (int64_t)blockIdx.x * MPB + grp;
    const bool valid = b < batch;
    const V* xb = x + (valid ? b : 0) * stride;
    const V* gb = g + (valid ? b : 0) * stride;
    V* ob = ga + (valid ? b : 0) * stride;
    V* Hm = reinterpret_cast<V*>(smem_raw) + (size_t)grp * 3 * REG;
    V* Xm = Hm + REG;
    V* Tm = Hm + 2 * REG;
    const int np = (n + P - 1) / P * P;

    for (int k = 0; k < NB; ++k) {
        V xv = mk<V>(R(0)), hv = mk<V>(R(0));
        if (valid && j < n && k < n) {
            xv = xb[k * n + j];
            hv = scal(add(gb[k * n + j], cj(gb[j * n + k])), R(0.5));
        }
        Xm[j * LD + k] = xv;
        Hm[j * LD + k] = hv;
    }
    __syncthreads();
    // t_ij = sum_k conj(gh_ki) x_kj
    for (int i = 0; i < np; ++i) {
        V acc = mk<V>(R(0));
        for (int p = 0; p < np / P; ++p) {
            const Pk<V> u = ldpk(Hm + i * LD + p * P);
            const Pk<V> w = ldpk(Xm + j * LD + p * P);
#pragma unroll
            for (int c = 0; c < P; ++c) madd(acc, cj(u.v[c]), w.v[c]);
        }
        Tm[j * LD + i] = acc;
    }
    __syncthreads();
    // gA_ij = -sum_k conj(x_ki) t_kj, upper half + mirror
    for (int i = 0; i < np; ++i) {
        V acc = mk<V>(R(0));
        for (int p = 0; p < np / P; ++p) {
            const Pk<V> u = ldpk(Xm + i * LD + p * P);
            const Pk<V> w = ldpk(Tm + j * LD + p * P);
#pragma unroll
            for (int c = 0; c < P; ++c) msub(acc, cj(u.v[c]), w.v[c]);
        }
        if (valid && j < n && i < n && i <= j) {
            const V v = (i == j) ? realpart_only(acc) : acc;
            ob[i * n + j] = v;
            if (i < j) ob[j * n + i] = cj(v);
        }
    }
}

// Orders 9..16, FP32 element types: both products on the matrix cores.  One
// wave owns four matrices; X and Gh are staged in LDS (rows padded to 17),
// T = Gh X is one MFMA 16 x 16 x 4 chain per matrix (complex: four real
// products), and it lands in the FP32 accumulator layout (lane (g, c) holds
// T[4 g + v][c]), which is the B operand of gA = -X T when step t takes
// k = 4 g + t.  The upper half of gA is staged back through LDS and written
// with its conjugate mirror.
constexpr int B16_LD = 17;
constexpr int B16_MAT = 16 * B16_LD;

CI_D float b16_re(float v) { return v; }
CI_D float b16_re(cf v) { return v.re; }
CI_D float b16_im(float) { return 0.f; }
CI_D float b16_im(cf v) { return v.im; }

template <class V>
__global__ void __launch_bounds__(64)
k_bwd16_mfma(const V* __restrict__ x, const V* __restrict__ g, V* __restrict__ ga, int64_t batch,
             int n, int64_t stride)
{
    using R = typename vt<V>::real;
    constexpr bool C = vt<V>::cplx;
    __shared__ __align__(16) V Xs[4 * B16_MAT];
    __shared__ __align__(16) V Hs[4 * B16_MAT];
    const int lane = threadIdx.x;
    const int lg = lane / 16, lc = lane % 16;
    const int64_t b0 = (int64_t)blockIdx.x * 4;
    // stage X and G (zero beyond n and past the batch): every load is issued
    // before the first LDS store, so the copy is not one latency per row
    V xr[16], gr[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int e = lane + 64 * q;
        const int m = e / 256, i = (e / 16) % 16, j = e % 16;
        const int64_t b = b0 + m;
        xr[q] = mk<V>(R(0));
        gr[q] = mk<V>(R(0));
        if (b < batch && i < n && j < n) {
            xr[q] = x[b * stride + (int64_t)i * n + j];
            gr[q] = g[b * stride + (int64_t)i * n + j];
        }
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int e = lane + 64 * q;
        const int m = e / 256, i = (e / 16) % 16, j = e % 16;
        Xs[m * B16_MAT + i * B16_LD + j] = xr[q];
        Hs[m * B16_MAT + i * B16_LD + j] = gr[q];
    }
    __syncthreads();
    // Gh = (G + G^H) / 2 in place: each unordered pair (i <= j) by one lane
    for (int e = lane; e < 4 * 136; e += 64) {
        const int m = e / 136;
        int r = e % 136, i = 0;
        while (r >= 16 - i) { r -= 16 - i; ++i; }
        const int j = i + r;
        V* H = Hs + m * B16_MAT;
        const V gij = H[i * B16_LD + j], gji = H[j * B16_LD + i];
        const V h = scal(add(gij, cj(gji)), R(0.5));
        H[i * B16_LD + j] = (i == j) ? realpart_only(h) : h;
        H[j * B16_LD + i] = (i == j) ? realpart_only(h) : cj(h);
    }
    __syncthreads();
    for (int m = 0; m < 4; ++m) {
        const V* Xm = Xs + m * B16_MAT;
        const V* Hm = Hs + m * B16_MAT;
        // T = Gh X
        gf4 tr = {0, 0, 0, 0}, ti = {0, 0, 0, 0};
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int k = 4 * t + lg;
            const V hv = Hm[lc * B16_LD + k];      // Gh[c][k]
            const V xv = Xm[k * B16_LD + lc];      // X[k][c]
            tr = mfma16(b16_re(hv), b16_re(xv), tr);
            if constexpr (C) {
                tr = mfma16(-b16_im(hv), b16_im(xv), tr);
                ti = mfma16(b16_re(hv), b16_im(xv), ti);
                ti = mfma16(b16_im(hv), b16_re(xv), ti);
            }
        }
        // gA = -X T, step t taking k = 4 lg + t (T's rows held by this lane)
        gf4 ar = {0, 0, 0, 0}, ai = {0, 0, 0, 0};
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const V xv = Xm[lc * B16_LD + 4 * lg + t];   // X[c][k]
            ar = mfma16(-b16_re(xv), tr[t], ar);
            if constexpr (C) {
                ar = mfma16(b16_im(xv), ti[t], ar);
                ai = mfma16(-b16_re(xv), ti[t], ai);
                ai = mfma16(-b16_im(xv), tr[t], ai);
            }
        }
        __syncthreads();                 // every lane has read matrix m's X
        V* Om = Xs + m * B16_MAT;        // gA replaces X: rows 4 lg + v, column lc
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = 4 * lg + v;
            V val;
            if constexpr (C) val = V{ar[v], ai[v]};
            else val = ar[v];
            if (i == lc) Om[i * B16_LD + lc] = realpart_only(val);
            if (i < lc) {
                Om[i * B16_LD + lc] = val;
                Om[lc * B16_LD + i] = cj(val);
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int e = lane + 64 * q;
        const int m = e / 256, i = (e / 16) % 16, j = e % 16;
        const int64_t b = b0 + m;
        if (b < batch && i < n && j < n) ga[b * stride + (int64_t)i * n + j] = Xs[m * B16_MAT + i * B16_LD + j];
    }
}

template <class V>
static hipError_t bwd_run(int n, const void* x, const void* g, void* ga, int64_t batch,
                          int64_t stride, hipStream_t s)
{
    if constexpr (sizeof(typename vt<V>::real) == 4) {
        if (n > 8 && n <= 16) {
            hipLaunchKernelGGL(k_bwd16_mfma<V>, dim3((unsigned)((batch + 3) / 4)), dim3(64), 0, s,
                               (const V*)x, (const V*)g, (V*)ga, batch, n, stride);
            return hipGetLastError();
        }
    }
    auto grp = [&](auto kern, int G) {
        const int mpb = GROUP_BLOCK / G;
        hipLaunchKernelGGL(kern, dim3((unsigned)((batch + mpb - 1) / mpb)), dim3(GROUP_BLOCK), 0,
                           s, (const V*)x, (const V*)g, (V*)ga, batch, n, stride);
        return hipGetLastError();
    };
    auto lds = [&](auto kern, int NB, size_t smem) {
        const int mpb = 64 / NB;
        hipLaunchKernelGGL(kern, dim3((unsigned)((batch + mpb - 1) / mpb)), dim3(64), smem, s,
                           (const V*)x, (const V*)g, (V*)ga, batch, n, stride);
        return hipGetLastError();
    };
    if (n <= 4) return grp(k_bwd_group<V, 4, 4>, 4);
    if (n <= 8) return grp(k_bwd_group<V, 8, 4>, 4);
    if (n <= 16) return grp(k_bwd_group<V, 16, 16>, 16);
    if (n <= 32) {
        constexpr size_t sm = 2 * 3 * 32 * WPM_LD<V, 32> * sizeof(V);
        return lds(k_bwd_lds<V, 32>, 32, sm);
    }
    if constexpr (sizeof(V) <= 8) {
        if (n <= 64) {
            constexpr size_t sm = 3 * 64 * WPM_LD<V, 64> * sizeof(V);
            auto kern = k_bwd_lds<V, 64>;
            if (sm > 65536) {
                static bool once = false;
                if (!once) {
                    hipError_t e = hipFuncSetAttribute((const void*)kern,
                                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                                       (int)sm);
                    if (e != hipSuccess) return e;
                    once = true;
                }
            }
            return lds(kern, 64, sm);
        }
    }
    return hipErrorNotSupported;
}

}  // namespace ci
