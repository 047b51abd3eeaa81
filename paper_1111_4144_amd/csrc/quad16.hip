// quad16.hip -- batched inversion of orders 9..16 (float and complex float
// elements) with four lanes per matrix and sixteen matrices per wave.
//
// Each quad of lanes owns one matrix: lane q holds columns q, q+4, q+8, q+12
// in registers (group_core with G = 4: the factorisation of eqs. 3-4 /
// 10-11 and the Section IV back-substitution, with row broadcasts inside the
// quad by DPP quad_perm).  Compared with sixteen lanes per matrix, every
// broadcast feeds up to four columns and far fewer multiply-adds fall on
// columns that are already finished, so the instruction count per matrix is
// about half.
//
// The upper triangle of A is staged once in LDS, packed (136 entries per
// matrix, row-major upper triangle), with coalesced loads; the lanes take
// their columns from it.  In mixed precision the packed copy stays for the
// Newton-Schulz step, which runs on the matrix cores one matrix at a time
// over the whole wave: the X-hat columns of four matrices at a time go to an
// LDS tile (rows padded to 17 entries), then for each of them
//   E = I - A X   FP64 MFMA 16x16x4 on exactly converted FP32 values,
//   F = X E       FP32 MFMA 16x16x4,
//   X <- X + F    upper half, diagonal real, lower half the conjugate mirror,
// (complex products with three real products each), and the tile is stored
// to HBM with coalesced row accesses.  Plain FP32 uses the same staging for
// the stores.
//
// All LDS traffic of a block is inside its single wave.  The places where
// one lane reads what another lane of the wave wrote are ordered by a
// wavefront-scope release/acquire fence plus a wave barrier (no workgroup
// barrier is needed and none is used after the staging).
#include "group16_mfma.hpp"
#include "group_impl.hpp"
#include "mfma.hpp"

namespace ci {

namespace {

constexpr int Q16_MPW = 16;               // matrices per wave
constexpr int Q16_PK = 136;               // packed upper-triangle entries (order 16)
#ifndef CI_Q16_TILE
#define CI_Q16_TILE 2
#endif
constexpr int Q16_TILE = CI_Q16_TILE;     // matrices per Newton-Schulz / store round

// packed index of (i, j), i <= j, row-major upper triangle of order 16
CI_D int q16_pk(int i, int j) { return i * (31 - i) / 2 + j; }

// One Newton-Schulz step for one staged matrix: A from the packed upper
// triangle (a_ck = conj(a_kc) for c > k), X full in the padded tile, in place.
// aoff / aconj: the lane's four packed offsets of a_{c, 4t+g} and whether the
// entry is taken conjugated (precomputed per lane).
template <class V>
CI_D void q16_ns_step(const V* __restrict__ Ap, V* __restrict__ Xs, const int (&aoff)[4],
                      const bool (&aconj)[4], int lane)
{
    constexpr bool C = vt<V>::cplx;
    const int g = lane / 16, c = lane % 16;
    gd4 p1 = {0, 0, 0, 0}, p2 = {0, 0, 0, 0}, p3 = {0, 0, 0, 0};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int k = 4 * t + g;
        V av = Ap[aoff[t]];                    // A[c][k]
        if (aconj[t]) av = cj(av);
        const V xv = Xs[k * G16_LD + c];       // X[k][c]
        const double ar = g16_re(av), xr = g16_re(xv);
        p1 = mfma16(ar, xr, p1);
        if constexpr (C) {
            const double ai = g16_im(av), xi = g16_im(xv);
            p2 = mfma16(ai, xi, p2);
            p3 = mfma16(ar + ai, xr + xi, p3);
        }
    }
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
    V xn[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int i = 4 * g + v;
        const float fr = C ? q1[v] - q2[v] : q1[v];
        const float fi = C ? q3[v] - q1[v] - q2[v] : 0.f;
        const V xo = Xs[i * G16_LD + c];
        xn[v] = g16_make<V>(g16_re(xo) + fr, C ? g16_im(xo) + fi : 0.f);
    }
    wave_sync();                               // every read of X precedes the writes
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

#ifndef CI_Q16_WAVES
#define CI_Q16_WAVES 2
#endif

// Occupancy target CI_Q16_WAVES waves per SIMD (the register budget the
// scheduler may use; LDS allows about two such waves per SIMD as well).
template <class V, int METHOD, int MIXED>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(CI_Q16_WAVES)))
k_quad16(const V* __restrict__ a, V* __restrict__ x, int64_t batch, int n, int64_t lda, int64_t sa,
         int64_t ldx, int64_t sx, int ns_steps, int fill, int32_t* __restrict__ info)
{
    using R = typename vt<V>::real;
    using P = typename std::conditional<MIXED, double, R>::type;   // pivot precision
    constexpr int NB = 16, G = 4, S = 4;
    __shared__ __align__(16) V Ap[Q16_MPW * Q16_PK];
    __shared__ __align__(16) V Xs[Q16_TILE * G16_MAT];
    __shared__ int s_fail[Q16_MPW];
    const int lane = threadIdx.x;
    const int mq = lane / G, q = lane % G;
    const int64_t b0 = (int64_t)blockIdx.x * Q16_MPW;

    // ---- stage the upper triangles (identity beyond n and past the batch)
    // A full block of dense order-16 matrices is one contiguous run of
    // 16 x 256 entries: 16-byte loads, eight in flight per lane.
    constexpr int VPP = 16 / (int)sizeof(V);                      // entries per 16 bytes
    const bool dense = n == 16 && lda == 16 && sa == 256 && b0 + Q16_MPW <= batch;
    if (dense) {
        const uint4* src = reinterpret_cast<const uint4*>(a + b0 * 256);
        constexpr int NPK = Q16_MPW * 256 / VPP / 64;             // packets per lane
#pragma unroll
        for (int part = 0; part < NPK / 8; ++part) {
            uint4 pk[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) pk[u] = src[lane + 64 * (8 * part + u)];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                V v[VPP];
                __builtin_memcpy(v, &pk[u], 16);
                const int e0 = (lane + 64 * (8 * part + u)) * VPP;
#pragma unroll
                for (int c = 0; c < VPP; ++c) {
                    const int e = e0 + c, m = e / 256, i = (e / 16) % 16, j = e % 16;
                    if (i <= j) Ap[m * Q16_PK + q16_pk(i, j)] = (i == j) ? realpart_only(v[c]) : v[c];
                }
            }
        }
    } else {
#pragma unroll
        for (int part = 0; part < 4; ++part) {
            V ar[16];
#pragma unroll
            for (int qq = 0; qq < 16; ++qq) {
                const int e = lane + 64 * (16 * part + qq);
                const int m = e / 256, i = (e / 16) % 16, j = e % 16;
                const int64_t b = b0 + m;
                ar[qq] = mk<V>(R(i == j ? 1 : 0));
                if (b < batch && i < n && j < n && i <= j) ar[qq] = a[b * sa + (int64_t)i * lda + j];
            }
#pragma unroll
            for (int qq = 0; qq < 16; ++qq) {
                const int e = lane + 64 * (16 * part + qq);
                const int m = e / 256, i = (e / 16) % 16, j = e % 16;
                if (i <= j) Ap[m * Q16_PK + q16_pk(i, j)] = (i == j) ? realpart_only(ar[qq]) : ar[qq];
            }
        }
    }
    __syncthreads();

    // ---- columns j = 4 s + q of this quad's matrix (upper part; zero below)
    const V* Am = Ap + mq * Q16_PK;
    V M[S][NB];
    P piv[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int j = s * G + q;
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            M[s][k] = mk<V>(R(0));
            if (k <= s * G + G - 1 && k <= j) M[s][k] = Am[q16_pk(k, j)];
        }
        piv[s] = (P)re(Am[q16_pk(j, j)]);
    }
    R dall[NB];
    const int fail = group_core<V, NB, G, OP_INV, METHOD, MIXED>(M, piv, dall, q);
    if (q == 0) {
        s_fail[mq] = fail;
        if (info && b0 + mq < batch) info[b0 + mq] = fail;
    }

    int aoff[4];
    bool aconj[4];
    {
        const int g = lane / 16, c = lane % 16;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int k = 4 * t + g;
            aoff[t] = c <= k ? q16_pk(c, k) : q16_pk(k, c);
            aconj[t] = c > k;
        }
    }

    // ---- four matrices at a time: X-hat to the tile, refinement, store ----
#pragma unroll 1
    for (int r = 0; r < Q16_MPW / Q16_TILE; ++r) {
        wave_sync();                           // the previous round's stores have read the tile
        const int slot = mq - r * Q16_TILE;
        if (slot >= 0 && slot < Q16_TILE) {
            V* Xm = Xs + slot * G16_MAT;
#pragma unroll
            for (int s = 0; s < S; ++s)
#pragma unroll
                for (int k = 0; k < NB; ++k) Xm[k * G16_LD + s * G + q] = M[s][k];
        }
        wave_sync();
        if constexpr (MIXED) {
            for (int st = 0; st < ns_steps; ++st)
                for (int t = 0; t < Q16_TILE; ++t)
                    q16_ns_step<V>(Ap + (r * Q16_TILE + t) * Q16_PK, Xs + t * G16_MAT, aoff, aconj,
                                   lane);
        }
        if (dense && fill && ldx == 16 && sx == 256) {
            // the tile's matrices are contiguous in x: 16-byte stores
            uint4* dst = reinterpret_cast<uint4*>(x + (b0 + r * Q16_TILE) * 256);
#pragma unroll
            for (int u = 0; u < Q16_TILE * 256 / VPP / 64; ++u) {
                const int e0 = (lane + 64 * u) * VPP;
                V v[VPP];
#pragma unroll
                for (int c = 0; c < VPP; ++c) {
                    const int e = e0 + c, t = e / 256, i = (e / 16) % 16, j = e % 16;
                    v[c] = s_fail[r * Q16_TILE + t] ? nan_value<V>()
                                                    : Xs[t * G16_MAT + i * G16_LD + j];
                }
                uint4 pk;
                __builtin_memcpy(&pk, v, 16);
                dst[lane + 64 * u] = pk;
            }
        } else {
#pragma unroll
            for (int e = lane; e < Q16_TILE * 256; e += 64) {
                const int t = e / 256, i = (e / 16) % 16, j = e % 16;
                const int m = r * Q16_TILE + t;
                const int64_t b = b0 + m;
                if (b < batch && i < n && j < n && (fill || i <= j)) {
                    const V v = s_fail[m] ? nan_value<V>() : Xs[t * G16_MAT + i * G16_LD + j];
                    x[b * sx + (int64_t)i * ldx + j] = v;
                }
            }
        }
    }
}

template <class V, int METHOD, int MIXED>
hipError_t quad16_run(const BatchArgs& p, int n, hipStream_t s)
{
    const int64_t blocks = (p.batch + Q16_MPW - 1) / Q16_MPW;
    hipLaunchKernelGGL((k_quad16<V, METHOD, MIXED>), dim3((unsigned)blocks), dim3(64), 0, s,
                       (const V*)p.a, (V*)p.x, p.batch, n, p.lda, p.sa, p.ldx, p.sx,
                       MIXED ? p.ns_steps : 0, p.fill, p.info);
    return hipGetLastError();
}

template <class V>
hipError_t quad16_dispatch(const BatchArgs& p, int n, int method, int mixed, hipStream_t s)
{
    if (mixed)
        return method == 0 ? quad16_run<V, 0, 1>(p, n, s) : quad16_run<V, 1, 1>(p, n, s);
    return method == 0 ? quad16_run<V, 0, 0>(p, n, s) : quad16_run<V, 1, 0>(p, n, s);
}

}  // namespace

hipError_t launch_quad16(int dtype, int n, int op, int method, int mixed, const BatchArgs& p,
                         hipStream_t s)
{
    if (op != OP_INV || n < 1 || n > 16) return hipErrorNotSupported;
    if (p.batch > (int64_t)Q16_MPW * 0xffffffffLL / 64) return hipErrorInvalidValue;
    switch (dtype) {
    case DT_F32: return quad16_dispatch<float>(p, n, method, mixed, s);
    case DT_C64: return quad16_dispatch<cf>(p, n, method, mixed, s);
    default: return hipErrorNotSupported;
    }
}

}  // namespace ci
