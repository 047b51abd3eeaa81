// tpm_impl.hpp -- batched small-matrix kernels, one lane per matrix ("thread
// per matrix").  Included by one translation unit per element type.
//
// Each lane holds its whole matrix in registers (every loop below is fully
// unrolled on the compile-time order N, so every array index is a constant)
// and runs, with no cross-lane traffic:
//   1. the factorisation, row by row: Cholesky eqs. (3)-(4) or LDL eqs.
//      (10)-(11) (Section II / II.A);
//   2. the proposed back-substitution of Section IV: R X = S, where S is the
//      known upper triangle of the skipped first solve, diag(1/r_ii) (eq. 24)
//      or diag(1/d_i) (eq. 29); only the upper half x_ij, i <= j, is computed
//      and the lower half is its conjugate mirror;
//   3. (mixed precision only) Newton-Schulz steps X <- X + X(I - AX) with the
//      residual I - AX in FP64.
//
// Memory movement.  With dense packing a block's 64 matrices are one
// contiguous chunk of HBM.  The block copies the chunk with 16-byte accesses,
// consecutive lanes on consecutive units (coalesced), into per-lane LDS slots
// that hold only the packed upper triangle (the inverse reads nothing else);
// on the way out the lower half of X is generated from the slot as the
// conjugate mirror.  Slot strides are odd (in elements), which keeps the
// per-lane slot accesses free of bank conflicts.  The persistent kernel
// additionally prefetches its next chunk into registers while it computes.
// The direct variant (any strides) reads each lane's matrix straight from HBM.
#pragma once

#include <algorithm>
#include <utility>

#include "ci_launch.hpp"
#include "ci_types.hpp"

namespace ci {

template <class V>
CI_D typename vt<V>::real sub_abs2_r(typename vt<V>::real acc, V a);
template <> CI_D float sub_abs2_r<float>(float acc, float a) { return fmaf(-a, a, acc); }
template <> CI_D double sub_abs2_r<double>(double acc, double a) { return fma(-a, a, acc); }
template <> CI_D float sub_abs2_r<cf>(float acc, cf a) {
    acc = fmaf(-a.re, a.re, acc);
    return fmaf(-a.im, a.im, acc);
}
template <> CI_D double sub_abs2_r<cd>(double acc, cd a) {
    acc = fma(-a.re, a.re, acc);
    return fma(-a.im, a.im, acc);
}
template <class V>
CI_D typename vt<V>::real abs2_r(V a) {
    return -sub_abs2_r<V>(typename vt<V>::real(0), a);
}

// An empty asm that claims to modify a register value: the compiler must keep
// the value in a VGPR and cannot reuse anything it derived from it before.
// Used so that FP64 copies of A are rebuilt per column instead of all kept live.
#ifndef CI_OPAQUE_DEFINED
#define CI_OPAQUE_DEFINED
CI_D void opaque(float& v) { asm volatile("" : "+v"(v)); }
CI_D void opaque(double& v) { asm volatile("" : "+v"(v)); }
CI_D void opaque(cf& v) { asm volatile("" : "+v"(v.re), "+v"(v.im)); }
CI_D void opaque(cd& v) { asm volatile("" : "+v"(v.re), "+v"(v.im)); }
#endif

// ---- wide memory moves ------------------------------------------------------
template <class V> constexpr int WORDS = sizeof(V) / 4;

template <class V>
CI_D V from_words(const uint32_t* w)
{
    V v;
    __builtin_memcpy(&v, w, sizeof(V));
    return v;
}
template <class V>
CI_D void to_words(V v, uint32_t* w)
{
    __builtin_memcpy(w, &v, sizeof(V));
}

// Largest power-of-two byte width (<= 16) dividing a byte count.
template <int BYTES> constexpr int UNIT = (BYTES % 16 == 0) ? 16 : (BYTES % 8 == 0) ? 8 : 4;

template <int U> struct unit_t;
template <> struct unit_t<16> { using type = uint4; };
template <> struct unit_t<8>  { using type = uint2; };
template <> struct unit_t<4>  { using type = uint32_t; };

template <int U>
CI_D void unit_to_words(const typename unit_t<U>::type& u, uint32_t* w)
{
    __builtin_memcpy(w, &u, U);
}
template <int U>
CI_D typename unit_t<U>::type words_to_unit(const uint32_t* w)
{
    typename unit_t<U>::type u;
    __builtin_memcpy(&u, w, U);
    return u;
}

// One lane loads / stores CNT consecutive elements with the widest accesses.
template <class V, int CNT>
CI_D void load_vec(const V* p, V* out)
{
    constexpr int BYTES = CNT * (int)sizeof(V);
    constexpr int U = UNIT<BYTES>;
    using UT = typename unit_t<U>::type;
    uint32_t w[BYTES / 4];
    const UT* q = reinterpret_cast<const UT*>(p);
#pragma unroll
    for (int k = 0; k < BYTES / U; ++k) {
        const UT u = q[k];
        unit_to_words<U>(u, w + k * (U / 4));
    }
#pragma unroll
    for (int e = 0; e < CNT; ++e) out[e] = from_words<V>(w + e * WORDS<V>);
}

template <class V, int CNT>
CI_D void store_vec(V* p, const V* in)
{
    constexpr int BYTES = CNT * (int)sizeof(V);
    constexpr int U = UNIT<BYTES>;
    using UT = typename unit_t<U>::type;
    uint32_t w[BYTES / 4];
#pragma unroll
    for (int e = 0; e < CNT; ++e) to_words<V>(in[e], w + e * WORDS<V>);
    UT* q = reinterpret_cast<UT*>(p);
#pragma unroll
    for (int k = 0; k < BYTES / U; ++k) q[k] = words_to_unit<U>(w + k * (U / 4));
}

// ---- LDS slot layouts ---------------------------------------------------------
constexpr int odd_at_least(int n) { return n | 1; }

// Packed upper triangle, row by row: (i, j), i <= j.
template <int N>
CI_D constexpr int pidx(int i, int j) { return i * N - (i * (i - 1)) / 2 + (j - i); }

template <int N, bool PACKED> struct Slot;
template <int N> struct Slot<N, true> {
    static constexpr int SIZE = odd_at_least(N * (N + 1) / 2);
};
template <int N> struct Slot<N, false> {
    static constexpr int SIZE = odd_at_least(N * N);
};

// Output policies: where tpm_body writes entry (i, j), i <= j, of its result.
template <class V> struct OutDense {       // row major, optional conjugate mirror
    V* p;
    int64_t ld;
    bool mirror;
    CI_D void put(int i, int j, V v) const {
        p[i * ld + j] = v;
        if (mirror && i < j) p[j * ld + i] = cj(v);
    }
    CI_D V get(int i, int j) const { return p[i * ld + j]; }
};
template <class V, int N> struct OutPacked {  // packed upper slot in LDS
    V* p;
    CI_D void put(int i, int j, V v) const { p[pidx<N>(i, j)] = v; }
    CI_D V get(int i, int j) const { return p[pidx<N>(i, j)]; }
};

// Element e of a block's chunk (matrix e / N^2, entry e % N^2) into its slot;
// PACKED slots keep only i <= j.
template <class V, int N, bool PACKED>
CI_D void unpack_unit(V* sm, int e, const uint32_t* w)
{
    constexpr int NN = N * N, SL = Slot<N, PACKED>::SIZE;
    const int m = e / NN;
    const int q = e - m * NN;
    if constexpr (PACKED) {
        const int i = q / N, j = q - i * N;
        if (j >= i) sm[m * SL + pidx<N>(i, j)] = from_words<V>(w);
    } else {
        sm[m * SL + q] = from_words<V>(w);
    }
}

// Chunk geometries where one row of 16-byte units (64 lanes x 16 bytes) holds
// whole matrices: then unit r of lane t always maps to the same entry of a
// matrix r * (64*16/sizeof(V)/N^2) further on.
template <class V, int N>
constexpr bool REGULAR = (TPM_BLOCK * (16 / (int)sizeof(V))) % (N * N) == 0 &&
                         16 % (int)sizeof(V) == 0;

// Per-lane slot offsets of the EPU elements of a unit (for REGULAR chunks).
template <class V, int N, bool PACKED>
struct SlotMap {
    static constexpr int EPU = 16 / (int)sizeof(V);
    int off[EPU];    // stage_in: slot offset of element c
    bool keep[EPU];  // stage_in: element c is stored (packed: upper triangle)
    int src[EPU];    // stage_out: slot offset that element c is read from
    bool conj[EPU];  // stage_out: conjugate it (mirror of the upper triangle)
    CI_D explicit SlotMap(int t) {
        constexpr int NN = N * N, SL = Slot<N, PACKED>::SIZE;
#pragma unroll
        for (int c = 0; c < EPU; ++c) {
            const int e = t * EPU + c;
            const int m = e / NN, q = e - m * NN;
            const int i = q / N, j = q - i * N;
            if constexpr (PACKED) {
                keep[c] = j >= i;
                off[c] = m * SL + pidx<N>(i, j < i ? i : j);
                src[c] = m * SL + (j >= i ? pidx<N>(i, j) : pidx<N>(j, i));
                conj[c] = j < i;
            } else {
                keep[c] = true;
                off[c] = src[c] = m * SL + q;
                conj[c] = false;
            }
        }
    }
};

// Cooperative copy of a block's contiguous chunk (nvalid matrices of N*N
// elements from batch index b0) into LDS slots.  Whole blocks use 16-byte
// loads, all issued before any LDS write.
template <class V, int N, bool PACKED>
CI_D void stage_in(const V* __restrict__ a, V* sm, int64_t b0, int nvalid, int t)
{
    constexpr int NN = N * N;
    constexpr int BYTES = TPM_BLOCK * NN * (int)sizeof(V);
    constexpr int EPU = 16 / (int)sizeof(V);
    constexpr bool VEC = (BYTES / 16) % TPM_BLOCK == 0;
    constexpr int NU = VEC ? BYTES / 16 / TPM_BLOCK : 1;
    const V* src = a + b0 * NN;
    if (VEC && nvalid == TPM_BLOCK) {
        const uint4* q = reinterpret_cast<const uint4*>(src);
        uint4 u[NU];
#pragma unroll
        for (int r = 0; r < NU; ++r) u[r] = q[r * TPM_BLOCK + t];
        if constexpr (REGULAR<V, N>) {
            // every unit row r covers whole matrices: the slot offsets depend on
            // the lane only, so they are computed once
            SlotMap<V, N, PACKED> mp(t);
#pragma unroll
            for (int r = 0; r < NU; ++r) {
                uint32_t w[4];
                unit_to_words<16>(u[r], w);
                V* base = sm + r * (TPM_BLOCK * EPU / NN) * Slot<N, PACKED>::SIZE;
#pragma unroll
                for (int c = 0; c < EPU; ++c)
                    if (mp.keep[c]) base[mp.off[c]] = from_words<V>(w + c * WORDS<V>);
            }
        } else {
#pragma unroll
            for (int r = 0; r < NU; ++r) {
                uint32_t w[4];
                unit_to_words<16>(u[r], w);
#pragma unroll
                for (int c = 0; c < EPU; ++c)
                    unpack_unit<V, N, PACKED>(sm, (r * TPM_BLOCK + t) * EPU + c, w + c * WORDS<V>);
            }
        }
    } else {
        const int total = nvalid * NN;
        for (int e = t; e < total; e += TPM_BLOCK) {
            uint32_t w[WORDS<V>];
            to_words<V>(src[e], w);
            unpack_unit<V, N, PACKED>(sm, e, w);
        }
    }
}

// Element e of the output chunk from the LDS slots: packed slots give the
// upper triangle and its conjugate mirror.
template <class V, int N, bool PACKED>
CI_D V slot_elem(const V* sm, int e)
{
    constexpr int NN = N * N, SL = Slot<N, PACKED>::SIZE;
    const int m = e / NN;
    const int q = e - m * NN;
    if constexpr (PACKED) {
        const int i = q / N, j = q - i * N;
        return (j >= i) ? sm[m * SL + pidx<N>(i, j)] : cj(sm[m * SL + pidx<N>(j, i)]);
    } else {
        return sm[m * SL + q];
    }
}

// The reverse copy.  With all == false only upper-triangle elements are
// written (an inverse without fill leaves X's strict lower part alone).
template <class V, int N, bool PACKED>
CI_D void stage_out(V* x, const V* sm, int64_t b0, int nvalid, int t, bool all)
{
    constexpr int NN = N * N;
    constexpr int BYTES = TPM_BLOCK * NN * (int)sizeof(V);
    constexpr int EPU = 16 / (int)sizeof(V);
    constexpr bool VEC = (BYTES / 16) % TPM_BLOCK == 0;
    constexpr int NU = VEC ? BYTES / 16 / TPM_BLOCK : 1;
    V* out = x + b0 * NN;
    if (VEC && all && nvalid == TPM_BLOCK) {
        uint4* q = reinterpret_cast<uint4*>(out);
        if constexpr (REGULAR<V, N>) {
            SlotMap<V, N, PACKED> mp(t);
#pragma unroll
            for (int r = 0; r < NU; ++r) {
                uint32_t w[4];
                const V* base = sm + r * (TPM_BLOCK * EPU / NN) * Slot<N, PACKED>::SIZE;
#pragma unroll
                for (int c = 0; c < EPU; ++c) {
                    const V v = base[mp.src[c]];
                    to_words<V>(mp.conj[c] ? cj(v) : v, w + c * WORDS<V>);
                }
                q[r * TPM_BLOCK + t] = words_to_unit<16>(w);
            }
        } else {
#pragma unroll
            for (int r = 0; r < NU; ++r) {
                uint32_t w[4];
#pragma unroll
                for (int c = 0; c < EPU; ++c)
                    to_words<V>(slot_elem<V, N, PACKED>(sm, (r * TPM_BLOCK + t) * EPU + c),
                                w + c * WORDS<V>);
                q[r * TPM_BLOCK + t] = words_to_unit<16>(w);
            }
        }
    } else {
        const int total = nvalid * NN;
        for (int e = t; e < total; e += TPM_BLOCK) {
            const int q = e % NN;
            if (all || (q % N) >= (q / N)) out[e] = slot_elem<V, N, PACKED>(sm, e);
        }
    }
}

// x-hat: the entry (k, j) of the Hermitian X from its computed upper half.
#define XH(k, j) ((k) <= (j) ? X[k][j] : cj(X[j][k]))

// The per-lane computation on a matrix whose upper triangle is in A:
// factorisation, and for OP_INV the Section IV back-substitution and the
// optional Newton-Schulz steps.  Entries (i, j), i <= j, of the result (R,
// or X) go to `out`; with vec_full_store the full X is instead written to
// xfull with wide stores.  Returns info (0 or the 1-based failing pivot).
template <class V, int N, int OP, int METHOD, int MIXED, class Out>
CI_D int tpm_body(V (&A)[N][N], const Out& out, int ns_steps, bool vec_full_store, V* xfull,
                  typename vt<V>::real* dout_b)
{
    using R = typename vt<V>::real;
    using W = typename vt<V>::wide;
    constexpr int NN = N * N;
    int fail = 0;
    // ---------------- factorisation (Section II / II.A) -------------------
    V Rm[N][N];
    R s[N];          // 1/r_ii (eq. 24) or 1/d_i (eq. 29)
    R d[N];          // LDL pivots d_i
    double dd[N];    // LDL pivots in FP64 (mixed)
#pragma unroll
    for (int i = 0; i < N; ++i) {
        if constexpr (METHOD == 0) {
            // eq. (3): r_ii = sqrt(a_ii - sum_{k<i} |r_ki|^2)
            if constexpr (MIXED) {
                double rad = (double)re(A[i][i]);
#pragma unroll
                for (int k = 0; k < i; ++k) rad = sub_abs2_d(rad, Rm[k][i]);
                if (!pivot_ok(rad) && !fail) fail = i + 1;
                double r, y;
                sqrt_rsqrt_est(rad, r, y);
                s[i] = (R)y;
                Rm[i][i] = mk<V>((R)r);
            } else {
                R rad = re(A[i][i]);
#pragma unroll
                for (int k = 0; k < i; ++k) rad = sub_abs2_r<V>(rad, Rm[k][i]);
                if (!pivot_ok(rad) && !fail) fail = i + 1;
                const R r = sqrt(rad);
                s[i] = R(1) / r;
                Rm[i][i] = mk<V>(r);
            }
            // eq. (4): r_ij = (1/r_ii)(a_ij - sum_{k<i} r_ki^* r_kj)
#pragma unroll
            for (int j = i + 1; j < N; ++j) {
                V acc = A[i][j];
#pragma unroll
                for (int k = 0; k < i; ++k) msubc(acc, Rm[k][i], Rm[k][j]);
                Rm[i][j] = scal(acc, s[i]);
            }
        } else {
            // eq. (10): d_i = a_ii - sum_{k<i} r_ki^* r_ki d_k, with the per-row
            // helper t_k = r_ki^* d_k
            V tk[N];
#pragma unroll
            for (int k = 0; k < i; ++k) tk[k] = scal(cj(Rm[k][i]), d[k]);
            R di_r;
            bool ok;
            if constexpr (MIXED) {
                double di = (double)re(A[i][i]);
#pragma unroll
                for (int k = 0; k < i; ++k) di = fma(-dd[k], abs2_d(Rm[k][i]), di);
                dd[i] = di;
                di_r = (R)di;
                s[i] = (R)rcp_est(di);
                ok = (OP == OP_LDL_FACTOR) ? (di != 0.0 && di - di == 0.0) : pivot_ok(di);
            } else {
                R di = re(A[i][i]);
#pragma unroll
                for (int k = 0; k < i; ++k) di = fma(-d[k], abs2_r<V>(Rm[k][i]), di);
                di_r = di;
                s[i] = R(1) / di;
                ok = (OP == OP_LDL_FACTOR) ? (di != R(0) && di - di == R(0)) : pivot_ok(di);
            }
            if (!ok && !fail) fail = i + 1;
            d[i] = di_r;
            Rm[i][i] = mk<V>(R(1));
            // eq. (11): r_ij = (1/d_i)(a_ij - sum_{k<i} r_ki^* r_kj d_k)
#pragma unroll
            for (int j = i + 1; j < N; ++j) {
                V acc = A[i][j];
#pragma unroll
                for (int k = 0; k < i; ++k) msub(acc, tk[k], Rm[k][j]);
                Rm[i][j] = scal(acc, s[i]);
            }
        }
    }

    if constexpr (OP == OP_CHOL_FACTOR || OP == OP_LDL_FACTOR) {
        // upper triangle of A <- R (LDL: strict upper only; d separately)
        constexpr int J0 = (OP == OP_LDL_FACTOR) ? 1 : 0;
#pragma unroll
        for (int i = 0; i < N; ++i)
#pragma unroll
            for (int j = i + J0; j < N; ++j) out.put(i, j, Rm[i][j]);
        if constexpr (OP == OP_LDL_FACTOR) {
#pragma unroll
            for (int i = 0; i < N; ++i) dout_b[i] = d[i];
        }
    } else {
        // ------------- Section IV: R X = S, upper half of X ----------------
        // Rows bottom-up; in row i the off-diagonal entries first (they need
        // rows > i only), then x_ii (it needs x_ik, k > i, of row i).
        V X[N][N];
#pragma unroll
        for (int i = N - 1; i >= 0; --i) {
#pragma unroll
            for (int j = N - 1; j > i; --j) {
                V acc = mk<V>(R(0));
#pragma unroll
                for (int k = i + 1; k < N; ++k) msub(acc, Rm[i][k], XH(k, j));
                X[i][j] = (METHOD == 0) ? scal(acc, s[i]) : acc;
            }
            V acc = mk<V>(s[i]);
#pragma unroll
            for (int k = i + 1; k < N; ++k) msub(acc, Rm[i][k], cj(X[i][k]));
            X[i][i] = realpart_only((METHOD == 0) ? scal(acc, s[i]) : acc);
        }

        if (MIXED && ns_steps > 0) {
            // ------------- Newton-Schulz: X <- X + X(I - A X) ---------------
            // E = I - A X column by column in FP64 (A, X upcast exactly; each
            // upper entry of A is upcast once per column and used for both
            // a_km and a_mk = conj(a_km)); then the upper half of X E in FP32.
            // X + XE = X(2I - AX) is Hermitian.  Column j of the new X goes to
            // `out`; between steps X is read back from there.
            for (int step = 0; step < ns_steps; ++step) {
                if (step > 0) {
#pragma unroll
                    for (int i = 0; i < N; ++i)
#pragma unroll
                        for (int j = i; j < N; ++j) X[i][j] = out.get(i, j);
                }
#pragma unroll
                for (int j = 0; j < N; ++j) {
#pragma unroll
                    for (int k = 0; k < N; ++k)
#pragma unroll
                        for (int m = k; m < N; ++m) opaque(A[k][m]);
                    W xj[N];
                    W e[N];
#pragma unroll
                    for (int m = 0; m < N; ++m) xj[m] = widen(XH(m, j));
#pragma unroll
                    for (int k = 0; k < N; ++k) e[k] = widen(mk<V>(R(k == j ? 1 : 0)));
#pragma unroll
                    for (int k = 0; k < N; ++k) {
                        // a_kk is real: two FMAs
                        const double akk = (double)re(A[k][k]);
                        if constexpr (vt<V>::cplx) {
                            e[k].re = fma(-akk, xj[k].re, e[k].re);
                            e[k].im = fma(-akk, xj[k].im, e[k].im);
                        } else {
                            e[k] = fma(-akk, xj[k], e[k]);
                        }
#pragma unroll
                        for (int m = k + 1; m < N; ++m) {
                            const W akm = widen(A[k][m]);
                            msub(e[k], akm, xj[m]);
                            msubc(e[m], akm, xj[k]);
                        }
                    }
                    V ef[N];
#pragma unroll
                    for (int k = 0; k < N; ++k) ef[k] = narrow<V>(e[k]);
#pragma unroll
                    for (int i = 0; i <= j; ++i) {
                        V acc = X[i][j];
#pragma unroll
                        for (int k = 0; k < N; ++k) madd(acc, XH(i, k), ef[k]);
                        if (i == j) acc = realpart_only(acc);
                        out.put(i, j, acc);
                    }
                }
            }
            if (fail) {
#pragma unroll
                for (int i = 0; i < N; ++i)
#pragma unroll
                    for (int j = i; j < N; ++j) out.put(i, j, nan_value<V>());
            }
        } else {
            if (fail) {
#pragma unroll
                for (int i = 0; i < N; ++i)
#pragma unroll
                    for (int j = i; j < N; ++j) X[i][j] = nan_value<V>();
            }
            if (vec_full_store) {
                V full[NN];
#pragma unroll
                for (int i = 0; i < N; ++i)
#pragma unroll
                    for (int j = i; j < N; ++j) {
                        full[i * N + j] = X[i][j];
                        if (j > i) full[j * N + i] = cj(X[i][j]);
                    }
                store_vec<V, NN>(xfull, full);
            } else {
#pragma unroll
                for (int i = 0; i < N; ++i)
#pragma unroll
                    for (int j = i; j < N; ++j) out.put(i, j, X[i][j]);
            }
        }
    }
    return fail;
}

#undef XH

// One-shot kernel: one block of 64 lanes = 64 matrices.  STAGE: dense chunk
// through LDS (packed slots for the inverse, full slots for the in-place
// factorisations, whose strict lower triangle is written back unchanged).
template <class V, int N, int OP, int METHOD, int MIXED, bool STAGE>
__global__ void __launch_bounds__(TPM_BLOCK)
k_tpm(const V* __restrict__ a, V* x, int64_t batch, int64_t lda, int64_t sa, int64_t ldx,
      int64_t sx, int ns_steps, int fill, int32_t* __restrict__ info,
      typename vt<V>::real* __restrict__ dout)
{
    constexpr int NN = N * N;
    constexpr bool PACKED = (OP == OP_INV);
    constexpr int SL = Slot<N, PACKED>::SIZE;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    V* sm = reinterpret_cast<V*>(smem_raw);

    const int t = threadIdx.x;
    const int64_t b0 = (int64_t)blockIdx.x * TPM_BLOCK;
    const int64_t b = b0 + t;
    const int nvalid = (int)((batch - b0) < TPM_BLOCK ? (batch - b0) : TPM_BLOCK);
    const bool active = t < nvalid;
    // Dense packing without staging: whole matrices with 16-byte accesses.
    const bool dense_direct = !STAGE && lda == N && ldx == N && sa == NN && sx == NN;

    V A[N][N];
    if constexpr (STAGE) {
        stage_in<V, N, PACKED>(a, sm, b0, nvalid, t);
        __syncthreads();
        if (active) {
            const V* slot = sm + t * SL;
#pragma unroll
            for (int i = 0; i < N; ++i)
#pragma unroll
                for (int j = i; j < N; ++j) A[i][j] = PACKED ? slot[pidx<N>(i, j)] : slot[i * N + j];
        }
    } else if (active) {
        if (dense_direct) {
            V full[NN];
            load_vec<V, NN>(a + b * NN, full);    // the lower half is loaded, never used
#pragma unroll
            for (int i = 0; i < N; ++i)
#pragma unroll
                for (int j = i; j < N; ++j) A[i][j] = full[i * N + j];
        } else {
            const V* p = a + b * sa;
#pragma unroll
            for (int i = 0; i < N; ++i)
#pragma unroll
                for (int j = i; j < N; ++j) A[i][j] = p[i * lda + j];
        }
    }

    if (active) {
        typename vt<V>::real* db = dout ? dout + b * N : nullptr;
        int fail;
        if constexpr (STAGE && PACKED) {
            fail = tpm_body<V, N, OP, METHOD, MIXED>(A, OutPacked<V, N>{sm + t * SL}, ns_steps,
                                                     false, nullptr, db);
        } else if constexpr (STAGE) {
            fail = tpm_body<V, N, OP, METHOD, MIXED>(A, OutDense<V>{sm + t * SL, N, false},
                                                     ns_steps, false, nullptr, db);
        } else {
            fail = tpm_body<V, N, OP, METHOD, MIXED>(
                A, OutDense<V>{x + b * sx, ldx, OP == OP_INV && fill != 0}, ns_steps,
                dense_direct && fill && OP == OP_INV, x + b * NN, db);
        }
        if (info) info[b] = fail;
    }

    if constexpr (STAGE) {
        __syncthreads();
        stage_out<V, N, PACKED>(x, sm, b0, nvalid, t, (OP != OP_INV) || fill);
    }
}

// Persistent, software-pipelined form of the staged inverse for dense batches
// of whole 64-matrix chunks: each wave walks the chunks c = blockIdx.x,
// blockIdx.x + gridDim.x, ...; while it computes chunk c, the 16-byte loads of
// its next chunk are already in flight (held in registers P), so HBM traffic
// overlaps the arithmetic.
template <class V, int N, int METHOD, int MIXED>
__global__ void __launch_bounds__(TPM_BLOCK)
k_tpm_persist(const V* __restrict__ a, V* __restrict__ x, int64_t nchunks, int ns_steps,
              int fill, int32_t* __restrict__ info)
{
    constexpr int NN = N * N;
    constexpr int SL = Slot<N, true>::SIZE;
    constexpr int BYTES = TPM_BLOCK * NN * (int)sizeof(V);
    static_assert((BYTES / 16) % TPM_BLOCK == 0, "whole 16-byte units per lane");
    constexpr int EPU = 16 / (int)sizeof(V);
    constexpr int NU = BYTES / 16 / TPM_BLOCK;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    V* sm = reinterpret_cast<V*>(smem_raw);
    const int t = threadIdx.x;

    uint4 P[NU];
    int64_t c = blockIdx.x;
    if (c < nchunks) {
        const uint4* q = reinterpret_cast<const uint4*>(a + c * TPM_BLOCK * NN);
#pragma unroll
        for (int r = 0; r < NU; ++r) P[r] = q[r * TPM_BLOCK + t];
    }
    for (; c < nchunks; c += gridDim.x) {
        if constexpr (REGULAR<V, N>) {
            SlotMap<V, N, true> mp(t);
#pragma unroll
            for (int r = 0; r < NU; ++r) {
                uint32_t w[4];
                unit_to_words<16>(P[r], w);
                V* base = sm + r * (TPM_BLOCK * EPU / NN) * SL;
#pragma unroll
                for (int k = 0; k < EPU; ++k)
                    if (mp.keep[k]) base[mp.off[k]] = from_words<V>(w + k * WORDS<V>);
            }
        } else {
#pragma unroll
            for (int r = 0; r < NU; ++r) {
                uint32_t w[4];
                unit_to_words<16>(P[r], w);
#pragma unroll
                for (int k = 0; k < EPU; ++k)
                    unpack_unit<V, N, true>(sm, (r * TPM_BLOCK + t) * EPU + k, w + k * WORDS<V>);
            }
        }
        __syncthreads();
        const int64_t cn = c + gridDim.x;
        if (cn < nchunks) {
            const uint4* q = reinterpret_cast<const uint4*>(a + cn * TPM_BLOCK * NN);
#pragma unroll
            for (int r = 0; r < NU; ++r) P[r] = q[r * TPM_BLOCK + t];
        }
        V A[N][N];
        const V* slot = sm + t * SL;
#pragma unroll
        for (int i = 0; i < N; ++i)
#pragma unroll
            for (int j = i; j < N; ++j) A[i][j] = slot[pidx<N>(i, j)];
        const int fail = tpm_body<V, N, OP_INV, METHOD, MIXED>(
            A, OutPacked<V, N>{sm + t * SL}, ns_steps, false, nullptr, nullptr);
        if (info) info[c * TPM_BLOCK + t] = fail;
        __syncthreads();
        stage_out<V, N, true>(x, sm, c * TPM_BLOCK, TPM_BLOCK, t, fill != 0);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// dispatch (instantiated per element type by tpm_<type>.hip)
// ---------------------------------------------------------------------------
template <class V, int N, bool PACKED>
constexpr size_t tpm_smem() { return (size_t)TPM_BLOCK * Slot<N, PACKED>::SIZE * sizeof(V); }

template <class V, int N, int OP, int METHOD, int MIXED, bool STAGE>
static hipError_t tpm_run_one(const BatchArgs& p, hipStream_t s)
{
    using R = typename vt<V>::real;
    auto kern = k_tpm<V, N, OP, METHOD, MIXED, STAGE>;
    const size_t smem = STAGE ? tpm_smem<V, N, OP == OP_INV>() : 0;
    if (smem > 65536) {
        static bool once = false;
        if (!once) {
            hipError_t e = hipFuncSetAttribute((const void*)kern,
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)smem);
            if (e != hipSuccess) return e;
            once = true;
        }
    }
    const int64_t blocks = (p.batch + TPM_BLOCK - 1) / TPM_BLOCK;
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(TPM_BLOCK), smem, s,
                       (const V*)p.a, (V*)p.x, p.batch, p.lda, p.sa, p.ldx, p.sx, p.ns_steps,
                       p.fill, p.info, (R*)p.dout);
    return hipGetLastError();
}

// The persistent pipelined kernel on the whole 64-matrix chunks and the
// one-shot staged kernel on the ragged tail.
template <class V, int N, int METHOD, int MIXED>
static hipError_t tpm_run_persist(const BatchArgs& p, hipStream_t s)
{
    auto kern = k_tpm_persist<V, N, METHOD, MIXED>;
    const size_t smem = tpm_smem<V, N, true>();
    const int64_t nchunks = p.batch / TPM_BLOCK;
    if (nchunks > 0) {
        static int blocks_per_cu = -1;
        if (blocks_per_cu < 0) {
            int nb = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)kern, TPM_BLOCK,
                                                             smem) != hipSuccess || nb < 1)
                nb = 1;
            blocks_per_cu = nb;
        }
        const int64_t grid = std::min<int64_t>(nchunks, (int64_t)device_cus() * blocks_per_cu);
        hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(TPM_BLOCK), smem, s, (const V*)p.a,
                           (V*)p.x, nchunks, p.ns_steps, p.fill, p.info);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int64_t done = nchunks * TPM_BLOCK;
    if (done == p.batch) return hipSuccess;
    BatchArgs q = p;
    q.a = (const V*)p.a + done * N * N;
    q.x = (V*)p.x + done * N * N;
    q.batch = p.batch - done;
    q.info = p.info ? p.info + done : nullptr;
    return tpm_run_one<V, N, OP_INV, METHOD, MIXED, true>(q, s);
}

template <class V, int N, int OP, int METHOD, int MIXED>
static hipError_t tpm_run_stage(const BatchArgs& p, hipStream_t s)
{
    // Staging needs dense packing (leading dimension N, stride N*N, same for
    // a and x) and at most 64 KiB of LDS per block.
    constexpr bool fits = tpm_smem<V, N, OP == OP_INV>() <= 65536;
    constexpr bool whole_units = ((size_t)TPM_BLOCK * N * N * sizeof(V) / 16) % TPM_BLOCK == 0;
    const bool dense = p.lda == N && p.ldx == N && p.sa == (int64_t)N * N &&
                       p.sx == (int64_t)N * N;
    if constexpr (fits) {
        const int v = p.variant != VARIANT_AUTO ? p.variant : tpm_default_variant();
        if (dense && v != VARIANT_DIRECT) {
            if constexpr (OP == OP_INV && whole_units) {
                if (v == VARIANT_PERSIST)
                    return tpm_run_persist<V, N, METHOD, MIXED>(p, s);
            }
            return tpm_run_one<V, N, OP, METHOD, MIXED, true>(p, s);
        }
    }
    return tpm_run_one<V, N, OP, METHOD, MIXED, false>(p, s);
}

template <class V, int N>
static hipError_t tpm_run_n(int op, int method, int mixed, const BatchArgs& p, hipStream_t s)
{
    constexpr bool f32 = sizeof(typename vt<V>::real) == 4;
    if (op == OP_INV) {
        if (method == 0) {
            if (mixed) {
                if constexpr (f32) return tpm_run_stage<V, N, OP_INV, 0, 1>(p, s);
                return hipErrorNotSupported;
            }
            return tpm_run_stage<V, N, OP_INV, 0, 0>(p, s);
        }
        if (mixed) {
            if constexpr (f32) return tpm_run_stage<V, N, OP_INV, 1, 1>(p, s);
            return hipErrorNotSupported;
        }
        return tpm_run_stage<V, N, OP_INV, 1, 0>(p, s);
    }
    if (op == OP_CHOL_FACTOR) return tpm_run_stage<V, N, OP_CHOL_FACTOR, 0, 0>(p, s);
    if (op == OP_LDL_FACTOR) return tpm_run_stage<V, N, OP_LDL_FACTOR, 1, 0>(p, s);
    return hipErrorNotSupported;
}

// Orders LO+0 .. LO+len-1.
template <class V, int LO, int... Ns>
static hipError_t tpm_run_range(int n, int op, int method, int mixed, const BatchArgs& p,
                                hipStream_t s, std::integer_sequence<int, Ns...>)
{
    hipError_t r = hipErrorNotSupported;
    ((n == LO + Ns ? (r = tpm_run_n<V, LO + Ns>(op, method, mixed, p, s), 0) : 0), ...);
    return r;
}

}  // namespace ci
