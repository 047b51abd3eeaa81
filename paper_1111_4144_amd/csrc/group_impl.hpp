// group_impl.hpp -- batched small-matrix kernels, G lanes per matrix.
// Included by one translation unit per element type.
//
// The G lanes of a group share one matrix of order n <= NB (a padded bucket:
// entries beyond n are those of the identity, which changes no entry of the
// n x n result).  Columns are dealt cyclically: lane q owns columns
// j = s*G + q (slot s).  Each lane keeps, per owned column, one register
// array M[s][0..NB) that holds
//   * during the factorisation: column j of the partly reduced A, whose
//     entries k <= j become column j of R (right-looking form of eqs. 3-4 or
//     10-11; the FP64 / compute-precision pivot accumulator is separate);
//   * during the Section IV back-substitution, which runs over rows
//     i = NB-1 .. 0: entries k < i still hold R, entries k >= i hold column j
//     of the Hermitian X-hat (x_kj for k <= j, conj(x_jk) for k > j).  Row i of
//     R dies exactly when row i of X is born, so R and X share the storage.
// Row i of R is broadcast from its owners with cross-lane moves inside the
// group (DPP quad_perm / row_newbcast, ds_swizzle or readlane by G).
// Mixed precision keeps column j of A (full Hermitian) for the Newton-Schulz
// residual E = I - A X, accumulated in FP64 one k at a time.
#pragma once

#include <utility>

#include "ci_launch.hpp"
#include "ci_types.hpp"

namespace ci {

#ifndef CI_OPAQUE_DEFINED
#define CI_OPAQUE_DEFINED
// An empty asm that claims to modify a register value: the compiler must keep
// the value in a VGPR and cannot move its producer past this point.
CI_D void opaque(float& v) { asm volatile("" : "+v"(v)); }
CI_D void opaque(double& v) { asm volatile("" : "+v"(v)); }
CI_D void opaque(cf& v) { asm volatile("" : "+v"(v.re), "+v"(v.im)); }
CI_D void opaque(cd& v) { asm volatile("" : "+v"(v.re), "+v"(v.im)); }
#endif

// ---- cross-lane broadcast inside a group of G lanes ---------------------------
template <int G, int K>
CI_D int bc32_k(int v)
{
    static_assert(K >= 0 && K < G, "source lane inside the group");
    if constexpr (G == 1) {
        return v;
    } else if constexpr (G == 2) {
        return __builtin_amdgcn_mov_dpp(v, K | (K << 2) | ((K + 2) << 4) | ((K + 2) << 6), 0xf,
                                        0xf, false);
    } else if constexpr (G == 4) {
        return __builtin_amdgcn_mov_dpp(v, K | (K << 2) | (K << 4) | (K << 6), 0xf, 0xf, false);
    } else if constexpr (G == 8) {
        // ds_swizzle bit mode: lane' = (lane & 0b11000) | K inside each 32 lanes
        return __builtin_amdgcn_ds_swizzle(v, 0x18 | (K << 5));
    } else if constexpr (G == 16) {
        return __builtin_amdgcn_mov_dpp(v, 0x150 + K, 0xf, 0xf, false);   // row_newbcast:K
    } else if constexpr (G == 32) {
        return __builtin_amdgcn_ds_swizzle(v, K << 5);                   // lane' = K
    } else {
        static_assert(G == 64, "group size");
        return __builtin_amdgcn_readlane(v, K);
    }
}

template <int G, int... Ks>
CI_D int bc32_dispatch(int v, int k, std::integer_sequence<int, Ks...>)
{
    int r = v;
    ((k == Ks ? (r = bc32_k<G, Ks>(v), 0) : 0), ...);
    return r;
}

// k must fold to a constant (every caller sits in fully unrolled loops).
template <int G>
CI_D int bc32(int v, int k)
{
    return bc32_dispatch<G>(v, k, std::make_integer_sequence<int, G>{});
}

// 64-bit broadcast inside 16-lane rows: one v_mov_b64 with DPP row_newbcast.
// The tied "old" operand is an unconstrained register from an empty asm (all
// lanes are written, so its value never shows), which avoids a copy.
template <int K>
CI_D long bc64_16_k(long u)
{
    long old;
    asm volatile("" : "=v"(old));
    return __builtin_amdgcn_update_dpp(old, u, 0x150 + K, 0xf, 0xf, false);
}
template <int... Ks>
CI_D long bc64_16_dispatch(long v, int k, std::integer_sequence<int, Ks...>)
{
    long r = v;
    ((k == Ks ? (r = bc64_16_k<Ks>(v), 0) : 0), ...);
    return r;
}
CI_D long bc64_16(long v, int k)
{
    return bc64_16_dispatch(v, k, std::make_integer_sequence<int, 16>{});
}

template <int G> CI_D float bc(float v, int k) { return __builtin_bit_cast(float, bc32<G>(__builtin_bit_cast(int, v), k)); }
template <int G> CI_D double bc(double v, int k) {
    if constexpr (G == 16) {
        return __builtin_bit_cast(double, bc64_16(__builtin_bit_cast(long, v), k));
    } else {
        const uint64_t u = __builtin_bit_cast(uint64_t, v);
        const int lo = bc32<G>((int)(uint32_t)u, k), hi = bc32<G>((int)(uint32_t)(u >> 32), k);
        return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
    }
}
template <int G> CI_D cf bc(cf v, int k) {
    if constexpr (G == 16) return __builtin_bit_cast(cf, bc64_16(__builtin_bit_cast(long, v), k));
    else return cf{bc<G>(v.re, k), bc<G>(v.im, k)};
}
template <int G> CI_D cd bc(cd v, int k) { return cd{bc<G>(v.re, k), bc<G>(v.im, k)}; }
template <int G> CI_D int bci(int v, int k) { return bc32<G>(v, k); }

// Broadcast from a run-time source lane k of the group (k uniform across the
// wave): readlane for whole-wave groups, ds_bpermute otherwise.
template <int G>
CI_D int bcr32(int v, int k)
{
    if constexpr (G == 1) {
        return v;
    } else if constexpr (G == 64) {
        return __builtin_amdgcn_readlane(v, k);
    } else {
        const int src = ((int)(threadIdx.x & 63) & ~(G - 1)) | k;
        return __builtin_amdgcn_ds_bpermute(src << 2, v);
    }
}
template <int G> CI_D float bcr(float v, int k) { return __builtin_bit_cast(float, bcr32<G>(__builtin_bit_cast(int, v), k)); }
template <int G> CI_D double bcr(double v, int k) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const int lo = bcr32<G>((int)(uint32_t)u, k), hi = bcr32<G>((int)(uint32_t)(u >> 32), k);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
template <int G> CI_D cf bcr(cf v, int k) { return cf{bcr<G>(v.re, k), bcr<G>(v.im, k)}; }
template <int G> CI_D cd bcr(cd v, int k) { return cd{bcr<G>(v.re, k), bcr<G>(v.im, k)}; }

template <class V>
CI_D V sel(bool c, V a, V b) { return c ? a : b; }
// Complex values select part by part: a conditional on whole structs becomes
// a copy from a selected address, which keeps the arrays involved in scratch
// memory instead of registers.
CI_D cf sel(bool c, cf a, cf b) { return cf{c ? a.re : b.re, c ? a.im : b.im}; }
CI_D cd sel(bool c, cd a, cd b) { return cd{c ? a.re : b.re, c ? a.im : b.im}; }

// Sum over the 16 lanes of a DPP row, every lane getting the total: quad
// exchanges (xor 1, xor 2), then row_half_mirror (quad 0 <-> 1, 2 <-> 3) and
// row_mirror (half 0 <-> 1).  Each step adds a value and its partner's in
// either order, so all lanes hold bitwise the same sum.
template <int CTRL>
CI_D float dpp_f(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xf,
                                                              0xf, false));
}
template <int CTRL>
CI_D double dpp_f(double v)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)u, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
template <class T>
CI_D T row_sum16(T v)
{
    v += dpp_f<0xB1>(v);    // quad_perm [1, 0, 3, 2]
    v += dpp_f<0x4E>(v);    // quad_perm [2, 3, 0, 1]
    v += dpp_f<0x141>(v);   // row_half_mirror
    v += dpp_f<0x140>(v);   // row_mirror
    return v;
}
CI_D float quad_sumv(float v) { return quad_sum<4>(v); }
CI_D double quad_sumv(double v) { return quad_sum<4>(v); }
CI_D cf quad_sumv(cf v) { return cf{quad_sum<4>(v.re), quad_sum<4>(v.im)}; }
CI_D cd quad_sumv(cd v) { return cd{quad_sum<4>(v.re), quad_sum<4>(v.im)}; }
CI_D float row_sum16v(float v) { return row_sum16(v); }
CI_D double row_sum16v(double v) { return row_sum16(v); }
CI_D cf row_sum16v(cf v) { return cf{row_sum16(v.re), row_sum16(v.im)}; }
CI_D cd row_sum16v(cd v) { return cd{row_sum16(v.re), row_sum16(v.im)}; }

// re(conj(a) b) in precision P (products of FP32 values are exact in FP64)
template <class P> CI_D P dot_re(float a, float b) { return (P)a * (P)b; }
template <class P> CI_D P dot_re(double a, double b) { return (P)(a * b); }
template <class P> CI_D P dot_re(cf a, cf b) { return (P)a.re * (P)b.re + (P)a.im * (P)b.im; }
template <class P> CI_D P dot_re(cd a, cd b) { return (P)(a.re * b.re + a.im * b.im); }

// ---- factorisation and Section IV back-substitution on one group ----------------
// On entry M[s][k] holds column j = s*G + q of A for k <= j (zero below) and
// piv[s] its diagonal entry in the pivot precision P.  On return M holds
// column j of R (factor operations) or of the Hermitian X-hat (OP_INV: x_kj
// for k <= j, conj(x_jk) for k > j), and dall the LDL pivots.  Returns the
// 1-based index of the first failing pivot (0 if none; beyond n for padding
// is impossible since padded pivots are 1).
template <class V, int NB, int G, int OP, int METHOD, int MIXED, int S, class P>
CI_D int group_core(V (&M)[S][NB], P (&piv)[S], typename vt<V>::real (&dall)[NB], int q)
{
    using R = typename vt<V>::real;
    int fail = 0;
    R sall[NB];     // 1/r_ii or 1/d_i, broadcast to every lane
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int qi = i % G, si = i / G;
        // pivot on the owner of column i
        const P pv = piv[si];
        bool ok;
        R rdiag, sinv, dval;
        // results used in FP32 (mixed, or plain FP32) take the estimate forms
        constexpr bool EST = MIXED || sizeof(R) == 4;
        if constexpr (METHOD == 0) {
            ok = pivot_ok(pv);
            if constexpr (EST) {
                P r, y;
                sqrt_rsqrt_est(pv, r, y);
                rdiag = (R)r;
                sinv = (R)y;
            } else {
                const P r = sqrt(pv);
                rdiag = (R)r;
                sinv = (R)(P(1) / r);
            }
            dval = rdiag;
        } else {
            ok = (OP == OP_LDL_FACTOR) ? (pv != P(0) && pv - pv == P(0)) : pivot_ok(pv);
            dval = (R)pv;
            sinv = EST ? (R)rcp_est(pv) : (R)(P(1) / pv);
            rdiag = R(1);
        }
        const int okb = bci<G>(ok ? 1 : 0, qi);
        if (!okb && !fail) fail = i + 1;
        sinv = bc<G>(sinv, qi);
        dval = bc<G>(dval, qi);
        sall[i] = sinv;
        dall[i] = dval;
        // row i of R on every owned column j > i.  The trailing update takes
        // w_ij = r_ij (Cholesky) or the unscaled u_ij = d_i r_ij (LDL):
        //   a_kj -= conj(r_ik) w_ij,   pivot_j -= re(conj(r_ij) w_ij)
        V wv[S];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int j = s * G + q;
            const V u = M[s][i];
            const V r = scal(u, sinv);
            wv[s] = (METHOD == 0) ? r : u;
            M[s][i] = sel(j > i, r, sel(j == i, mk<V>(rdiag), M[s][i]));
            const P dlt = dot_re<P>(r, wv[s]);
            piv[s] = (j > i) ? piv[s] - dlt : piv[s];
        }
#pragma unroll
        for (int k = i + 1; k < NB; ++k) {
            const V rik = bc<G>(M[k / G][i], k % G);
#pragma unroll
            for (int s = 0; s < S; ++s) {
                if (s * G + G - 1 >= k) {
                    msubc(M[s][k], rik, wv[s]);
                    opaque(M[s][k]);   // product next to its broadcast (bounds live ranges)
                }
            }
        }
        __builtin_amdgcn_sched_barrier(0);   // bound live ranges between steps
    }

    if constexpr (OP == OP_INV) {
        // ---- Section IV: rows i = NB-1 .. 0 of R X = S ------------------------
#pragma unroll
        for (int i = NB - 1; i >= 0; --i) {
            const int qi = i % G, si = i / G;
            // (a) x_ij, j > i: -s_i sum_{k>i} r_ik xh_kj (chol) or without s_i (LDL)
            V acc[S];
#pragma unroll
            for (int s = 0; s < S; ++s) acc[s] = mk<V>(R(0));
#pragma unroll
            for (int k = i + 1; k < NB; ++k) {
                // the same broadcast as in factor step i: without the empty asm
                // on its source the compiler reuses that one and keeps all of
                // R's broadcast rows live from the factorisation to here
                V src = M[k / G][i];
                opaque(src);
                const V rik = bc<G>(src, k % G);
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    if (s * G + G - 1 > i) {          // a column j > i in this slot
                        msub(acc[s], rik, M[s][k]);
                        opaque(acc[s]);
                    }
                }
            }
            V xnew[S];
#pragma unroll
            for (int s = 0; s < S; ++s) xnew[s] = (METHOD == 0) ? scal(acc[s], sall[i]) : acc[s];
            // (b) deliver conj(x_ij), j > i, into column i (owner qi, slot si)
#pragma unroll
            for (int j = i + 1; j < NB; ++j) {
                const V v = bc<G>(xnew[j / G], j % G);
                M[si][j] = sel(q == qi, cj(v), M[si][j]);
            }
            // (c) x_ii = s_i (s_i - sum_{k>i} r_ik conj(x_ik)) on the owner; row i
            // of R is still in place (it is replaced only below)
            V d = mk<V>(sall[i]);
            if constexpr (S == 1 && G == 16) {
                // lane k > i holds both r_ik (row i of its column of R) and x_ik
                // (its xnew): one local product each, summed across the row
                V prod = mk<V>(R(0));
                madd(prod, M[0][i], cj(xnew[0]));
                prod = sel(q > i, prod, mk<V>(R(0)));
                d = add(d, neg(row_sum16v(prod)));
            } else if constexpr (G == 4) {
                // the same with four columns per lane: local products over the
                // lane's columns k > i, then a sum over the quad
                V prod = mk<V>(R(0));
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    if (s * G + G - 1 > i) {
                        V t = mk<V>(R(0));
                        madd(t, M[s][i], cj(xnew[s]));
                        prod = add(prod, sel(s * G + q > i, t, mk<V>(R(0))));
                    }
                }
                d = add(d, neg(quad_sumv(prod)));
            } else {
#pragma unroll
                for (int k = i + 1; k < NB; ++k) {
                    // broadcast again rather than keep (a)'s broadcasts live across
                    // (b) (or the factorisation's)
                    V src = M[k / G][i];
                    opaque(src);
                    const V rik = bc<G>(src, k % G);
                    msub(d, rik, M[si][k]);
                    opaque(d);
                }
            }
            d = realpart_only((METHOD == 0) ? scal(d, sall[i]) : d);
            // row i of X replaces row i of R
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const int j = s * G + q;
                M[s][i] = sel(j > i, xnew[s], sel(j == i, d, M[s][i]));
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    return fail;
}

// ---- one matrix per group ------------------------------------------------------
// All G lanes of the group call this together (valid or not: the cross-lane
// moves need every lane); `valid` only gates memory accesses.
template <class V, int NB, int G, int OP, int METHOD, int MIXED>
CI_D void group_matrix(const V* __restrict__ a, int64_t lda, int n, V* x, int64_t ldx, bool valid,
                       int fill, int ns_steps, int q, int32_t* info_b,
                       typename vt<V>::real* dout_b)
{
    using R = typename vt<V>::real;
    using W = typename vt<V>::wide;
    using P = typename std::conditional<MIXED, double, R>::type;   // pivot precision
    constexpr int S = (NB + G - 1) / G;                             // slots per lane

    V M[S][NB];
    V Af[MIXED ? S : 1][MIXED ? NB : 1];
    P piv[S];
#pragma unroll
    for (int s = 0; s < S; ++s) piv[s] = P(1);
    // ---- load column j = s*G + q (upper part from column j, lower part from
    // row j, i.e. only the upper triangle of A is read); identity padding
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int j = s * G + q;
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            V v = mk<V>(R(k == j ? 1 : 0));
            if (valid && j < n && k < n) {
                if (k <= j) v = a[k * lda + j];      // one load, from the upper triangle
                else v = cj(a[j * lda + k]);
                if (k == j) v = realpart_only(v);
            }
            if constexpr (MIXED) Af[s][k] = v;
            M[s][k] = sel(k <= j, v, mk<V>(R(0)));
            if (k == j) piv[s] = (P)re(v);
        }
    }
    R dall[NB];     // LDL pivots
    const int fail = group_core<V, NB, G, OP, METHOD, MIXED>(M, piv, dall, q);

    if constexpr (OP == OP_CHOL_FACTOR || OP == OP_LDL_FACTOR) {
        constexpr int J0 = (OP == OP_LDL_FACTOR) ? 1 : 0;
        if (valid) {
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const int j = s * G + q;
                if (j < n) {
#pragma unroll
                    for (int k = 0; k < NB; ++k)
                        if (k + J0 <= j && k < n) x[k * ldx + j] = M[s][k];
                }
            }
            if constexpr (OP == OP_LDL_FACTOR) {
#pragma unroll
                for (int i = 0; i < NB; ++i)
                    if (i % G == q && i < n) dout_b[i] = dall[i];
            }
        }
    } else {
        // ---- Newton-Schulz: X <- X + X(I - A X), residual in FP64 -------------
        // For every k: e_kj = delta_kj - sum_m a_km xh_mj (FP64, column k of A
        // from its owner; a_km = conj(a_mk)), then X E accumulates
        // upd_ij += xh_ik e_kj for all i (column k of X-hat from its owner).
        if (MIXED && ns_steps > 0) {
            for (int step = 0; step < ns_steps; ++step) {
                V upd[S][NB];
#pragma unroll
                for (int s = 0; s < S; ++s)
#pragma unroll
                    for (int i = 0; i < NB; ++i) upd[s][i] = M[s][i];
                if constexpr (S == 1 && NB > 16) {
                    // one column per lane: the source lane of column k is k itself,
                    // so k can stay a run-time loop (code size NB^2, not NB^3)
#pragma unroll 1
                    for (int k = 0; k < NB; ++k) {
                        W e = widen(mk<V>(R(q == k ? 1 : 0)));
#pragma unroll
                        for (int m = 0; m < NB; ++m)
                            msubc(e, widen(bcr<G>(Af[0][m], k)), widen(M[0][m]));
                        const V ef = narrow<V>(e);
#pragma unroll
                        for (int i2 = 0; i2 < NB; ++i2) madd(upd[0][i2], bcr<G>(M[0][i2], k), ef);
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < NB; ++k) {
                        W e[S];
#pragma unroll
                        for (int s = 0; s < S; ++s) e[s] = widen(mk<V>(R(s * G + q == k ? 1 : 0)));
#pragma unroll
                        for (int m = 0; m < NB; ++m) {
                            const W amk = widen(bc<G>(Af[k / G][m], k % G));   // a_mk
#pragma unroll
                            for (int s = 0; s < S; ++s) {
                                msubc(e[s], amk, widen(M[s][m]));
                                opaque(e[s]);
                            }
                        }
#pragma unroll
                        for (int s = 0; s < S; ++s) {
                            const V ef = narrow<V>(e[s]);
#pragma unroll
                            for (int i2 = 0; i2 < NB; ++i2) {
                                madd(upd[s][i2], bc<G>(M[k / G][i2], k % G), ef);
                                opaque(upd[s][i2]);
                            }
                        }
                        __builtin_amdgcn_sched_barrier(0);
                    }
                }
#pragma unroll
                for (int s = 0; s < S; ++s)
#pragma unroll
                    for (int i = 0; i < NB; ++i) {
                        const int j = s * G + q;
                        M[s][i] = sel(i == j, realpart_only(upd[s][i]), upd[s][i]);
                    }
            }
        }

        // ---- store: column j upper part (i <= j), lower part mirrored from the
        // upper part of the later columns (exactly conjugate)
        if (valid) {
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const int j = s * G + q;
                if (j < n) {
#pragma unroll
                    for (int i = 0; i < NB; ++i) {
                        if (i < n && i <= j) {
                            const V v = sel(fail != 0, nan_value<V>(), M[s][i]);
                            x[i * ldx + j] = v;
                            if (fill && i < j) x[j * ldx + i] = cj(v);
                        }
                    }
                }
            }
        }
    }
    if (valid && q == 0 && info_b) *info_b = (fail > n) ? 0 : fail;
}

// ---- uniform-batch kernel ---------------------------------------------------------
constexpr int GROUP_BLOCK = 256;

template <class V, int NB, int G, int OP, int METHOD, int MIXED>
__global__ void __launch_bounds__(GROUP_BLOCK)
k_group(const V* __restrict__ a, V* x, int64_t batch, int n, int64_t lda, int64_t sa,
        int64_t ldx, int64_t sx, int ns_steps, int fill, int32_t* __restrict__ info,
        typename vt<V>::real* __restrict__ dout)
{
    constexpr int MPB = GROUP_BLOCK / G;
    const int q = threadIdx.x % G;
    const int64_t b = (int64_t)blockIdx.x * MPB + threadIdx.x / G;
    const bool valid = b < batch;
    const int64_t bb = valid ? b : 0;
    group_matrix<V, NB, G, OP, METHOD, MIXED>(a + bb * sa, lda, n, x + bb * sx, ldx, valid, fill,
                                              ns_steps, q, info ? info + bb : nullptr,
                                              dout ? dout + bb * n : nullptr);
}

template <class V, int NB, int G, int OP, int METHOD, int MIXED>
static hipError_t group_run(const BatchArgs& p, int n, hipStream_t s)
{
    using Rt = typename vt<V>::real;
    constexpr int MPB = GROUP_BLOCK / G;
    const int64_t blocks = (p.batch + MPB - 1) / MPB;
    hipLaunchKernelGGL((k_group<V, NB, G, OP, METHOD, MIXED>), dim3((unsigned)blocks),
                       dim3(GROUP_BLOCK), 0, s, (const V*)p.a, (V*)p.x, p.batch, n, p.lda, p.sa,
                       p.ldx, p.sx, p.ns_steps, p.fill, p.info, (Rt*)p.dout);
    return hipGetLastError();
}

template <class V, int NB, int G>
static hipError_t group_run_ops(int n, int op, int method, int mixed, const BatchArgs& p,
                                hipStream_t s)
{
    constexpr bool f32 = sizeof(typename vt<V>::real) == 4;
    if (op == OP_INV) {
        if (mixed) {
            if constexpr (f32) {
                if (method == 0) return group_run<V, NB, G, OP_INV, 0, 1>(p, n, s);
                return group_run<V, NB, G, OP_INV, 1, 1>(p, n, s);
            }
            return hipErrorNotSupported;
        }
        if (method == 0) return group_run<V, NB, G, OP_INV, 0, 0>(p, n, s);
        return group_run<V, NB, G, OP_INV, 1, 0>(p, n, s);
    }
    if (op == OP_CHOL_FACTOR) return group_run<V, NB, G, OP_CHOL_FACTOR, 0, 0>(p, n, s);
    if (op == OP_LDL_FACTOR) return group_run<V, NB, G, OP_LDL_FACTOR, 1, 0>(p, n, s);
    return hipErrorNotSupported;
}

}  // namespace ci
