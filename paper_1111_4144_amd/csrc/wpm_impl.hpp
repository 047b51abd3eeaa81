// wpm_impl.hpp -- batched inverse for orders 17..64: a group of G = NB lanes
// (32 or 64) per matrix, the matrix resident in LDS, run-time loops.
// Included by one translation unit per element type.
//
// Lane j owns column j.  All matrices are stored column-major in LDS with a
// padded leading dimension LD (a column is contiguous, so both operands of
// every inner product are read as 16-byte packets: one is the same address for
// all lanes (a broadcast), the other the lane's own column; the padding makes
// the per-lane packet reads bank-conflict free).  Regions (NB x LD each):
//   A  the Hermitian input, both triangles (mixed precision only: kept for the
//      Newton-Schulz residual)
//   W  R during the factorisation (zero below the diagonal), then E = I - A X
//   X  the Hermitian X-hat (both triangles)
// Entries that are not computed yet are exactly zero, so a packet that runs
// past the end of a partial sum adds exact zeros and no masking is needed.
//
// Steps: eqs. (3)-(4) / (10)-(11) in row order (row i of R from rows < i:
// r_ij = (a_ij - sum_{k<i} conj(r_ki) r_kj)/r_ii), the Section IV
// back-substitution over rows i = n-1..0, then (mixed) Newton-Schulz steps.
#pragma once

#include "ci_launch.hpp"
#include "ci_types.hpp"

namespace ci {

template <class V> constexpr int WPM_P = 16 / (int)sizeof(V);                  // elements per packet
template <class V, int NB> constexpr int WPM_LD = NB + WPM_P<V>;                // padded column stride
// Per matrix: the regions plus 2*NB+1 broadcast scalars (1/r_ii or 1/d_i,
// d_i, the pivot flag), rounded to 16 bytes.
template <class V, int NB, int MIXED>
constexpr size_t wpm_smem_per_matrix()
{
    return ((size_t)(MIXED ? 3 : 2) * NB * WPM_LD<V, NB> * sizeof(V) +
            (2 * NB + 1) * sizeof(typename vt<V>::real) + 15) / 16 * 16;
}

// 16-byte packet of P elements
template <class V>
struct Pk { V v[WPM_P<V>]; };

template <class V>
CI_D Pk<V> ldpk(const V* p)
{
    Pk<V> r;
    const uint4 u = *reinterpret_cast<const uint4*>(p);
    __builtin_memcpy(&r, &u, 16);
    return r;
}

// Loop over packets p0, p0 + STRIDE, ... below p1: fetch(p, u, w) loads the two operand packets,
// body(p, u, w) consumes them.  Four packets are fetched before their bodies
// run, so several LDS loads are in flight at once.
template <class V, int STRIDE = 1, class F, class B>
CI_D void pk_loop(int p0, int p1, F fetch, B body)
{
    int p = p0;
    for (; p + 3 * STRIDE < p1; p += 4 * STRIDE) {
        Pk<V> u[4], w[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) fetch(p + q * STRIDE, u[q], w[q]);
#pragma unroll
        for (int q = 0; q < 4; ++q) body(p + q * STRIDE, u[q], w[q]);
    }
    for (; p < p1; p += STRIDE) {
        Pk<V> u, w;
        fetch(p, u, w);
        body(p, u, w);
    }
}

// Sum over the TPC adjacent lanes that share a column.
template <int TPC> CI_D float tpc_sum(float v) { return quad_sum<TPC>(v); }
template <int TPC> CI_D double tpc_sum(double v) { return quad_sum<TPC>(v); }
template <int TPC> CI_D cf tpc_sum(cf v) { return cf{tpc_sum<TPC>(v.re), tpc_sum<TPC>(v.im)}; }
template <int TPC> CI_D cd tpc_sum(cd v) { return cd{tpc_sum<TPC>(v.re), tpc_sum<TPC>(v.im)}; }

// acc -= sum over the packet of conj(a) * b   (P-length partial dot)
template <class V>
CI_D void pk_msubc(V& acc, const Pk<V>& a, const Pk<V>& b)
{
#pragma unroll
    for (int c = 0; c < WPM_P<V>; ++c) msubc(acc, a.v[c], b.v[c]);
}
template <class V>
CI_D void pk_msub(V& acc, const Pk<V>& a, const Pk<V>& b)
{
#pragma unroll
    for (int c = 0; c < WPM_P<V>; ++c) msub(acc, a.v[c], b.v[c]);
}

// One matrix per group of NB * TPC lanes; `lds` is the group's LDS area
// (wpm_smem_per_matrix bytes), j the lane's column and h its index among the
// TPC adjacent lanes of that column: lane h takes packets h, h + TPC, ... of
// every inner product (combined by lane shuffles), and every TPC-th row of
// the loads, stores and refinement loops.  Every lane of the block must call
// this together (it synchronises the block); `valid` only gates global
// memory accesses.
template <class V, int NB, int OP, int METHOD, int MIXED, int TPC = 1>
CI_D void wpm_matrix(const V* __restrict__ ab, V* xb, int n, bool valid, int64_t lda, int64_t ldx,
                     int ns_steps, int fill, int32_t* info_b, typename vt<V>::real* dout_b,
                     unsigned char* lds, int j, int h = 0)
{
    using R = typename vt<V>::real;
    using W = typename vt<V>::wide;
    constexpr int P = WPM_P<V>;
    constexpr int LD = WPM_LD<V, NB>;
    constexpr int REG = NB * LD;
    const int np = (n + P - 1) / P * P;          // padded order (identity)
    V* base = reinterpret_cast<V*>(lds);
    V* Am = MIXED ? base + 2 * REG : nullptr;
    V* Wm = base;
    V* Xm = base + REG;
    R* sv = reinterpret_cast<R*>(base + (MIXED ? 3 : 2) * REG);   // broadcast scalars
    const V zero = mk<V>(R(0));

    // ---- load: column j of the Hermitian A (only the upper triangle is read),
    // identity beyond n; W and X start at zero
    for (int k = h; k < NB; k += TPC) {
        V v = mk<V>(R(k == j ? 1 : 0));
        if (valid && j < n && k < n) {
            v = (k <= j) ? ab[k * lda + j] : cj(ab[j * lda + k]);
            if (k == j) v = realpart_only(v);
        }
        if constexpr (MIXED) Am[j * LD + k] = v;
        Wm[j * LD + k] = (k <= j) ? v : zero;       // a_kj, k <= j; R is built over it
        Xm[j * LD + k] = zero;
    }
    __syncthreads();

    // ---- factorisation in row order (the sums are over completed rows k < i;
    // W column j holds r_kj for k < i and the untouched a_kj for k >= i, so
    // the sums must stop at i: the last packet is masked)
    int fail = 0;
    // mixed: FP64 sum over completed rows k of |r_kj|^2 (Cholesky) or
    // d_k |r_kj|^2 (LDL), accumulated as lane j produces r_kj; the pivot of
    // row j is re(a_jj) minus it
    double sq = 0.0;
    for (int i = 0; i < np; ++i) {
        const V* ci_ = Wm + i * LD;     // column i
        const V* cj_ = Wm + j * LD;     // column j
        V part = zero;                  // this lane's share of the sum
        const int full = i / P;
        pk_loop<V, TPC>(
            h, full,
            [&](int p, Pk<V>& u, Pk<V>& w) {
                u = ldpk(ci_ + p * P);
                w = ldpk(cj_ + p * P);
            },
            [&](int p, const Pk<V>& u, const Pk<V>& w) {
                if constexpr (METHOD == 0) {
                    pk_msubc(part, u, w);
                } else {
                    // LDL: sum conj(r_ki) d_k r_kj with d_k in sv[NB + k]
#pragma unroll
                    for (int c = 0; c < P; ++c)
                        msubc(part, scal(u.v[c], sv[NB + p * P + c]), w.v[c]);
                }
            });
        if (h == 0) {
            for (int k = full * P; k < i; ++k) {
                const V u = ci_[k];
                if constexpr (METHOD == 0) msubc(part, u, cj_[k]);
                else msubc(part, scal(u, sv[NB + k]), cj_[k]);
            }
        }
        const V acc = add(cj_[i], tpc_sum<TPC>(part));   // a_ij - sum (j >= i)
        const double pd = (double)re(cj_[i]) - sq;   // meaningful on lane i only
        // lane i owns the pivot: FP64 when mixed, else the compute precision
        const R prc = MIXED ? (R)pd : re(acc);
        __syncthreads();                       // every lane has read row i inputs
        if (j == i && h == 0) {
            bool ok;
            R sinv, rdiag;
            if constexpr (METHOD == 0) {
                if constexpr (MIXED) {
                    ok = pivot_ok(pd);
                    const double r = sqrt(pd);
                    rdiag = (R)r;
                    sinv = (R)(1.0 / r);
                } else {
                    ok = pivot_ok(prc);
                    rdiag = sqrt(prc);
                    sinv = R(1) / rdiag;
                }
                Wm[i * LD + i] = mk<V>(rdiag);
            } else {
                const double dv = MIXED ? pd : (double)prc;
                ok = (OP == OP_LDL_FACTOR) ? (dv != 0.0 && dv - dv == 0.0) : pivot_ok(dv);
                sinv = (R)(1.0 / dv);
                sv[NB + i] = (R)dv;
                Wm[i * LD + i] = mk<V>(R(1));
            }
            sv[i] = sinv;
            sv[2 * NB] = ok ? R(1) : R(0);
        }
        __syncthreads();
        if (!(sv[2 * NB] > R(0)) && !fail) fail = i + 1;
        if (j > i) {
            const V rij = scal(acc, sv[i]);
            if (h == 0) Wm[j * LD + i] = rij;
            if constexpr (MIXED) {
                if constexpr (METHOD == 0) sq += abs2_d(rij);
                else sq = fma((double)sv[NB + i], abs2_d(rij), sq);
            }
        }
        __syncthreads();
    }

    if constexpr (OP == OP_CHOL_FACTOR || OP == OP_LDL_FACTOR) {
        constexpr int J0 = (OP == OP_LDL_FACTOR) ? 1 : 0;
        if (valid && j < n) {
            for (int k = h; k + J0 <= j; k += TPC) xb[k * ldx + j] = Wm[j * LD + k];
            if constexpr (OP == OP_LDL_FACTOR) if (h == 0) dout_b[j] = sv[NB + j];
        }
        if (valid && j == 0 && h == 0 && info_b) *info_b = fail;
        return;
    } else {
        // ---- Section IV back-substitution, rows i = np-1 .. 0 ----------------
        // Row i of R is copied into the unused lower part of column i of W
        // (W[i][k] = r_ik for k > i), so both operands below are contiguous
        // packets.  Entries k <= i of that column still hold R's column i, but
        // they meet rows <= i of X, which are zero until row i is produced.
        for (int k = h; k < j; k += TPC) Wm[k * LD + j] = Wm[j * LD + k];
        __syncthreads();
        for (int i = np - 1; i >= 0; --i) {
            const R si = sv[i];
            const V* ri = Wm + i * LD;
            const int p0 = (i + 1) / P;
            if (j > i) {
                // x_ij = -s_i sum_{k>i} r_ik xh_kj  (LDL: without s_i)
                V acc = zero;
                const V* xc = Xm + j * LD;
                pk_loop<V, TPC>(
                    p0 + h, np / P,
                    [&](int p, Pk<V>& u, Pk<V>& w) {
                        u = ldpk(ri + p * P);
                        w = ldpk(xc + p * P);
                    },
                    [&](int, const Pk<V>& u, const Pk<V>& w) { pk_msub(acc, u, w); });
                acc = tpc_sum<TPC>(acc);
                const V xij = (METHOD == 0) ? scal(acc, si) : acc;
                if (h == 0) {
                    Xm[j * LD + i] = xij;
                    Xm[i * LD + j] = cj(xij);
                }
            }
            __syncthreads();
            if (j == i) {
                // x_ii = s_i (s_i - sum_{k>i} r_ik conj(x_ik)); X column i rows > i
                // now hold conj(x_ik), rows <= i are zero
                V d = zero;
                const V* xc = Xm + i * LD;
                pk_loop<V, TPC>(
                    p0 + h, np / P,
                    [&](int p, Pk<V>& u, Pk<V>& w) {
                        u = ldpk(ri + p * P);
                        w = ldpk(xc + p * P);
                    },
                    [&](int, const Pk<V>& u, const Pk<V>& w) { pk_msub(d, u, w); });
                d = add(mk<V>(si), tpc_sum<TPC>(d));
                if (h == 0) Xm[i * LD + i] = realpart_only((METHOD == 0) ? scal(d, si) : d);
            }
            __syncthreads();
        }

        // ---- Newton-Schulz steps (mixed): E = I - A X into W (FP64 sums), then
        // X1 = X + X E, written straight to the output; later steps reload X.
        if (MIXED && ns_steps > 0) {
            for (int step = 0; step < ns_steps; ++step) {
                for (int k = h; k < np; k += TPC) {
                    // e_kj = delta_kj - sum_m a_km x_mj = delta - sum_m conj(a_mk) x_mj
                    W e = widen(mk<V>(R(k == j ? 1 : 0)));
                    const V* ak = Am + k * LD;
                    const V* xc = Xm + j * LD;
                    pk_loop<V>(
                        0, np / P,
                        [&](int p, Pk<V>& u, Pk<V>& w) {
                            u = ldpk(ak + p * P);
                            w = ldpk(xc + p * P);
                        },
                        [&](int, const Pk<V>& u, const Pk<V>& w) {
#pragma unroll
                            for (int c = 0; c < P; ++c) msubc(e, widen(u.v[c]), widen(w.v[c]));
                        });
                    Wm[j * LD + k] = narrow<V>(e);
                }
                __syncthreads();
                // X1_ij = x_ij + sum_k x_ik e_kj = x_ij + sum_k conj(x_ki) e_kj; the
                // upper half goes to the output (and is read back by a later step)
                for (int i = h; i < np; i += TPC) {
                    V acc = Xm[j * LD + i];
                    const V* xi = Xm + i * LD;
                    const V* ec = Wm + j * LD;
                    pk_loop<V>(
                        0, np / P,
                        [&](int p, Pk<V>& u, Pk<V>& w) {
                            u = ldpk(xi + p * P);
                            w = ldpk(ec + p * P);
                        },
                        [&](int, const Pk<V>& u, const Pk<V>& w) {
#pragma unroll
                            for (int c = 0; c < P; ++c) madd(acc, cj(u.v[c]), w.v[c]);
                        });
                    if (i == j) acc = realpart_only(acc);
                    if (valid && j < n && i < n && i <= j) {
                        const V v = fail ? nan_value<V>() : acc;
                        xb[i * ldx + j] = v;
                        if (fill && i < j) xb[j * ldx + i] = cj(v);
                    }
                }
                if (step + 1 < ns_steps) {
                    // reload the Hermitian X from the upper half just written
                    __syncthreads();
                    if (valid) {
                        for (int k = h; k < n; k += TPC)
                            if (j < n) Xm[j * LD + k] = (k <= j) ? xb[k * ldx + j] : cj(xb[j * ldx + k]);
                    }
                    __syncthreads();
                }
            }
        } else if (valid && j < n) {
            for (int k = h; k < n; k += TPC) {
                if (k <= j) {
                    const V v = fail ? nan_value<V>() : Xm[j * LD + k];
                    xb[k * ldx + j] = v;
                    if (fill && k < j) xb[j * ldx + k] = cj(v);
                }
            }
        }
        if (valid && j == 0 && h == 0 && info_b) *info_b = fail;
    }
}

// Lanes per column of the uniform-batch kernels: order-64 matrices spread
// over four waves, order-32 pairs over two (more waves in flight for the same
// LDS per matrix).
template <int NB> constexpr int WPM_TPC = NB == 64 ? 4 : 2;

template <class V, int NB, int OP, int METHOD, int MIXED>
__global__ void __launch_bounds__(64 * WPM_TPC<NB>)
k_wpm(const V* __restrict__ a, V* x, int64_t batch, int n, int64_t lda, int64_t sa, int64_t ldx,
      int64_t sx, int ns_steps, int fill, int32_t* __restrict__ info,
      typename vt<V>::real* __restrict__ dout)
{
    constexpr int TPC = WPM_TPC<NB>;
    constexpr int MPB = 64 / NB;                  // matrices per block
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int g = threadIdx.x / (NB * TPC);
    const int r = threadIdx.x % (NB * TPC);
    const int j = r / TPC, h = r % TPC;
    const int64_t b = (int64_t)blockIdx.x * MPB + g;
    const bool valid = b < batch;
    const int64_t bb = valid ? b : 0;
    wpm_matrix<V, NB, OP, METHOD, MIXED, TPC>(
        a + bb * sa, x + bb * sx, n, valid, lda, ldx, ns_steps, fill, info ? info + bb : nullptr,
        dout ? dout + bb * n : nullptr, smem_raw + (size_t)g * wpm_smem_per_matrix<V, NB, MIXED>(),
        j, h);
}

template <class V, int NB, int OP, int METHOD, int MIXED>
static hipError_t wpm_run(const BatchArgs& p, int n, hipStream_t s)
{
    using Rt = typename vt<V>::real;
    constexpr int MPB = 64 / NB;
    const size_t smem = MPB * wpm_smem_per_matrix<V, NB, MIXED>();
    auto kern = k_wpm<V, NB, OP, METHOD, MIXED>;
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
    const int64_t blocks = (p.batch + MPB - 1) / MPB;
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(64 * WPM_TPC<NB>), smem, s, (const V*)p.a,
                       (V*)p.x, p.batch, n, p.lda, p.sa, p.ldx, p.sx, p.ns_steps, p.fill, p.info,
                       (Rt*)p.dout);
    return hipGetLastError();
}

template <class V, int NB>
static hipError_t wpm_run_ops(int n, int op, int method, int mixed, const BatchArgs& p,
                              hipStream_t s)
{
    constexpr bool f32 = sizeof(typename vt<V>::real) == 4;
    if (op == OP_INV) {
        if (mixed) {
            if constexpr (f32) {
                if (method == 0) return wpm_run<V, NB, OP_INV, 0, 1>(p, n, s);
                return wpm_run<V, NB, OP_INV, 1, 1>(p, n, s);
            }
            return hipErrorNotSupported;
        }
        if (method == 0) return wpm_run<V, NB, OP_INV, 0, 0>(p, n, s);
        return wpm_run<V, NB, OP_INV, 1, 0>(p, n, s);
    }
    if (op == OP_CHOL_FACTOR) return wpm_run<V, NB, OP_CHOL_FACTOR, 0, 0>(p, n, s);
    if (op == OP_LDL_FACTOR) return wpm_run<V, NB, OP_LDL_FACTOR, 1, 0>(p, n, s);
    return hipErrorNotSupported;
}

}  // namespace ci
