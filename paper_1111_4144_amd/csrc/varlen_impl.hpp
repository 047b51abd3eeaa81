// varlen_impl.hpp -- persistent launches for a packed batch of matrices of
// uneven orders (1..64).  Included by one translation unit per element type.
//
// Device-side prologue (no host synchronisation, capturable in a HIP graph):
//   1. count   histogram of the orders;
//   2. scan    orders are laid out largest first: per order n its first item
//              in the sorted index list and its tile range;
//   3. scatter every matrix index into the sorted list.
// Tiles: an order n <= 8 tile is up to 64 matrices (one lane each,
// registers); 9..16 up to 16 or 4 matrices (4- or 16-lane groups padded to
// 16 with the identity, which leaves the n x n block exact); 17..32 up to 2
// (LDS-resident, one lane per column) and 33..64 one matrix: one wave on the
// matrix cores for real float by Cholesky without refinement, else four
// waves with four lanes per column (LDS-resident).  The edge of the last
// bucket (33) can move down to 25 or 17 (a tuned choice): those orders then
// go to the last bucket's kernel.  Persistent kernels take tiles from their
// own atomic counters until none are left (every wave reaches that exit):
// first the last bucket (one kernel, or on the matrix cores one per padded
// order 64, 48 and 32), then the rest, largest orders first within each.
// The order of a tile comes from the plan's per-order table held one order
// per lane (a ballot, no dependent loads).  Results do not depend on which
// wave takes which tile.
#pragma once

#include "group_impl.hpp"
#include "leaf_impl.hpp"
#include "tpm_impl.hpp"
#include "wpm_impl.hpp"

namespace ci {

struct VarlenPlan {
    int next;              // tile counter of the orders <= 32 kernel (starts at nbig)
    int ntiles;
    int next_big;          // tile counter of the last bucket's orders 49..64 (starts at 0)
    int next_48;           // the same for its orders 33..48 (starts at tile_end[49])
    int next_32;           // the same for its orders up to 32 (starts at tile_end[33])
    int nbig;              // tiles of orders big_from..64 (one matrix each, first in the order)
    int big_from;          // smallest order of the last bucket (17, 25 or 33)
    int count[65];         // matrices per order
    int item_start[65];    // first position of order n in the sorted list
    int tile_start[65];    // tile range of order n: [tile_start, tile_end)
    int tile_end[65];
    int cursor[65];        // scatter cursors
};

// Lanes per matrix of orders 9..16: four (sixteen matrices a wave) for real
// float without refinement, else sixteen (four a wave; the four-lane form's
// registers would also cap the other orders' occupancy there).
template <class V, int MIXED>
constexpr int vl_g16() { return (std::is_same<V, float>::value && !MIXED) ? 4 : 16; }
CI_D int vl_tile_size(int n, int g16) { return n <= 8 ? 64 : n <= 16 ? 64 / g16 : n <= 32 ? 2 : 1; }

// Order of tile t.  Tiles run largest order first, so the orders whose tile
// range ends at or before t form the top of (lo, 64]; lane l of the wave holds
// te = tile_end of order l + 1, and one ballot counts them (no chain of
// dependent loads).  Every lane of the wave calls this together.
CI_D int vl_order_of(int t, int te, int lo)
{
    const int l = (int)(threadIdx.x % 64);
    return 64 - __popcll(__ballot(l + 1 > lo && t >= te));
}
CI_D int vl_lane_of(int v, int n) { return __builtin_amdgcn_readlane(v, n - 1); }

__global__ void k_vl_init(VarlenPlan* plan)
{
    int* p = reinterpret_cast<int*>(plan);
    for (int i = threadIdx.x; i < (int)(sizeof(VarlenPlan) / sizeof(int)); i += blockDim.x) p[i] = 0;
}

// Orders are counted per block in LDS first, so each block adds to a global
// counter once per order present instead of once per matrix.
__global__ void __launch_bounds__(256)
k_vl_count(const int32_t* __restrict__ ns, int64_t batch, int nmax, VarlenPlan* plan,
           int32_t* __restrict__ info)
{
    __shared__ int local[65];
    for (int t = threadIdx.x; t < 65; t += blockDim.x) local[t] = 0;
    __syncthreads();
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b < batch) {
        const int n = ns[b];
        if (n < 0 || n > nmax) {
            if (info) info[b] = -1;
        } else if (n == 0) {
            if (info) info[b] = 0;
        } else {
            atomicAdd(&local[n], 1);
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < 65; t += blockDim.x)
        if (local[t]) atomicAdd(&plan->count[t], local[t]);
}

__global__ void k_vl_scan(VarlenPlan* plan, int big_from, int g16)
{
    if (threadIdx.x != 0) return;
    int items = 0, tiles = 0;
    plan->big_from = big_from;
    for (int n = 64; n >= 1; --n) {
        const int c = plan->count[n];
        const int ts = n >= big_from ? 1 : vl_tile_size(n, g16);
        plan->item_start[n] = items;
        plan->tile_start[n] = tiles;
        tiles += (c + ts - 1) / ts;
        plan->tile_end[n] = tiles;
        items += c;
    }
    plan->ntiles = tiles;
    plan->nbig = plan->tile_end[big_from];
    plan->next = plan->nbig;
    plan->next_big = 0;
    plan->next_48 = plan->tile_end[49];
    plan->next_32 = plan->tile_end[33];
}

// Each block reserves one contiguous range per order with a single global
// atomic and places its matrices inside it with LDS atomics.  The order of
// matrices within an order's range is therefore not the batch order; results
// do not depend on it.
__global__ void __launch_bounds__(256)
k_vl_scatter(const int32_t* __restrict__ ns, int64_t batch, int nmax, VarlenPlan* plan,
             int32_t* __restrict__ sorted)
{
    __shared__ int local[65], base[65];
    for (int t = threadIdx.x; t < 65; t += blockDim.x) local[t] = 0;
    __syncthreads();
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int n = 0, slot = -1;
    if (b < batch) {
        n = ns[b];
        if (n >= 1 && n <= nmax) slot = atomicAdd(&local[n], 1);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < 65; t += blockDim.x)
        if (local[t]) base[t] = plan->item_start[t] + atomicAdd(&plan->cursor[t], local[t]);
    __syncthreads();
    if (slot >= 0) sorted[base[n] + slot] = (int32_t)b;
}

// One lane, one matrix of order N (dense, leading dimension N).
template <class V, int N, int METHOD, int MIXED>
CI_D int vl_lane(const V* __restrict__ a, V* x, int ns_steps, int fill)
{
    V A[N][N];
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = i; j < N; ++j) A[i][j] = a[i * N + j];
    return tpm_body<V, N, OP_INV, METHOD, MIXED>(A, OutDense<V>{x, N, fill != 0}, ns_steps, false,
                                                 nullptr, nullptr);
}

template <class V, int METHOD, int MIXED>
__global__ void __launch_bounds__(64)
k_varlen(const V* __restrict__ a, V* x, const int64_t* __restrict__ offs,
         const int32_t* __restrict__ sorted, VarlenPlan* plan, int ns_steps, int fill,
         int32_t* __restrict__ info)
{
    constexpr int G16 = vl_g16<V, MIXED>();
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int s_tile;
    const int lane = threadIdx.x;
    // the plan's per-order table, order lane + 1 in lane `lane`
    const int te = plan->tile_end[lane + 1], ts = plan->tile_start[lane + 1];
    const int is = plan->item_start[lane + 1], ct = plan->count[lane + 1];
    const int ntiles = plan->ntiles;
    for (;;) {
        if (lane == 0) s_tile = atomicAdd(&plan->next, 1);
        __syncthreads();
        const int t = s_tile;
        __syncthreads();
        if (t >= ntiles) break;
        const int n = vl_order_of(t, te, 1);
        const int per = vl_tile_size(n, G16);
        const int k = t - vl_lane_of(ts, n);
        const int first = vl_lane_of(is, n) + k * per;
        const int cnt = min(per, vl_lane_of(ct, n) - k * per);
        if (n <= 8) {
            if (lane < cnt) {
                const int b = sorted[first + lane];
                const int64_t o = offs[b];
                int f = 0;
                switch (n) {
                case 1: f = vl_lane<V, 1, METHOD, MIXED>(a + o, x + o, ns_steps, fill); break;
                case 2: f = vl_lane<V, 2, METHOD, MIXED>(a + o, x + o, ns_steps, fill); break;
                case 3: f = vl_lane<V, 3, METHOD, MIXED>(a + o, x + o, ns_steps, fill); break;
                case 4: f = vl_lane<V, 4, METHOD, MIXED>(a + o, x + o, ns_steps, fill); break;
                case 5: f = vl_lane<V, 5, METHOD, MIXED>(a + o, x + o, ns_steps, fill); break;
                case 6: f = vl_lane<V, 6, METHOD, MIXED>(a + o, x + o, ns_steps, fill); break;
                case 7: f = vl_lane<V, 7, METHOD, MIXED>(a + o, x + o, ns_steps, fill); break;
                default: f = vl_lane<V, 8, METHOD, MIXED>(a + o, x + o, ns_steps, fill); break;
                }
                if (info) info[b] = f;
            }
        } else if (n <= 16) {
            const int g = lane / G16;
            const bool valid = g < cnt;
            const int b = sorted[first + (valid ? g : 0)];
            const int64_t o = offs[b];
            group_matrix<V, 16, G16, OP_INV, METHOD, MIXED>(a + o, n, n, x + o, n, valid, fill,
                                                            ns_steps, lane % G16,
                                                            (valid && info) ? info + b : nullptr,
                                                            nullptr);
        } else {
            const int g = lane / 32;
            const bool valid = g < cnt;
            const int b = sorted[first + (valid ? g : 0)];
            const int64_t o = offs[b];
            wpm_matrix<V, 32, OP_INV, METHOD, MIXED>(
                a + o, x + o, n, valid, n, n, ns_steps, fill, (valid && info) ? info + b : nullptr,
                nullptr, smem_raw + (size_t)g * wpm_smem_per_matrix<V, 32, MIXED>(), lane % 32);
        }
        __syncthreads();
    }
}

// Orders big_from..64 (big_from = 33 by default, 17 or 25 when the tuner
// finds it faster): one matrix per 256-lane block, four lanes per column.
constexpr int VL_BIG_TPC = 4;

template <class V, int METHOD, int MIXED>
__global__ void __launch_bounds__(64 * VL_BIG_TPC)
k_varlen_big(const V* __restrict__ a, V* x, const int64_t* __restrict__ offs,
             const int32_t* __restrict__ sorted, VarlenPlan* plan, int ns_steps, int fill,
             int32_t* __restrict__ info)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int s_tile;
    const int j = threadIdx.x / VL_BIG_TPC, h = threadIdx.x % VL_BIG_TPC, l = threadIdx.x % 64;
    const int te = plan->tile_end[l + 1], ts = plan->tile_start[l + 1];
    const int is = plan->item_start[l + 1];
    const int nbig = plan->nbig, lo = plan->big_from;
    for (;;) {
        if (threadIdx.x == 0) s_tile = atomicAdd(&plan->next_big, 1);
        __syncthreads();
        const int t = s_tile;
        __syncthreads();
        if (t >= nbig) break;
        const int n = vl_order_of(t, te, lo);
        const int b = sorted[vl_lane_of(is, n) + (t - vl_lane_of(ts, n))];
        const int64_t o = offs[b];
        wpm_matrix<V, 64, OP_INV, METHOD, MIXED, VL_BIG_TPC>(a + o, x + o, n, true, n, n, ns_steps,
                                                             fill, info ? info + b : nullptr,
                                                             nullptr, smem_raw, j, h);
        __syncthreads();
    }
}

// The last bucket for real float matrices by Cholesky without refinement:
// one wave per matrix, padded with the identity to order NB (64, 48 or 32,
// one launch each), no workgroup barriers, nine to eighteen matrices in
// flight per compute unit.  R and Y = R^{-1} by 16-column sub-blocks: the diagonal sub-block in registers (one lane per
// column, rows reach the other lanes by readlane), its panel row and the
// trailing update as MFMA 16 x 16 x 4 tiles; then the off-diagonal blocks of
// Y bottom-up, Y_{a,>a} = -Y_aa (R_{a,>a} Y_{>a,>a}), and X = Y Y^T (the
// Section III.B product, whose leading operation count equals Section IV's
// once R^{-1} skips its zero blocks), all as MFMA tiles.  One NB x 68 LDS
// array per wave: the upper triangle of A is overwritten by R above the
// diagonal, while Y goes below it transposed (y_ij, i <= j, at row j, column
// i); the diagonal of R is not kept, as only 1/r_ii, the diagonal of Y, is
// used once a diagonal sub-block is done.  X then goes above the diagonal,
// where R was: the off-diagonal tiles as they finish, the diagonal tiles
// (which overwrite the diagonal of Y) last.  Row pitch 68 keeps the MFMA
// operand reads of rows and of columns free of bank conflicts.  A is read
// and X written row by row (one uniform base address per row, all rows of A
// in flight at once), and the next matrix's index and offset are fetched
// while the current one runs.
constexpr int VW_LD = 68;
template <int NB, int MIXED>
constexpr size_t vw_smem()
{
    return (size_t)NB * VW_LD * sizeof(float) + (MIXED ? NB * sizeof(double) : 0);
}

// NB = 64 takes the orders 49..64 (tiles [0, tile_end[49]), counter
// next_big), NB = 48 the orders 33..48 and NB = 32 those below 33 when the
// bucket starts there: less work per matrix and smaller LDS arrays, so
// twelve and eighteen waves per compute unit instead of nine.
template <int NB, int MIXED>
__global__ void __launch_bounds__(64, 3)
k_varlen_wave(const float* __restrict__ a, float* x, const int64_t* __restrict__ offs,
              const int32_t* __restrict__ sorted, VarlenPlan* plan, int fill,
              int32_t* __restrict__ info)
{
    static_assert(NB == 64 || NB == 48 || NB == 32, "padded order");
    constexpr int SB = LF_SB, LD = VW_LD, NSB = NB / SB;
    using Acc = typename mfma_acc<float>::type;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float* M = reinterpret_cast<float*>(smem_raw);
    double* dl = reinterpret_cast<double*>(M + NB * LD);
    const int lane = threadIdx.x, g = lane / 16, cc = lane % 16;
    // y_ij of Y = R^{-1}, zero below its diagonal; Yz once the upper parts of
    // the diagonal blocks hold zeros (every read below Y's diagonal falls
    // there: the operands below never cross blocks that way)
    auto Y = [&](int i, int j) { return i <= j ? M[j * LD + i] : 0.f; };
    auto Yz = [&](int i, int j) { return M[j * LD + i]; };
    auto row = [&](int v) { return mfma_acc<float>::row(g, v); };
    // one wave per workgroup: LDS writes by one lane reach the reads other
    // lanes issue later in program order, so ordering needs no barrier, only
    // that the compiler keeps LDS accesses on their side of this point
    auto wave_sync = [] {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    const int te = plan->tile_end[lane + 1], ts = plan->tile_start[lane + 1];
    const int is = plan->item_start[lane + 1];
    const int lo = plan->big_from;
    // end of this kernel's tile range and its counter
    const int nbig = NB == 64 ? vl_lane_of(te, 49) : NB == 48 ? vl_lane_of(te, 33) : plan->nbig;
    int* const counter = NB == 64 ? &plan->next_big : NB == 48 ? &plan->next_48 : &plan->next_32;
    auto grab = [&]() {
        int v = 0;
        if (lane == 0) v = atomicAdd(counter, 1);
        return __builtin_amdgcn_readfirstlane(v);
    };
    auto item = [&](int tt) {
        const int nn = vl_order_of(tt, te, lo);
        return sorted[vl_lane_of(is, nn) + (tt - vl_lane_of(ts, nn))];
    };
    // the next tile's matrix index and offset are fetched while this one runs
    int t = grab(), b = 0;
    int64_t o = 0;
    if (t < nbig) {
        b = item(t);
        o = offs[b];
    }
    while (t < nbig) {
        const int n = vl_order_of(t, te, lo);
        const float* ab = a + o;
        float* xb = x + o;
        const int t2 = grab();
        const int b2 = t2 < nbig ? item(t2) : 0;
        // rows of A (row k in lanes j < n, one uniform base address per row),
        // all in flight at once; their upper triangle goes to LDS, the
        // identity beyond n.  The lane index goes through an opaque copy so
        // that the per-row masks and addresses are not hoisted out of the loop
        // (they would hold registers for the whole kernel).
        wave_sync();                                     // the last matrix is stored
        {
            int li = lane;
            asm volatile("" : "+v"(li));
            float v[NB];
#pragma unroll
            for (int k = 0; k < NB; ++k) v[k] = (k < n && li < n && k <= li) ? ab[k * n + li] : 0.f;
#pragma unroll
            for (int k = 0; k < NB; ++k)
                if (k <= li && li < NB) M[k * LD + li] = li < n ? v[k] : (k == li ? 1.f : 0.f);
        }
        wave_sync();
        if (MIXED && lane < NB) dl[lane] = lane < n ? (double)M[lane * LD + lane] : 1.0;
        int fail = 0;
        for (int bb = 0; bb < NSB; ++bb) {
            const int b0 = bb * SB, b1 = b0 + SB, nr = NB - b1;
            // ---- diagonal sub-block in registers, one lane per column
            {
                const int j = lane;                          // column b0 + j (lanes >= SB idle)
                float c[SB];
#pragma unroll
                for (int k = 0; k < SB; ++k)
                    c[k] = (j < SB && k <= j) ? M[(b0 + k) * LD + b0 + j] : 0.f;
                double dj = (MIXED && j < SB) ? dl[b0 + j] : 0.0;
                float sv[SB];                                // 1/r_kk, uniform
#pragma unroll
                for (int i = 0; i < SB; ++i) {
                    // the pivot reaches every lane first, so the square
                    // root needs no broadcast after it
                    float s_i, r_ii;
                    bool ok;
                    if constexpr (MIXED) {
                        const double piv = lf_bcast(dj, i);
                        double r, yv;
                        sqrt_rsqrt_est(piv, r, yv);
                        ok = piv > 0.0 && piv < __builtin_inf();
                        s_i = (float)yv;
                        r_ii = (float)r;
                    } else {
                        const float piv = lf_bcast(c[i], i);
                        sqrt_rsqrt_nr(piv, r_ii, s_i);
                        ok = piv > 0.f && piv < __builtin_inff();
                    }
                    if (!ok && !fail && b0 + i < n) fail = b0 + i + 1;
                    sv[i] = s_i;
                    c[i] = (j > i) ? c[i] * s_i : ((j == i) ? r_ii : c[i]);
                    if (MIXED && j > i) dj = fma(-(double)c[i], (double)c[i], dj);
#pragma unroll
                    for (int k = i + 1; k < SB; ++k) c[k] -= lf_bcast(c[i], k) * c[i];
                }
                // R_bb above the diagonal to LDS first: the back-substitution
                // reads its entries from there (one LDS broadcast read each
                // instead of a cross-lane move on the vector unit)
                if (j < SB) {
#pragma unroll
                    for (int k = 0; k < SB; ++k)
                        if (k < j) M[(b0 + k) * LD + b0 + j] = c[k];
                }
                wave_sync();
                // column j of Y_bb bottom-up, y_kj = -s_k sum_{m > k} r_km y_mj,
                // each y_mj added to every row above it as soon as it is known
                // (two dependent operations per row instead of a serial sum)
                float y[SB], acc[SB];
#pragma unroll
                for (int k = 0; k < SB; ++k) acc[k] = 0.f;
#pragma unroll
                for (int m = SB - 1; m >= 0; --m) {
                    y[m] = (j > m) ? -sv[m] * acc[m] : ((j == m) ? sv[m] : 0.f);
#pragma unroll
                    for (int k = 0; k < m; ++k) acc[k] += M[(b0 + k) * LD + b0 + m] * y[m];
                }
                if (j < SB) {
#pragma unroll
                    for (int k = 0; k < SB; ++k)
                        if (k <= j) M[(b0 + j) * LD + b0 + k] = y[k];
                }
            }
            wave_sync();
            if (nr == 0) break;
            // ---- panel row R_{b,>b} = Y_bb^T A_{b,>b}, one column tile at a time
            const int ptn = nr / 16;
            for (int tc = 0; tc < ptn; ++tc) {
                Acc d = Acc{0, 0, 0, 0};
                lf_tile<float>(d, SB, g, cc, [&](int r, int k) { return Y(b0 + k, b0 + r); },
                               [&](int k, int cl) { return M[(b0 + k) * LD + b1 + 16 * tc + cl]; });
#pragma unroll
                for (int v = 0; v < 4; ++v) M[(b0 + row(v)) * LD + b1 + 16 * tc + cc] = d[v];
            }
            wave_sync();
            // ---- FP64 pivots of the remaining columns, and the upper part of
            // A_{>b,>b} -= R_{b,>b}^T R_{b,>b}
            if (MIXED) {
                for (int jj = lane; jj < nr; jj += 64) {
                    double q = dl[b1 + jj];
#pragma unroll 8
                    for (int k = 0; k < SB; ++k) {
                        const double v = (double)M[(b0 + k) * LD + b1 + jj];
                        q = fma(-v, v, q);
                    }
                    dl[b1 + jj] = q;
                }
            }
            for (int tr = 0; tr < ptn; ++tr) {
                for (int tc = tr; tc < ptn; ++tc) {
                    Acc d = Acc{0, 0, 0, 0};
                    lf_tile<float>(d, SB, g, cc,
                                   [&](int r, int k) { return M[(b0 + k) * LD + b1 + 16 * tr + r]; },
                                   [&](int k, int cl) { return M[(b0 + k) * LD + b1 + 16 * tc + cl]; });
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int i = b1 + 16 * tr + row(v), jc = b1 + 16 * tc + cc;
                        if (jc >= i) M[i * LD + jc] -= d[v];
                    }
                }
            }
            wave_sync();
        }
        // R's diagonal blocks are not read again: zero their upper parts
        if (lane < NB) {
#pragma unroll
            for (int u = 0; u < 15; ++u) {
                const int k = (lane & ~15) + u;
                if (k < lane) M[k * LD + lane] = 0.f;
            }
        }
        wave_sync();
        // ---- off-diagonal blocks of Y, block rows bottom-up, one column tile
        // at a time: T = R_{a,>a} Y_{>a,>a}, then Y_{a,>a} = -Y_aa T
        for (int aa = NSB - 2; aa >= 0; --aa) {
            const int a0 = aa * SB, b1 = a0 + SB, ptn = (NB - b1) / 16;
            for (int tc = 0; tc < ptn; ++tc) {
                const int c0 = b1 + 16 * tc;
                Acc d = Acc{0, 0, 0, 0};
                lf_tile<float>(d, 16 * (tc + 1), g, cc,
                               [&](int r, int k) { return M[(a0 + r) * LD + b1 + k]; },
                               [&](int k, int cl) { return Yz(b1 + k, c0 + cl); });
#pragma unroll
                for (int v = 0; v < 4; ++v) M[(c0 + cc) * LD + a0 + row(v)] = d[v];
                wave_sync();
                Acc e = Acc{0, 0, 0, 0};
                lf_tile<float>(e, SB, g, cc, [&](int r, int k) { return Yz(a0 + r, a0 + k); },
                               [&](int k, int cl) { return M[(c0 + cl) * LD + a0 + k]; });
#pragma unroll
                for (int v = 0; v < 4; ++v) M[(c0 + cc) * LD + a0 + row(v)] = -e[v];
                wave_sync();
            }
        }
        const int64_t o2 = t2 < nbig ? offs[b2] : 0;
        // ---- X = Y Y^T: x_ij = sum_{k >= j} y_ik y_jk (i <= j); tile (tr, tc)
        // sums from k = 16 tc
        Acc xd[NSB];
#pragma unroll
        for (int tc = 0; tc < NSB; ++tc) {
#pragma unroll
            for (int tr = 0; tr <= tc; ++tr) {
                Acc d = Acc{0, 0, 0, 0};
                lf_tile<float>(d, NB - 16 * tc, g, cc,
                               [&](int r, int k) { return Yz(16 * tr + r, 16 * tc + k); },
                               [&](int k, int cl) { return Yz(16 * tc + cl, 16 * tc + k); });
                if (tr < tc) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) M[(16 * tr + row(v)) * LD + 16 * tc + cc] = d[v];
                } else {
                    xd[tc] = d;
                }
            }
        }
        wave_sync();
#pragma unroll
        for (int tq = 0; tq < NSB; ++tq) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = 16 * tq + row(v), jc = 16 * tq + cc;
                if (jc >= i) M[i * LD + jc] = xd[tq][v];
            }
        }
        wave_sync();
        // rows of X (row i in lanes j < n, the mirror below the diagonal when
        // filling), read from LDS in batches of sixteen rows before their stores
        int li = lane;
        asm volatile("" : "+v"(li));
#pragma unroll
        for (int i0 = 0; i0 < NB; i0 += 16) {
            float w[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int i = i0 + u;
                w[u] = li >= i ? M[i * LD + li] : M[li * LD + i];
            }
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int i = i0 + u;
                if (i < n && li < n && (li >= i || fill))
                    xb[i * n + li] = fail ? __builtin_nanf("") : w[u];
            }
        }
        if (lane == 0 && info) info[b] = fail;
        t = t2;
        b = b2;
        o = o2;
    }
}

constexpr size_t varlen_plan_bytes() { return (sizeof(VarlenPlan) + 255) / 256 * 256; }

template <class V, int METHOD, int MIXED>
static hipError_t varlen_run(int64_t batch, const int32_t* n_dev, const int64_t* off_dev, int n_max,
                             const void* a, void* x, int ns_steps, int fill, int32_t* info,
                             void* work, hipStream_t s, int big_from)
{
    if (big_from != 17 && big_from != 25) big_from = 33;
    VarlenPlan* plan = reinterpret_cast<VarlenPlan*>(work);
    int32_t* sorted = reinterpret_cast<int32_t*>((char*)work + varlen_plan_bytes());
    const unsigned gb = (unsigned)((batch + 255) / 256);
    hipLaunchKernelGGL(k_vl_init, dim3(1), dim3(256), 0, s, plan);
    hipLaunchKernelGGL(k_vl_count, dim3(gb), dim3(256), 0, s, n_dev, batch, n_max, plan, info);
    hipLaunchKernelGGL(k_vl_scan, dim3(1), dim3(64), 0, s, plan, big_from, vl_g16<V, MIXED>());
    hipLaunchKernelGGL(k_vl_scatter, dim3(gb), dim3(256), 0, s, n_dev, batch, n_max, plan, sorted);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;

    auto kbig = k_varlen_big<V, METHOD, MIXED>;
    auto kern = k_varlen<V, METHOD, MIXED>;
    constexpr size_t s64 = wpm_smem_per_matrix<V, 64, MIXED>();
    constexpr size_t s32 = 2 * wpm_smem_per_matrix<V, 32, MIXED>();
    static bool attr = false;
    if (!attr) {
        e = hipFuncSetAttribute((const void*)kbig, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)s64);
        if (e != hipSuccess) return e;
        e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)s32);
        if (e != hipSuccess) return e;
        attr = true;
    }
    auto grid_of = [](const void* k, int threads, size_t smem) {
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, threads, smem) !=
                hipSuccess || per_cu < 1)
            per_cu = 1;
        return (int64_t)device_cus() * per_cu;
    };
    if (n_max >= big_from) {
        bool leaf = false;       // real float, Cholesky, no refinement: the MFMA route
        if constexpr (std::is_same<V, float>::value && METHOD == 0) {
            leaf = !MIXED || ns_steps == 0;
            if (leaf) {
                auto kw = k_varlen_wave<64, MIXED>;
                constexpr size_t sw = vw_smem<64, MIXED>();
                hipLaunchKernelGGL(kw, dim3((unsigned)grid_of((const void*)kw, 64, sw)), dim3(64), sw,
                                   s, (const float*)a, (float*)x, off_dev, sorted, plan, fill, info);
                auto km = k_varlen_wave<48, MIXED>;
                constexpr size_t sm = vw_smem<48, MIXED>();
                hipLaunchKernelGGL(km, dim3((unsigned)grid_of((const void*)km, 64, sm)), dim3(64), sm,
                                   s, (const float*)a, (float*)x, off_dev, sorted, plan, fill, info);
                if (big_from < 33) {
                    auto ks = k_varlen_wave<32, MIXED>;
                    constexpr size_t ss = vw_smem<32, MIXED>();
                    hipLaunchKernelGGL(ks, dim3((unsigned)grid_of((const void*)ks, 64, ss)), dim3(64),
                                       ss, s, (const float*)a, (float*)x, off_dev, sorted, plan, fill,
                                       info);
                }
            }
        }
        if (!leaf)
            hipLaunchKernelGGL(kbig,
                               dim3((unsigned)grid_of((const void*)kbig, 64 * VL_BIG_TPC, s64)),
                               dim3(64 * VL_BIG_TPC), s64, s, (const V*)a, (V*)x, off_dev, sorted,
                               plan, ns_steps, fill, info);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const size_t smem = n_max > 16 ? s32 : 0;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid_of((const void*)kern, 64, smem)), dim3(64), smem, s,
                       (const V*)a, (V*)x, off_dev, sorted, plan, ns_steps, fill, info);
    return hipGetLastError();
}

template <class V>
static hipError_t varlen_dispatch(int64_t batch, const int32_t* n_dev, const int64_t* off_dev,
                                  int n_max, const void* a, void* x, int method, int mixed,
                                  int ns_steps, int fill, int32_t* info, void* work, hipStream_t s,
                                  int big_from)
{
    constexpr bool f32 = sizeof(typename vt<V>::real) == 4;
    if (mixed) {
        if constexpr (f32) {
            if (method == 0)
                return varlen_run<V, 0, 1>(batch, n_dev, off_dev, n_max, a, x, ns_steps, fill, info,
                                           work, s, big_from);
            return varlen_run<V, 1, 1>(batch, n_dev, off_dev, n_max, a, x, ns_steps, fill, info,
                                       work, s, big_from);
        }
        return hipErrorNotSupported;
    }
    if (method == 0)
        return varlen_run<V, 0, 0>(batch, n_dev, off_dev, n_max, a, x, 0, fill, info, work, s,
                                   big_from);
    return varlen_run<V, 1, 0>(batch, n_dev, off_dev, n_max, a, x, 0, fill, info, work, s,
                               big_from);
}

}  // namespace ci
