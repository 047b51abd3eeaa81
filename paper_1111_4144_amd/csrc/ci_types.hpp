// ci_types.hpp -- element types and scalar helpers shared by the gfx950 kernels.
//
// Real elements are float / double; complex elements are the interleaved
// (re, im) pairs cf (complex64) and cd (complex128).  Every helper is written
// with explicit fused multiply-adds so that a complex multiply-accumulate is
// exactly four FMAs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ci {

struct __align__(8) cf { float re, im; };
struct __align__(16) cd { double re, im; };

template <class V> struct vt;
template <> struct vt<float>  { using real = float;  using wide = double; static constexpr bool cplx = false; };
template <> struct vt<double> { using real = double; using wide = double; static constexpr bool cplx = false; };
template <> struct vt<cf>     { using real = float;  using wide = cd;     static constexpr bool cplx = true; };
template <> struct vt<cd>     { using real = double; using wide = cd;     static constexpr bool cplx = true; };

#define CI_D __device__ __forceinline__

// ---- construction / parts --------------------------------------------------
template <class V> CI_D V mk(typename vt<V>::real r);
template <> CI_D float  mk<float>(float r)   { return r; }
template <> CI_D double mk<double>(double r) { return r; }
template <> CI_D cf     mk<cf>(float r)      { return cf{r, 0.f}; }
template <> CI_D cd     mk<cd>(double r)     { return cd{r, 0.0}; }

CI_D float  re(float a)  { return a; }
CI_D double re(double a) { return a; }
CI_D float  re(cf a)     { return a.re; }
CI_D double re(cd a)     { return a.re; }

CI_D float  cj(float a)  { return a; }
CI_D double cj(double a) { return a; }
CI_D cf     cj(cf a)     { return cf{a.re, -a.im}; }
CI_D cd     cj(cd a)     { return cd{a.re, -a.im}; }

CI_D float  realpart_only(float a)  { return a; }
CI_D double realpart_only(double a) { return a; }
CI_D cf     realpart_only(cf a)     { return cf{a.re, 0.f}; }
CI_D cd     realpart_only(cd a)     { return cd{a.re, 0.0}; }

// ---- arithmetic ------------------------------------------------------------
// acc -= a * b
CI_D void msub(float& acc, float a, float b)    { acc = fmaf(-a, b, acc); }
CI_D void msub(double& acc, double a, double b) { acc = fma(-a, b, acc); }
CI_D void msub(cf& acc, cf a, cf b) {
    acc.re = fmaf(-a.re, b.re, acc.re); acc.re = fmaf(a.im, b.im, acc.re);
    acc.im = fmaf(-a.re, b.im, acc.im); acc.im = fmaf(-a.im, b.re, acc.im);
}
CI_D void msub(cd& acc, cd a, cd b) {
    acc.re = fma(-a.re, b.re, acc.re); acc.re = fma(a.im, b.im, acc.re);
    acc.im = fma(-a.re, b.im, acc.im); acc.im = fma(-a.im, b.re, acc.im);
}
// acc -= conj(a) * b
CI_D void msubc(float& acc, float a, float b)    { acc = fmaf(-a, b, acc); }
CI_D void msubc(double& acc, double a, double b) { acc = fma(-a, b, acc); }
CI_D void msubc(cf& acc, cf a, cf b) {
    acc.re = fmaf(-a.re, b.re, acc.re); acc.re = fmaf(-a.im, b.im, acc.re);
    acc.im = fmaf(-a.re, b.im, acc.im); acc.im = fmaf(a.im, b.re, acc.im);
}
CI_D void msubc(cd& acc, cd a, cd b) {
    acc.re = fma(-a.re, b.re, acc.re); acc.re = fma(-a.im, b.im, acc.re);
    acc.im = fma(-a.re, b.im, acc.im); acc.im = fma(a.im, b.re, acc.im);
}
// acc += a * b
CI_D void madd(float& acc, float a, float b)    { acc = fmaf(a, b, acc); }
CI_D void madd(double& acc, double a, double b) { acc = fma(a, b, acc); }
CI_D void madd(cf& acc, cf a, cf b) {
    acc.re = fmaf(a.re, b.re, acc.re); acc.re = fmaf(-a.im, b.im, acc.re);
    acc.im = fmaf(a.re, b.im, acc.im); acc.im = fmaf(a.im, b.re, acc.im);
}
CI_D void madd(cd& acc, cd a, cd b) {
    acc.re = fma(a.re, b.re, acc.re); acc.re = fma(-a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im); acc.im = fma(a.im, b.re, acc.im);
}
// a * s for real s
CI_D float  scal(float a, float s)   { return a * s; }
CI_D double scal(double a, double s) { return a * s; }
CI_D cf     scal(cf a, float s)      { return cf{a.re * s, a.im * s}; }
CI_D cd     scal(cd a, double s)     { return cd{a.re * s, a.im * s}; }
// a + b
CI_D float  add(float a, float b)   { return a + b; }
CI_D double add(double a, double b) { return a + b; }
CI_D cf     add(cf a, cf b)         { return cf{a.re + b.re, a.im + b.im}; }
CI_D cd     add(cd a, cd b)         { return cd{a.re + b.re, a.im + b.im}; }
CI_D float  neg(float a)  { return -a; }
CI_D double neg(double a) { return -a; }
CI_D cf     neg(cf a)     { return cf{-a.re, -a.im}; }
CI_D cd     neg(cd a)     { return cd{-a.re, -a.im}; }

// ---- widening / narrowing (exact up / rounding down) -----------------------
CI_D double widen(float a)  { return (double)a; }
CI_D double widen(double a) { return a; }
CI_D cd     widen(cf a)     { return cd{(double)a.re, (double)a.im}; }
CI_D cd     widen(cd a)     { return a; }
template <class V> CI_D V narrow(typename vt<V>::wide a);
template <> CI_D float  narrow<float>(double a)  { return (float)a; }
template <> CI_D double narrow<double>(double a) { return a; }
template <> CI_D cf     narrow<cf>(cd a)         { return cf{(float)a.re, (float)a.im}; }
template <> CI_D cd     narrow<cd>(cd a)         { return a; }

// |a|^2 accumulated in double: acc - |a|^2 (products of FP32 values are exact)
CI_D double sub_abs2_d(double acc, float a)  { double r = a; return fma(-r, r, acc); }
CI_D double sub_abs2_d(double acc, double a) { return fma(-a, a, acc); }
CI_D double sub_abs2_d(double acc, cf a) {
    double r = a.re, i = a.im;
    acc = fma(-r, r, acc);
    return fma(-i, i, acc);
}
CI_D double sub_abs2_d(double acc, cd a) { acc = fma(-a.re, a.re, acc); return fma(-a.im, a.im, acc); }
// |a|^2 in double (for the LDL pivot d_k |r_ki|^2)
CI_D double abs2_d(float a)  { double r = a; return r * r; }
CI_D double abs2_d(double a) { return a * a; }
CI_D double abs2_d(cf a)     { double r = a.re, i = a.im; return fma(r, r, i * i); }
CI_D double abs2_d(cd a)     { return fma(a.re, a.re, a.im * a.im); }

template <class V> CI_D V nan_value();
template <> CI_D float  nan_value<float>()  { return __builtin_nanf(""); }
template <> CI_D double nan_value<double>() { return __builtin_nan(""); }
template <> CI_D cf     nan_value<cf>()     { return cf{__builtin_nanf(""), __builtin_nanf("")}; }
template <> CI_D cd     nan_value<cd>()     { return cd{__builtin_nan(""), __builtin_nan("")}; }

// r = sqrt(v), s = 1/sqrt(v) and s = 1/v from the hardware estimates
// (v_rsq / v_rcp), for pivots whose results are used in FP32: the FP64 forms
// (mixed precision: FP64 pivots, FP32 factors) add one Newton step, which
// leaves an error far below FP32 rounding; the FP32 forms are within about
// one FP32 ulp.  Non-positive or non-finite v give NaN or infinity (the
// callers flag such pivots separately).
CI_D void sqrt_rsqrt_est(double v, double& r, double& s)
{
    const double y = __builtin_amdgcn_rsq(v);
    s = y * fma(-0.5 * v * y, y, 1.5);
    r = v * s;
}
CI_D void sqrt_rsqrt_est(float v, float& r, float& s)
{
    s = __builtin_amdgcn_rsqf(v);
    r = v * s;
}
// FP32 square root and its reciprocal from the hardware estimate and one
// Newton step on the reciprocal, y <- y + y (1 - v y^2) / 2 (about 1 ulp).
CI_D void sqrt_rsqrt_nr(float v, float& r, float& s)
{
    const float y = __builtin_amdgcn_rsqf(v);
    const float e = fmaf(-(v * y), y, 1.f);
    s = fmaf(0.5f * y, e, y);
    r = v * s;
}
CI_D double rcp_est(double v)
{
    const double y = __builtin_amdgcn_rcp(v);
    return y * fma(-v, y, 2.0);
}
CI_D float rcp_est(float v) { return __builtin_amdgcn_rcpf(v); }

// Sum over TPC = 1, 2 or 4 adjacent lanes (a quad), every lane getting the
// total, with DPP quad permutes (xor 1, then xor 2); partners add in either
// order, so the lanes hold bitwise the same sum.
template <int CTRL>
CI_D float quad_dpp(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xf,
                                                              0xf, false));
}
template <int CTRL>
CI_D double quad_dpp(double v)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)u, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
template <int TPC, class T>
CI_D T quad_sum(T v)
{
    static_assert(TPC == 1 || TPC == 2 || TPC == 4, "lanes per column");
    if constexpr (TPC >= 2) v += quad_dpp<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    if constexpr (TPC == 4) v += quad_dpp<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    return v;
}

CI_D bool pivot_ok(double v) { return v > 0.0 && v < __builtin_inf(); }
CI_D bool pivot_ok(float v)  { return v > 0.f && v < __builtin_inff(); }

}  // namespace ci
