// ivt.hpp -- interval operations generic over the endpoint type.
//
// F = float: the outward-rounded FP32 interval arithmetic of ivl.hpp.
// F = DF   : the same values plus one tangent (forward-mode derivative).
//            Rounding steps are the identity for tangents (the derivative
//            of the exact-arithmetic formula); selections (min, max, sign
//            branches) follow the values and take the first candidate in
//            the order lo*lo, lo*hi, hi*lo, hi*hi on a tie.
#pragma once
#include "ivl.hpp"

namespace leb {

struct DF { float v, d; };

__device__ __forceinline__ DF dfm(float v, float d) { DF r; r.v = v; r.d = d; return r; }

// scalar layer ----------------------------------------------------------
__device__ __forceinline__ float val(float x) { return x; }
__device__ __forceinline__ float val(DF x) { return x.v; }
__device__ __forceinline__ float tan_(float) { return 0.0f; }
__device__ __forceinline__ float tan_(DF x) { return x.d; }

__device__ __forceinline__ float s_mul(float a, float b) { return a * b; }
__device__ __forceinline__ DF s_mul(DF a, DF b) { return dfm(a.v * b.v, a.d * b.v + a.v * b.d); }
__device__ __forceinline__ float s_add(float a, float b) { return a + b; }
__device__ __forceinline__ DF s_add(DF a, DF b) { return dfm(a.v + b.v, a.d + b.d); }
__device__ __forceinline__ float s_sub(float a, float b) { return a - b; }
__device__ __forceinline__ DF s_sub(DF a, DF b) { return dfm(a.v - b.v, a.d - b.d); }
__device__ __forceinline__ float s_twice(float a) { return 2.0f * a; }
__device__ __forceinline__ DF s_twice(DF a) { return dfm(2.0f * a.v, 2.0f * a.d); }
__device__ __forceinline__ float s_dn(float a) { return dn(a); }
__device__ __forceinline__ DF s_dn(DF a) { return dfm(dn(a.v), a.d); }
__device__ __forceinline__ float s_up(float a) { return up(a); }
__device__ __forceinline__ DF s_up(DF a) { return dfm(up(a.v), a.d); }
__device__ __forceinline__ float s_dn8(float a) { return dn8(a); }
__device__ __forceinline__ DF s_dn8(DF a) { return dfm(dn8(a.v), a.d); }
__device__ __forceinline__ float s_up8(float a) { return up8(a); }
__device__ __forceinline__ DF s_up8(DF a) { return dfm(up8(a.v), a.d); }
// first-on-tie selections
__device__ __forceinline__ float s_min(float a, float b) { return fminf(a, b); }
__device__ __forceinline__ DF s_min(DF a, DF b) { return a.v <= b.v ? a : b; }
__device__ __forceinline__ float s_max(float a, float b) { return fmaxf(a, b); }
__device__ __forceinline__ DF s_max(DF a, DF b) { return a.v >= b.v ? a : b; }
__device__ __forceinline__ float s_sqrt(float a) { return __builtin_amdgcn_sqrtf(a); }
__device__ __forceinline__ DF s_sqrt(DF a) { float r = __builtin_amdgcn_sqrtf(a.v); return dfm(r, a.d * 0.5f / r); }
__device__ __forceinline__ float s_rcp(float a) { return __builtin_amdgcn_rcpf(a); }
__device__ __forceinline__ DF s_rcp(DF a) { float r = __builtin_amdgcn_rcpf(a.v); return dfm(r, -a.d * r * r); }
__device__ __forceinline__ float s_zero(float) { return 0.0f; }
__device__ __forceinline__ DF s_zero(DF) { return dfm(0.0f, 0.0f); }

// intervals -----------------------------------------------------------
template <class F> struct IV { F lo, hi; };
template <class F> __device__ __forceinline__ IV<F> iv(F lo, F hi) { IV<F> r; r.lo = lo; r.hi = hi; return r; }

template <class F> __device__ __forceinline__ IV<F> t_add(IV<F> a, IV<F> b) {
    return iv(s_dn(s_add(a.lo, b.lo)), s_up(s_add(a.hi, b.hi)));
}
template <class F> __device__ __forceinline__ IV<F> t_sub(IV<F> a, IV<F> b) {
    return iv(s_dn(s_sub(a.lo, b.hi)), s_up(s_sub(a.hi, b.lo)));
}
template <class F> __device__ __forceinline__ IV<F> t_twoa_minus_b(IV<F> a, IV<F> b) {
    return iv(s_dn(s_sub(s_twice(a.lo), b.hi)), s_up(s_sub(s_twice(a.hi), b.lo)));
}
template <class F> __device__ __forceinline__ IV<F> t_a_minus_twob(IV<F> a, IV<F> b) {
    return iv(s_dn(s_sub(a.lo, s_twice(b.hi))), s_up(s_sub(a.hi, s_twice(b.lo))));
}
// general product
template <class F> __device__ __forceinline__ IV<F> t_mul(IV<F> a, IV<F> b) {
    F p1 = s_mul(a.lo, b.lo), p2 = s_mul(a.lo, b.hi), p3 = s_mul(a.hi, b.lo), p4 = s_mul(a.hi, b.hi);
    return iv(s_dn(s_min(s_min(p1, p2), s_min(p3, p4))), s_up(s_max(s_max(p1, p2), s_max(p3, p4))));
}
// b >= 0
template <class F> __device__ __forceinline__ IV<F> t_mul_nonneg(IV<F> a, IV<F> b) {
    F lo = val(a.lo) >= 0.0f ? s_mul(a.lo, b.lo) : s_mul(a.lo, b.hi);
    F hi = val(a.hi) >= 0.0f ? s_mul(a.hi, b.hi) : s_mul(a.hi, b.lo);
    return iv(s_dn(lo), s_up(hi));
}
// a, b >= 0
template <class F> __device__ __forceinline__ IV<F> t_mul_nn(IV<F> a, IV<F> b) {
    return iv(s_dn(s_mul(a.lo, b.lo)), s_up(s_mul(a.hi, b.hi)));
}
// p contains 0: lo from (a.lo p.hi, a.hi p.lo), hi from (a.lo p.lo, a.hi p.hi)
template <class F> __device__ __forceinline__ IV<F> t_mul_z(IV<F> a, IV<F> p) {
    return iv(s_dn(s_min(s_mul(a.lo, p.hi), s_mul(a.hi, p.lo))), s_up(s_max(s_mul(a.lo, p.lo), s_mul(a.hi, p.hi))));
}
template <class F> __device__ __forceinline__ IV<F> t_sq(IV<F> a) {
    F l2 = s_mul(a.lo, a.lo), h2 = s_mul(a.hi, a.hi);
    if (val(a.lo) >= 0.0f) return iv(s_dn(l2), s_up(h2));
    if (val(a.hi) <= 0.0f) return iv(s_dn(h2), s_up(l2));
    return iv(s_zero(l2), s_up(s_max(l2, h2)));
}
// a contains 0
template <class F> __device__ __forceinline__ IV<F> t_sq_z(IV<F> a) {
    F l2 = s_mul(a.lo, a.lo), h2 = s_mul(a.hi, a.hi);
    return iv(s_zero(l2), s_up(s_max(l2, h2)));
}
template <class F> __device__ __forceinline__ IV<F> t_sqrt_pos(IV<F> a) {
    F lo = s_dn8(s_sqrt(a.lo));
    if (val(lo) < 0.0f) lo = s_zero(lo);
    return iv(lo, s_up8(s_sqrt(a.hi)));
}
template <class F> __device__ __forceinline__ IV<F> t_rcp_pos(IV<F> a) {
    F lo = s_dn8(s_rcp(a.hi));
    if (val(lo) < 0.0f) lo = s_zero(lo);
    return iv(lo, s_up8(s_rcp(a.lo)));
}

}  // namespace leb
