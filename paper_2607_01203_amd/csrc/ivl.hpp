// ivl.hpp -- outward-rounded FP32 interval arithmetic for gfx950 (CDNA4).
//
// Every FP32 operation is done in round-to-nearest and its result is then
// pushed outward:  up(p) = p + |p| 2^-23 (+ 2^-126 absolute).  For a normal
// result the relative step is at least one ulp, so it covers the at most
// half-ulp rounding error; the 2^-126 absolute term covers results in (or
// flushed from) the subnormal range.  Exact zeros therefore become tiny
// non-zero bounds; the bound kernels restore exact zeros at term level
// (a term whose displacement factor is exactly [0, 0] is exactly 0).
//
// Operations whose hardware result may be off by up to one ulp (v_rcp_f32,
// v_sqrt_f32) are widened by 8 ulps.  This file must be compiled with
// floating-point contraction off: the widening relies on each product
// being rounded on its own.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace leb {

struct fiv { float lo, hi; };     // FP32 interval
struct div_ { double lo, hi; };   // FP64 interval (accumulators)

__device__ __forceinline__ float up(float p) { return __builtin_fmaf(__builtin_fabsf(p), 0x1p-23f, p) + 0x1p-126f; }
__device__ __forceinline__ float dn(float p) { return __builtin_fmaf(-__builtin_fabsf(p), 0x1p-23f, p) - 0x1p-126f; }
__device__ __forceinline__ float up8(float p) { return __builtin_fmaf(__builtin_fabsf(p), 0x1p-20f, p) + 0x1p-126f; }
__device__ __forceinline__ float dn8(float p) { return __builtin_fmaf(-__builtin_fabsf(p), 0x1p-20f, p) - 0x1p-126f; }

// FP64 -> FP32 rounded down / up (exact for representable values).
__device__ __forceinline__ float rd32(double x) { float f = (float)x; return ((double)f > x) ? dn(f) : f; }
__device__ __forceinline__ float ru32(double x) { float f = (float)x; return ((double)f < x) ? up(f) : f; }

__device__ __forceinline__ fiv mk(float lo, float hi) { fiv r; r.lo = lo; r.hi = hi; return r; }
__device__ __forceinline__ fiv neg(fiv a) { return mk(-a.hi, -a.lo); }
__device__ __forceinline__ fiv add(fiv a, fiv b) { return mk(dn(a.lo + b.lo), up(a.hi + b.hi)); }
__device__ __forceinline__ fiv sub(fiv a, fiv b) { return mk(dn(a.lo - b.hi), up(a.hi - b.lo)); }
// 2a - b and a - 2b (scaling by 2 is exact)
__device__ __forceinline__ fiv twoa_minus_b(fiv a, fiv b) { return mk(dn(2.0f * a.lo - b.hi), up(2.0f * a.hi - b.lo)); }
__device__ __forceinline__ fiv a_minus_twob(fiv a, fiv b) { return mk(dn(a.lo - 2.0f * b.hi), up(a.hi - 2.0f * b.lo)); }

// general product: range of x*y over the two intervals
__device__ __forceinline__ fiv mul(fiv a, fiv b) {
    float p1 = a.lo * b.lo, p2 = a.lo * b.hi, p3 = a.hi * b.lo, p4 = a.hi * b.hi;
    return mk(dn(fminf(fminf(p1, p2), fminf(p3, p4))), up(fmaxf(fmaxf(p1, p2), fmaxf(p3, p4))));
}
// product with b >= 0 (b.lo >= 0)
__device__ __forceinline__ fiv mul_nonneg(fiv a, fiv b) {
    float blo = a.lo >= 0.0f ? b.lo : b.hi;
    float bhi = a.hi >= 0.0f ? b.hi : b.lo;
    return mk(dn(a.lo * blo), up(a.hi * bhi));
}
// product of two non-negative intervals
__device__ __forceinline__ fiv mul_nn(fiv a, fiv b) { return mk(dn(a.lo * b.lo), up(a.hi * b.hi)); }
// product with p containing 0 (p.lo <= 0 <= p.hi): extremes are
// min(a.lo p.hi, a.hi p.lo) and max(a.lo p.lo, a.hi p.hi)
__device__ __forceinline__ fiv mul_z(fiv a, fiv p) {
    return mk(dn(fminf(a.lo * p.hi, a.hi * p.lo)), up(fmaxf(a.lo * p.lo, a.hi * p.hi)));
}
// product of two intervals that both contain 0
__device__ __forceinline__ fiv mul_zz(fiv a, fiv b) {
    return mk(dn(fminf(a.lo * b.hi, a.hi * b.lo)), up(fmaxf(a.lo * b.lo, a.hi * b.hi)));
}
// interval square (never negative)
__device__ __forceinline__ fiv sq(fiv a) {
    float l2 = a.lo * a.lo, h2 = a.hi * a.hi;
    float mx = up(fmaxf(l2, h2));
    if (a.lo >= 0.0f) return mk(dn(l2), up(h2));
    if (a.hi <= 0.0f) return mk(dn(h2), up(l2));
    return mk(0.0f, mx);
}
// square of an interval containing 0
__device__ __forceinline__ fiv sq_z(fiv a) { return mk(0.0f, up(fmaxf(a.lo * a.lo, a.hi * a.hi))); }
// sqrt of a positive interval (v_sqrt_f32: <= 1 ulp)
__device__ __forceinline__ fiv sqrt_pos(fiv a) {
    return mk(fmaxf(dn8(__builtin_amdgcn_sqrtf(a.lo)), 0.0f), up8(__builtin_amdgcn_sqrtf(a.hi)));
}
// 1/a for a positive interval (v_rcp_f32: <= 1 ulp)
__device__ __forceinline__ fiv rcp_pos(fiv a) {
    return mk(fmaxf(dn8(__builtin_amdgcn_rcpf(a.hi)), 0.0f), up8(__builtin_amdgcn_rcpf(a.lo)));
}

// ------------------------------------------------------------ sin / cos
//
// Fast path for |x| <= 0.78 (< pi/4): Taylor polynomials evaluated in FP32.
// Truncation: sin after x^9 leaves <= |x|^11/11! (relative < 2^-28 there);
// cos after x^10 leaves <= x^12/12! (< 2^-32).  Coefficient and Horner
// rounding add a few 2^-24 relative; the result is widened by 2^-20
// relative plus 2^-126 absolute.
__device__ __forceinline__ float sin_poly(float x) {
    float y = x * x;
    float p = __builtin_fmaf(y, 2.7557319e-6f, -1.9841270e-4f);
    p = __builtin_fmaf(p, y, 8.3333333e-3f);
    p = __builtin_fmaf(p, y, -1.6666667e-1f);
    return __builtin_fmaf(x * y, p, x);
}
__device__ __forceinline__ float cos_poly(float x) {
    float y = x * x;
    float p = __builtin_fmaf(y, -2.7557319e-7f, 2.4801587e-5f);
    p = __builtin_fmaf(p, y, -1.3888889e-3f);
    p = __builtin_fmaf(p, y, 4.1666667e-2f);
    p = __builtin_fmaf(p, y, -0.5f);
    return __builtin_fmaf(y, p, 1.0f);
}

// Interval sine and cosine of [a, b] (FP64 endpoints), with the selected
// endpoint of each bound recorded for the adjoint: sel = 0 (endpoint a),
// 1 (endpoint b), 2 (an extremum inside: the bound is the constant +-1).
struct SinCos {
    fiv s, c;
    float fa, fb;          // fast path: FP32 endpoints fed to the polynomials
    uint8_t s_lo, s_hi, c_lo, c_hi;
    bool wide;
};

// FP64 path for wide or far-out intervals: library sin/cos (error far below
// 2^-40 relative for |x| <= 1024), widened by 2^-40 relative plus 2^-100
// absolute, with critical points detected using an outward pi.
__device__ __noinline__ void sincos_wide(double a, double b, SinCos* r) {
    const double PI_LO = 3.141592653589793115997963468544185161590576171875;
    const double PI_HI = 3.141592653589793560087173318606801331043243408203125;
    r->wide = true;
    if (!(b - a < 2.0 * PI_LO) || fabs(a) > 1024.0 || fabs(b) > 1024.0) {
        r->s = mk(-1.0f, 1.0f); r->c = mk(-1.0f, 1.0f);
        r->s_lo = r->s_hi = r->c_lo = r->c_hi = 2;
        return;
    }
    double sa = sin(a), sb = sin(b), ca = cos(a), cb = cos(b);
    auto wdn = [](double x) { return x - fabs(x) * 0x1p-40 - 0x1p-100; };
    auto wup = [](double x) { return x + fabs(x) * 0x1p-40 + 0x1p-100; };
    r->s_lo = sa <= sb ? 0 : 1;
    r->s_hi = sa >= sb ? 0 : 1;
    r->c_lo = ca <= cb ? 0 : 1;
    r->c_hi = ca >= cb ? 0 : 1;
    double slo = wdn(fmin(sa, sb)), shi = wup(fmax(sa, sb));
    double clo = wdn(fmin(ca, cb)), chi = wup(fmax(ca, cb));
    // may [a, b] contain x0 + 2 pi m ?  (slack 1e-12 makes the test err to "yes")
    auto may = [&](double frac) {
        double x0 = frac * PI_LO;
        double m = ceil((a - x0) / (2.0 * PI_HI) - 1e-12);
        double lo_crit = x0 + m * 2.0 * (m >= 0 ? PI_LO : PI_HI);
        return lo_crit <= b + 1e-12;
    };
    if (may(0.5)) { shi = 1.0; r->s_hi = 2; }
    if (may(-0.5)) { slo = -1.0; r->s_lo = 2; }
    if (may(0.0)) { chi = 1.0; r->c_hi = 2; }
    if (may(1.0)) { clo = -1.0; r->c_lo = 2; }
    r->s = mk(fmaxf(rd32(slo), -1.0f), fminf(ru32(shi), 1.0f));
    r->c = mk(fmaxf(rd32(clo), -1.0f), fminf(ru32(chi), 1.0f));
}

__device__ __forceinline__ void isincos(double a, double b, SinCos* r) {
    if (a >= -0.78 && b <= 0.78) {
        r->wide = false;
        const float fa = rd32(a), fb = ru32(b);
        r->fa = fa; r->fb = fb;
        const float sa = sin_poly(fa), sb = sin_poly(fb);        // sin increasing on [-pi/2, pi/2]
        const float ca = cos_poly(fa), cb = cos_poly(fb);
        r->s = mk(dn8(sa), up8(sb));
        r->s_lo = 0; r->s_hi = 1;
        r->c_lo = ca <= cb ? 0 : 1;
        r->c.lo = dn8(fminf(ca, cb));
        if (fa <= 0.0f && fb >= 0.0f) { r->c.hi = 1.0f; r->c_hi = 2; }
        else { r->c.hi = fminf(up8(fmaxf(ca, cb)), 1.0f); r->c_hi = ca >= cb ? 0 : 1; }
    } else {
        // the callee writes a local of this branch only, so the caller's
        // structures stay in registers on the common path
        SinCos w;
        sincos_wide(a, b, &w);
        *r = w;
    }
}

// FP64 accumulation of kappa * T into [lo, hi] (kappa a point).
__device__ __forceinline__ void acc_pos(div_& acc, double kappa, fiv t) {   // kappa >= 0
    acc.lo = __builtin_fma(kappa, (double)t.lo, acc.lo);
    acc.hi = __builtin_fma(kappa, (double)t.hi, acc.hi);
}
__device__ __forceinline__ void acc_neg(div_& acc, double kappa, fiv t) {   // kappa <= 0
    acc.lo = __builtin_fma(kappa, (double)t.hi, acc.lo);
    acc.hi = __builtin_fma(kappa, (double)t.lo, acc.hi);
}
__device__ __forceinline__ void acc_any(div_& acc, double kappa, fiv t) {
    float a = kappa >= 0.0 ? t.lo : t.hi;
    float b = kappa >= 0.0 ? t.hi : t.lo;
    acc.lo = __builtin_fma(kappa, (double)a, acc.lo);
    acc.hi = __builtin_fma(kappa, (double)b, acc.hi);
}

}  // namespace leb
