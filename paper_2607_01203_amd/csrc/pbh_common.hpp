// pbh_common.hpp -- staging helpers shared by the bound and adjoint kernels.
#pragma once
#include "spring.hpp"

namespace leb {

__device__ __forceinline__ double wlo64(double x) { return x - fabs(x) * 0x1p-45; }
__device__ __forceinline__ double whi64(double x) { return x + fabs(x) * 0x1p-45; }

// 1 unless the displacement interval is exactly [0, 0]
__device__ __forceinline__ double maskv(IV<float> d) { return (d.lo != 0.0f || d.hi != 0.0f) ? 1.0 : 0.0; }

// FP64 value with absolute error allowance err -> outward FP32 interval
__device__ __forceinline__ IV<float> from64(double lo, double hi, double err) {
    return iv(rd32(lo - err), ru32(hi + err));
}

// Separations of spring i over its four prefix boxes, formed in FP64 from
// the nominal positions and the displacement intervals, then rounded
// outward to FP32 (the allowance 2^-50 * sum|terms| covers the FP64 sums).
//   dxA: V1, V2 (px_i free)          dxB: V3, V4 (px_i, px_{i+1} free)
//   dz0: V1 (pz point)   dz1: V2, V3 (pz_i free)   dz2: V4 (pz_i, pz_{i+1} free)
struct SpringSetup {
    IV<float> dxA, dxB, dz0, dz1, dz2, Dxi, Dzi, Dxj, Dzj;
    double dxn, dzn;
};

__device__ __forceinline__ void spring_setup_v(double pxi, double pzi, double pxj, double pzj, IV<float> Dxi,
                                              IV<float> Dzi, IV<float> Dxj, IV<float> Dzj, double L0,
                                              SpringSetup& s) {
    s.Dxi = Dxi; s.Dzi = Dzi; s.Dxj = Dxj; s.Dzj = Dzj;
    s.dxn = L0 + pxj - pxi;
    s.dzn = pzj - pzi;
    const double sx = fabs(L0) + fabs(pxj) + fabs(pxi) + fabs(s.Dxi.lo) + fabs(s.Dxi.hi) + fabs(s.Dxj.lo) + fabs(s.Dxj.hi);
    const double sz = fabs(pzj) + fabs(pzi) + fabs(s.Dzi.lo) + fabs(s.Dzi.hi) + fabs(s.Dzj.lo) + fabs(s.Dzj.hi);
    const double ex = sx * 0x1p-50, ez = sz * 0x1p-50;
    const double dxn = s.dxn, dzn = s.dzn;
    s.dxA = from64(dxn - (double)s.Dxi.hi, dxn - (double)s.Dxi.lo, ex);
    s.dxB = from64(dxn + (double)s.Dxj.lo - (double)s.Dxi.hi, dxn + (double)s.Dxj.hi - (double)s.Dxi.lo, ex);
    s.dz0 = from64(dzn, dzn, ez);
    s.dz1 = from64(dzn - (double)s.Dzi.hi, dzn - (double)s.Dzi.lo, ez);
    s.dz2 = from64(dzn + (double)s.Dzj.lo - (double)s.Dzi.hi, dzn + (double)s.Dzj.hi - (double)s.Dzi.lo, ez);
}

__device__ __forceinline__ void spring_setup(const double* nom, const IV<float>* D, int i, double L0, SpringSetup& s) {
    const int pi_ = 6 * i, pj = 6 * (i + 1);
    spring_setup_v(nom[pi_], nom[pi_ + 1], nom[pj], nom[pj + 1], D[pi_], D[pi_ + 1], D[pj], D[pj + 1], L0, s);
}

// Displacement interval Delta = [min(mu - sigma, 0), max(mu + sigma, 0)] of
// one coordinate in FP32; the FP64 difference is widened by its rounding
// bound (exact zeros stay 0).
__device__ __forceinline__ IV<float> disp_interval(double m, double sg) {
    double l = m - sg, h = m + sg;
    l = l - fabs(l) * 0x1p-52;
    h = h + fabs(h) * 0x1p-52;
    return iv(rd32(fmin(l, 0.0)), ru32(fmax(h, 0.0)));
}

}  // namespace leb
