// node.hpp -- the two non-linear rows (vx_i+, vz_i+) of node i in the
// path-based Hessian bound (Theorem 1), shared by the bound kernel and the
// adjoint kernel so both evaluate identical primal values.
//
// Attitude block over the prefix box X^(theta_i) (inputs pinned at the
// nominal point), c = dt/m, s~ = u1~ + u2~:
//   vx: 1/2 c s~ sin(Theta) Dth^2 - c cos(Theta) Dth Du1 - c cos(Theta) Dth Du2
//   vz: -1/2 c s~ cos(Theta) Dth^2 - c sin(Theta) Dth Du1 - c sin(Theta) Dth Du2
// Own position pairs of node i: the right spring (force +F) and the left
// spring (force -F) contribute to the same Hessian entry, so their
// enclosures are subtracted as intervals (G = R - L) before the product
// with the displacement product.
#pragma once
#include "spring.hpp"

namespace leb {

struct NodeTerms {
    SinCos sc;
    IV<float> Ptt, Ptu1, Ptu2, Pxx, Pxz, Pzz;
    IV<float> G[5];         // own pairs: xxx, xxz, xzz (V1-V3), xzz (V2-V4), zzz
    IV<float> T[12];        // terms: 0..5 attitude (x: 0..2, z: 3..5), 6..11 own pairs (x: 6..8, z: 9..11)
    double k[12];           // point factors (masks included)
    uint8_t neg[12];        // 1: factor <= 0 (lower end takes the upper endpoint)
};

// thn, sn: nominal theta and u1 + u2; Dth, Du1, Du2, Dx, Dz: displacement
// intervals; R, L: spring pieces (zeros where a spring is absent); own:
// whether the node has any spring (U > 1).  Masks are 0/1 factors that
// make a term with an exactly-zero displacement factor exactly 0 (1 in the
// adjoint, which differentiates the exact formula).
__device__ __forceinline__ void node_terms(double thn, double sn, IV<float> Dth, IV<float> Du1, IV<float> Du2,
                                           IV<float> Dx, IV<float> Dz, const IV<float>* R, const IV<float>* L,
                                           bool own, double c, double K15, double K1, double K05,
                                           double mth, double mu1, double mu2, double mx, double mz,
                                           NodeTerms& o) {
    const double tlo = thn + (double)Dth.lo, thi = thn + (double)Dth.hi;
    const double et = (fabs(thn) + fabs(Dth.lo) + fabs(Dth.hi)) * 0x1p-51;
    isincos(tlo - et, thi + et, &o.sc);
    const IV<float> S = iv(o.sc.s.lo, o.sc.s.hi), Cs = iv(o.sc.c.lo, o.sc.c.hi);
    o.Ptt = t_sq_z(Dth);
    o.Ptu1 = t_mul_z(Dth, Du1);
    o.Ptu2 = t_mul_z(Dth, Du2);
    const double kth = 0.5 * c * sn * mth;
    o.T[0] = t_mul_z(S, o.Ptt);   o.k[0] = kth;               o.neg[0] = kth < 0.0;
    o.T[1] = t_mul_z(Cs, o.Ptu1); o.k[1] = -c * mth * mu1;    o.neg[1] = 1;
    o.T[2] = t_mul_z(Cs, o.Ptu2); o.k[2] = -c * mth * mu2;    o.neg[2] = 1;
    o.T[3] = t_mul_z(Cs, o.Ptt);  o.k[3] = -kth;              o.neg[3] = -kth < 0.0;
    o.T[4] = t_mul_z(S, o.Ptu1);  o.k[4] = -c * mth * mu1;    o.neg[4] = 1;
    o.T[5] = t_mul_z(S, o.Ptu2);  o.k[5] = -c * mth * mu2;    o.neg[5] = 1;
    if (own) {
        o.Pxx = t_sq_z(Dx);
        o.Pxz = t_mul_z(Dx, Dz);
        o.Pzz = t_sq_z(Dz);
#pragma unroll
        for (int q = 0; q < 5; ++q) o.G[q] = t_sub(R[q], L[q]);
        o.T[6] = t_mul_z(o.G[0], o.Pxx);  o.k[6] = K15 * mx;        o.neg[6] = 0;
        o.T[7] = t_mul_z(o.G[1], o.Pxz);  o.k[7] = -K1 * mx * mz;   o.neg[7] = 1;
        o.T[8] = t_mul_z(o.G[3], o.Pzz);  o.k[8] = K05 * mz;        o.neg[8] = 0;
        o.T[9] = t_mul_z(o.G[1], o.Pxx);  o.k[9] = -K05 * mx;       o.neg[9] = 1;
        o.T[10] = t_mul_z(o.G[2], o.Pxz); o.k[10] = K1 * mx * mz;   o.neg[10] = 0;
        o.T[11] = t_mul_z(o.G[4], o.Pzz); o.k[11] = K15 * mz;       o.neg[11] = 0;
    } else {
#pragma unroll
        for (int q = 6; q < 12; ++q) { o.T[q] = iv(0.0f, 0.0f); o.k[q] = 0.0; o.neg[q] = 0; }
    }
}

// row of term q: 0 (vx) for q in {0,1,2,6,7,8}, 1 (vz) otherwise
__device__ __forceinline__ int node_term_row(int q) { return (q < 3 || (q >= 6 && q < 9)) ? 0 : 1; }

}  // namespace leb
