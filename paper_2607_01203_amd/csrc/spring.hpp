// spring.hpp -- one spring of the planar-quadrotor chain in the path-based
// Hessian bound (Theorem 1), generic over the endpoint type so that the
// bound kernel (F = float) and the tangent passes of the adjoint kernel
// (F = DF) evaluate exactly the same expressions.
//
// Spring i joins nodes i and i+1; its separation is d = (L0 + px_{i+1} -
// px_i, pz_{i+1} - pz_i).  The non-linear part of the force is -k L0 grad|d|,
// so the Hessian of F_x, F_z in d is -k L0 times the symmetric third
// derivative tensor of |d|: with a = dx^2, b = dz^2, s2 = a + b,
// q = 1 / (s2^2 sqrt(s2)):
//   Txxx = 3kL0 dx b q, Txxz = -kL0 dz (2a - b) q, Txzz = kL0 dx (a - 2b) q, Tzzz = 3kL0 dz a q.
// Prefix boxes of the spring's entries (coordinate order px_i < pz_i <
// px_{i+1} < pz_{i+1}): V1 frees px_i, V2 adds pz_i, V3 adds px_{i+1}, V4
// adds pz_{i+1}.  The unit-coefficient enclosures T' (without the kL0
// factor) are evaluated per prefix box; the factor and c = dt/m are applied
// by the accumulator (K3 = 3 kL0 c, K15 = 1.5 kL0 c, K1 = kL0 c,
// K05 = 0.5 kL0 c).
//
// Accumulator slots: CX/CZ cross entries (node i x node i+1, added to row i
// and subtracted from row i+1), BX/BZ node i+1's own position pairs (row i
// only), AX/AZ node i's own position pairs (row i+1 only).  Node i's own
// pairs in row i and node i+1's own pairs in row i+1 are shared with the
// neighbouring spring; their enclosures leave in `R` (right spring of node
// i) and `L` (left spring of node i+1) and are summed by the node.
#pragma once
#include "ivt.hpp"

namespace leb {

enum { S_CX = 0, S_CZ = 1, S_BX = 2, S_BZ = 3, S_AX = 4, S_AZ = 5 };

template <class F> struct SpringPieces {
    IV<F> R[5];   // Txxx V1, Txxz V1, Txzz V1, Txzz V2, Tzzz V2
    IV<F> L[5];   // Txxx V3, Txxz V3, Txzz V3, Txzz V4, Tzzz V4
};

template <class F, class Acc>
__device__ __forceinline__ bool spring_core(IV<F> dxA, IV<F> dxB, IV<F> dz0, IV<F> dz1, IV<F> dz2,
                                            IV<F> Dxi, IV<F> Dzi, IV<F> Dxj, IV<F> Dzj,
                                            double mxi, double mzi, double mxj, double mzj,
                                            double K3, double K15, double K1, double K05,
                                            Acc& acc, SpringPieces<F>& out) {
    const IV<F> aA = t_sq(dxA), aB = t_sq(dxB), b0 = t_sq(dz0), b1 = t_sq(dz1), b2 = t_sq(dz2);
    const IV<F> s1 = t_add(aA, b0), s2 = t_add(aA, b1), s3 = t_add(aB, b1), s4 = t_add(aB, b2);
    const float smin = fminf(fminf(val(s1.lo), val(s2.lo)), fminf(val(s3.lo), val(s4.lo)));
    if (!(smin >= 0x1p-40f)) return false;
    const IV<F> q1 = t_rcp_pos(t_mul_nn(t_mul_nn(s1, s1), t_sqrt_pos(s1)));
    const IV<F> q2 = t_rcp_pos(t_mul_nn(t_mul_nn(s2, s2), t_sqrt_pos(s2)));
    const IV<F> q3 = t_rcp_pos(t_mul_nn(t_mul_nn(s3, s3), t_sqrt_pos(s3)));
    const IV<F> q4 = t_rcp_pos(t_mul_nn(t_mul_nn(s4, s4), t_sqrt_pos(s4)));
    const IV<F> Txxx1 = t_mul_nonneg(dxA, t_mul_nn(b0, q1));
    const IV<F> Txxz1 = t_mul(dz0, t_mul_nonneg(t_twoa_minus_b(aA, b0), q1));
    const IV<F> Txzz1 = t_mul(dxA, t_mul_nonneg(t_a_minus_twob(aA, b0), q1));
    const IV<F> Txxz2 = t_mul(dz1, t_mul_nonneg(t_twoa_minus_b(aA, b1), q2));
    const IV<F> Txzz2 = t_mul(dxA, t_mul_nonneg(t_a_minus_twob(aA, b1), q2));
    const IV<F> Tzzz2 = t_mul_nonneg(dz1, t_mul_nn(aA, q2));
    const IV<F> Txxx3 = t_mul_nonneg(dxB, t_mul_nn(b1, q3));
    const IV<F> Txxz3 = t_mul(dz1, t_mul_nonneg(t_twoa_minus_b(aB, b1), q3));
    const IV<F> Txzz3 = t_mul(dxB, t_mul_nonneg(t_a_minus_twob(aB, b1), q3));
    const IV<F> Txzz4 = t_mul(dxB, t_mul_nonneg(t_a_minus_twob(aB, b2), q4));
    const IV<F> Tzzz4 = t_mul_nonneg(dz2, t_mul_nn(aB, q4));
    // displacement products (every factor contains 0)
    const IV<F> C1 = t_mul_z(Dxi, Dxj), C2 = t_mul_z(Dxi, Dzj), C3 = t_mul_z(Dzi, Dxj), C4 = t_mul_z(Dzi, Dzj);
    const IV<F> Pxxi = t_sq_z(Dxi), Pxzi = t_mul_z(Dxi, Dzi), Pzzi = t_sq_z(Dzi);
    const IV<F> Pxxj = t_sq_z(Dxj), Pxzj = t_mul_z(Dxj, Dzj), Pzzj = t_sq_z(Dzj);
    // cross entries: +row i, -row i+1
    acc.neg(S_CX, -K3 * mxi * mxj, t_mul_z(Txxx1, C1));
    acc.pos(S_CX, K1 * mxi * mzj, t_mul_z(Txxz1, C2));
    acc.pos(S_CX, K1 * mzi * mxj, t_mul_z(Txxz2, C3));
    acc.neg(S_CX, -K1 * mzi * mzj, t_mul_z(Txzz2, C4));
    acc.pos(S_CZ, K1 * mxi * mxj, t_mul_z(Txxz1, C1));
    acc.neg(S_CZ, -K1 * mxi * mzj, t_mul_z(Txzz1, C2));
    acc.neg(S_CZ, -K1 * mzi * mxj, t_mul_z(Txzz2, C3));
    acc.neg(S_CZ, -K3 * mzi * mzj, t_mul_z(Tzzz2, C4));
    // row i: node i+1's own position pairs
    acc.pos(S_BX, K15 * mxj, t_mul_z(Txxx3, Pxxj));
    acc.neg(S_BX, -K1 * mxj * mzj, t_mul_z(Txxz3, Pxzj));
    acc.pos(S_BX, K05 * mzj, t_mul_z(Txzz4, Pzzj));
    acc.neg(S_BZ, -K05 * mxj, t_mul_z(Txxz3, Pxxj));
    acc.pos(S_BZ, K1 * mxj * mzj, t_mul_z(Txzz3, Pxzj));
    acc.pos(S_BZ, K15 * mzj, t_mul_z(Tzzz4, Pzzj));
    // row i+1: node i's own position pairs
    acc.pos(S_AX, K15 * mxi, t_mul_z(Txxx1, Pxxi));
    acc.neg(S_AX, -K1 * mxi * mzi, t_mul_z(Txxz1, Pxzi));
    acc.pos(S_AX, K05 * mzi, t_mul_z(Txzz2, Pzzi));
    acc.neg(S_AZ, -K05 * mxi, t_mul_z(Txxz1, Pxxi));
    acc.pos(S_AZ, K1 * mxi * mzi, t_mul_z(Txzz1, Pxzi));
    acc.pos(S_AZ, K15 * mzi, t_mul_z(Tzzz2, Pzzi));
    out.R[0] = Txxx1; out.R[1] = Txxz1; out.R[2] = Txzz1; out.R[3] = Txzz2; out.R[4] = Tzzz2;
    out.L[0] = Txxx3; out.L[1] = Txxz3; out.L[2] = Txzz3; out.L[3] = Txzz4; out.L[4] = Tzzz4;
    return true;
}

// FP64 accumulation of the primal bound (kappa * T into [lo, hi])
struct AccPrimal {
    div_ a[6];
    __device__ __forceinline__ AccPrimal() {
#pragma unroll
        for (int s = 0; s < 6; ++s) { a[s].lo = 0.0; a[s].hi = 0.0; }
    }
    __device__ __forceinline__ void pos(int s, double k, IV<float> t) {
        a[s].lo = __builtin_fma(k, (double)t.lo, a[s].lo);
        a[s].hi = __builtin_fma(k, (double)t.hi, a[s].hi);
    }
    __device__ __forceinline__ void neg(int s, double k, IV<float> t) {
        a[s].lo = __builtin_fma(k, (double)t.hi, a[s].lo);
        a[s].hi = __builtin_fma(k, (double)t.lo, a[s].hi);
    }
};

// Tangent pass: d L = sum over terms of adj(slot) . kappa d T
struct AccTangent {
    double alo[6], ahi[6];
    double g;
    __device__ __forceinline__ void pos(int s, double k, IV<DF> t) {
        g += alo[s] * k * (double)t.lo.d + ahi[s] * k * (double)t.hi.d;
    }
    __device__ __forceinline__ void neg(int s, double k, IV<DF> t) {
        g += alo[s] * k * (double)t.hi.d + ahi[s] * k * (double)t.lo.d;
    }
};

}  // namespace leb
