// chain_features.hpp -- inputs and outputs of the chain surrogate, shared by
// the standalone feature/decode kernels and the fused surrogate sweep.
//
// For node i of a chain at one timestep, the surrogate sees what the
// path-based bound of the node's two non-linear rows (vx_i+, vz_i+)
// depends on (Theorem 1 over the prefix boxes of its attitude block and
// of its two springs): nominal theta_i, u1_i + u2_i, the spring
// separations, and the displacement intervals
//   Delta_c = [min(mu_c - sigma_c, 0), max(mu_c + sigma_c, 0)]
// of theta_i, u1_i, u2_i and of the positions of nodes i-1, i, i+1.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "leb.h"

namespace leb {

constexpr float CHAIN_DSCALE = 20.0f;     // displacements of the tube scale to O(1)

// f[0..31] of node i of one unit (zn, vn, m, s: that unit's rows; m may be NULL)
__device__ __forceinline__ void chain_node_features(const double* zn, const double* vn, const double* m,
                                                    const double* s, int i, int U, double L0, float* f) {
    const int nx = 6 * U;
    auto dlo = [&](int c) { return (float)(fmin((m ? m[c] : 0.0) - s[c], 0.0) * CHAIN_DSCALE); };
    auto dhi = [&](int c) { return (float)(fmax((m ? m[c] : 0.0) + s[c], 0.0) * CHAIN_DSCALE); };
    const int th = 6 * i + 2, px = 6 * i, pz = 6 * i + 1, u1 = nx + 2 * i, u2 = u1 + 1;
    f[0] = (float)zn[th];
    f[1] = (float)((vn[2 * i] + vn[2 * i + 1]) * 0.1);
    f[2] = dlo(th); f[3] = dhi(th);
    f[4] = dlo(u1); f[5] = dhi(u1);
    f[6] = dlo(u2); f[7] = dhi(u2);
    f[8] = dlo(px); f[9] = dhi(px);
    f[10] = dlo(pz); f[11] = dhi(pz);
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const int j = side == 0 ? i + 1 : i - 1;      // right, then left neighbour
        const int o = 12 + 7 * side;
        if (j >= 0 && j < U) {
            const int a = side == 0 ? i : j, b = side == 0 ? j : i;   // spring from node a to node b = a + 1
            f[o] = 1.0f;
            f[o + 1] = (float)(L0 + zn[6 * b] - zn[6 * a]);
            f[o + 2] = (float)(zn[6 * b + 1] - zn[6 * a + 1]);
            f[o + 3] = dlo(6 * j); f[o + 4] = dhi(6 * j);
            f[o + 5] = dlo(6 * j + 1); f[o + 6] = dhi(6 * j + 1);
        } else {
#pragma unroll
            for (int t = 0; t < 7; ++t) f[o + t] = 0.0f;
        }
    }
#pragma unroll
    for (int t = 26; t < LEB_CHAIN_FEATURES; ++t) f[t] = 0.0f;
}

// predicted log-bounds (log hi, log(-lo)) of one row -> zonotope centre and radius
// (without padding).  A prediction that is not finite counts as a zero bound
// (the certified iteration then starts below the fixed point); bounds above 1
// are clamped.
__device__ __forceinline__ void chain_decode_row(float ylog_hi, float ylog_nlo, double* c, double* r) {
    const double yh = isfinite(ylog_hi) ? fmin((double)ylog_hi, 0.0) : -1e30;
    const double yl = isfinite(ylog_nlo) ? fmin((double)ylog_nlo, 0.0) : -1e30;
    const double hi = exp(yh), lo = -exp(yl);
    *c = 0.5 * (lo + hi);
    *r = 0.5 * (hi - lo);
}

}  // namespace leb
