// testdyn.hip -- the point Jacobians of chain dynamics (eq. linearizations)
// and the zonotope hull (eq. tight_tube_width).
#include <hip/hip_runtime.h>
#include <float.h>
#include <math.h>
#include <stdint.h>

#include "leb.h"
#include "leb_internal.hpp"
#include "pbh_common.hpp"
#include "pbh_node.hpp"

namespace leb {

// ------------------------------------------------------------ Jacobians
//
// x+ = x + dt xdot (forward Euler), so A = I + dt d(xdot)/dx, B = dt d(xdot)/du.
// Spring s joins nodes s and s+1 with d = (L0 + px_{s+1} - px_s, pz_{s+1} - pz_s)
// and F_s = k (|d| - L0) d / |d| on node s (-F_s on node s+1); its derivative in
// d is K_s = k ((1 - L0/|d|) I + L0 d d^T / |d|^3), and d(d)/d(p_{s+1}) = I,
// d(d)/d(p_s) = -I.  One thread per entry of [A | B].

struct JacArgs {
    const double *z, *v;
    double *A, *B;
    int64_t count;     // units * nx * (nx + nu)
    int U;
    double dt, m, k, L0, arm, inertia;
};

// K_s[r][c] of spring s at the nominal of one unit
__device__ __forceinline__ double spring_K(const double* zu, int s, int r, int c, double k, double L0) {
    const double dx = L0 + zu[6 * (s + 1)] - zu[6 * s];
    const double dz = zu[6 * (s + 1) + 1] - zu[6 * s + 1];
    const double d2 = dx * dx + dz * dz, d = sqrt(d2);
    const double dr = r == 0 ? dx : dz, dc = c == 0 ? dx : dz;
    return k * ((r == c ? 1.0 - L0 / d : 0.0) + L0 * dr * dc / (d2 * d));
}

__global__ void __launch_bounds__(256) chain_jac_kernel(JacArgs J) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= J.count) return;
    const int nx = 6 * J.U, nu = 2 * J.U, n = nx + nu;
    const int64_t u = q / ((int64_t)nx * n);
    const int rem = (int)(q - u * (int64_t)nx * n);
    const int l = rem / n, c = rem - l * n;
    const int i = l / 6, comp = l - 6 * i;
    const double* zu = J.z + u * nx;
    const double* vu = J.v + u * nu;
    const double th = zu[6 * i + 2], thrust = vu[2 * i] + vu[2 * i + 1];
    const double cm = J.dt / J.m;
    double val = 0.0;
    if (c < nx) {
        const int j = c / 6, cc = c - 6 * j;
        if (c == l) val = 1.0;
        if (comp <= 2 && j == i && cc == comp + 3) val += J.dt;
        if (comp == 3 || comp == 4) {
            const int r = comp - 3;
            if (j == i && cc == 2) val += comp == 3 ? -cm * thrust * cos(th) : -cm * thrust * sin(th);
            if (cc <= 1) {
                // force on node i: F_i - F_{i-1}; derivative in p_j
                double g = 0.0;
                if (i < J.U - 1) {
                    if (j == i + 1) g += spring_K(zu, i, r, cc, J.k, J.L0);
                    if (j == i) g -= spring_K(zu, i, r, cc, J.k, J.L0);
                }
                if (i > 0) {
                    if (j == i) g -= spring_K(zu, i - 1, r, cc, J.k, J.L0);
                    if (j == i - 1) g += spring_K(zu, i - 1, r, cc, J.k, J.L0);
                }
                val += cm * g;
            }
        }
        J.A[(u * nx + l) * nx + c] = val;
    } else {
        const int ci = c - nx, j = ci / 2, ua = ci - 2 * j;
        if (j == i) {
            if (comp == 3) val = -cm * sin(th);
            else if (comp == 4) val = cm * cos(th);
            else if (comp == 5) val = (ua == 0 ? 1.0 : -1.0) * J.dt * J.arm / J.inertia;
        }
        J.B[(u * nx + l) * nu + ci] = val;
    }
}

// ------------------------------------------------------------ zonotope hull
//
// One wave per row: lane partial sums over a stride of 64 columns, then a
// fixed butterfly, so the result does not depend on the launch.  The sum of
// n_gen non-negative terms is rounded upward by (n_gen / 64 + 8) 2^-52
// relative (each lane adds at most n_gen / 64 + 1 terms, the tree 6 levels).

__global__ void __launch_bounds__(256) zonotope_hull_kernel(int rows, int n_gen, const double* G, const double* c,
                                                            double* mu, double* sigma) {
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (row >= rows) return;
    const double* g = G + (size_t)row * n_gen;
    double s = 0.0;
    for (int j = lane; j < n_gen; j += 64) s += fabs(g[j]);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) {
        const double w = ((double)(n_gen / 64) + 8.0) * 0x1p-52;
        double sg = s + s * w;
        if (!(sg <= DBL_MAX)) sg = INFINITY;
        sigma[row] = sg;
        mu[row] = c ? c[row] : 0.0;
    }
}

int launch_chain_jacobians(const leb_dynamics* dyn, int64_t units, const double* z, const double* v, double* A,
                           double* B, hipStream_t s) {
    JacArgs J;
    J.z = z; J.v = v; J.A = A; J.B = B;
    J.U = dyn->n_units;
    J.count = units * (int64_t)dyn->nx * (dyn->nx + dyn->nu);
    if ((J.count + 255) / 256 > 0x7fffffff) return LEB_EINVAL;
    J.dt = dyn->dt; J.m = dyn->m; J.k = dyn->k_spring; J.L0 = dyn->rest_len; J.arm = dyn->arm;
    J.inertia = dyn->inertia;
    hipLaunchKernelGGL(chain_jac_kernel, dim3((unsigned)((J.count + 255) / 256)), dim3(256), 0, s, J);
    return hipGetLastError() == hipSuccess ? LEB_OK : LEB_EDEVICE;
}

}  // namespace leb

using namespace leb;

extern "C" int leb_zonotope_hull(int32_t rows, int32_t n_gen, const double* G, const double* c, double* mu,
                                 double* sigma, void* stream) {
    if (rows < 0 || n_gen < 0) return LEB_EINVAL;
    if (rows == 0) return LEB_OK;
    if (!mu || !sigma || (n_gen > 0 && !G)) return LEB_EINVAL;
    const void* ptrs[] = {G, c, mu, sigma};
    for (const void* p : ptrs)
        if (p && !aligned8(p)) return LEB_EINVAL;
    hipLaunchKernelGGL(zonotope_hull_kernel, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, (hipStream_t)stream, rows,
                       n_gen, G, c, mu, sigma);
    return hipGetLastError() == hipSuccess ? LEB_OK : LEB_EDEVICE;
}
