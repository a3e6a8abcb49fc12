// testdyn.hip -- the closed-form dynamics of leb_analytic_bound (LINEAR,
// QUADRATIC, SINCOS), the point Jacobians of chain dynamics (eq.
// linearizations) and the zonotope hull (eq. tight_tube_width).
//
// The test kinds evaluate the path-based bound of Theorem 1 with the same
// arithmetic as the chain kernel: displacement intervals rounded outward to
// FP32, Hessian entries and term products in outward-rounded FP32, sums in
// FP64.  Every term contains 0 (each has a displacement factor that does),
// so every lower-end summand is <= 0 and every upper-end summand >= 0: the
// FP64 sums do not cancel and one relative widening covers their rounding.
// A term whose displacement factor is exactly [0, 0] contributes exactly 0.
// One thread per unit; these kinds pin the interval machinery against closed
// forms and are not tuned.
#include <hip/hip_runtime.h>
#include <float.h>
#include <math.h>
#include <stdint.h>

#include "leb.h"
#include "leb_internal.hpp"
#include "pbh_common.hpp"
#include "pbh_node.hpp"

namespace leb {

constexpr int TD_MAX_N = 64;     // QUADRATIC: nx + nu

struct TestArgs {
    const double *z, *v, *mu, *sigma, *Q;
    double *r_lo, *r_hi, *c_bar, *rho_bar;
    uint32_t* flags;
    double pad;
    int64_t units;
    int nx, nu, kind;
};

__device__ __forceinline__ double td_nom(const TestArgs& A, int64_t u, int i) {
    return i < A.nx ? A.z[u * A.nx + i] : A.v[u * A.nu + (i - A.nx)];
}
__device__ __forceinline__ fiv td_disp(const TestArgs& A, int64_t u, int i) {
    const int n = A.nx + A.nu;
    const IV<float> d = disp_interval(A.mu ? A.mu[u * n + i] : 0.0, A.sigma[u * n + i]);
    return mk(d.lo, d.hi);
}
__device__ __forceinline__ bool td_zero(fiv d) { return d.lo == 0.0f && d.hi == 0.0f; }

// coordinate interval X_i = a~_i + Delta_i (FP64 endpoints, outward)
__device__ __forceinline__ void td_box(double a, fiv d, double* lo, double* hi) {
    const double l = a + (double)d.lo, h = a + (double)d.hi;
    *lo = l - fabs(l) * 0x1p-52;
    *hi = h + fabs(h) * 0x1p-52;
}

// -h * [t.lo, t.hi] for h an interval: neg(mul(h, t)) with outward rounding kept
__device__ __forceinline__ fiv td_negmul(fiv a, fiv b) { return neg(mul(a, b)); }

__global__ void __launch_bounds__(256) test_dyn_kernel(TestArgs A) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= A.units) return;
    const int n = A.nx + A.nu;
    uint32_t fl = 0;
    for (int i = 0; i < n; ++i) {
        const double a = td_nom(A, u, i), m = A.mu ? A.mu[u * n + i] : 0.0, s = A.sigma[u * n + i];
        if (!isfinite(a) || !isfinite(m) || !isfinite(s) || !(s >= 0.0)) fl |= LEB_FLAG_BAD_INPUT;
        if (fabs(m) > s) fl |= LEB_FLAG_HULL_EXTENDED;
    }
    for (int l = 0; l < A.nx; ++l) {
        div_ acc{0.0, 0.0};
        int terms = 0;
        bool unbounded = false;
        if (!(fl & LEB_FLAG_BAD_INPUT)) {
            if (A.kind == LEB_DYN_QUADRATIC) {
                // R_l = sum_{j<k} Q_l,kj (Delta_j Delta_k) + 1/2 sum_k Q_l,kk sq(Delta_k)
                const double* Ql = A.Q + (size_t)l * n * n;
                for (int k = 0; k < n; ++k) {
                    const fiv dk = td_disp(A, u, k);
                    for (int j = 0; j <= k; ++j) {
                        const double q = Ql[k * n + j];
                        if (!isfinite(q)) unbounded = true;
                        if (q == 0.0 || unbounded) continue;
                        const fiv dj = td_disp(A, u, j);
                        if (td_zero(dk) || td_zero(dj)) continue;
                        if (j < k) acc_any(acc, q, mul_zz(dj, dk));
                        else acc_any(acc, 0.5 * q, sq_z(dk));
                        ++terms;
                    }
                }
            } else if (A.kind == LEB_DYN_SINCOS && A.nx == 1) {
                // f = sin a: H = -sin over X^(1) = X; R = 1/2 H sq(Delta)
                const fiv d0 = td_disp(A, u, 0);
                if (!td_zero(d0)) {
                    double x0l, x0h;
                    td_box(td_nom(A, u, 0), d0, &x0l, &x0h);
                    SinCos s0;
                    isincos(x0l, x0h, &s0);
                    acc_pos(acc, 0.5, mul_z(neg(s0.s), sq_z(d0)));
                    ++terms;
                }
            } else if (A.kind == LEB_DYN_SINCOS) {
                // f_1 = sin a1 cos a2, f_2 = cos a1 sin a2.  Entries over their prefix
                // boxes: (1,1) and (2,1) over X^(1) = (X_1, a~_2), (2,2) over X^(2) = X.
                const fiv d0 = td_disp(A, u, 0), d1 = td_disp(A, u, 1);
                const double a0 = td_nom(A, u, 0), a1 = td_nom(A, u, 1);
                double x0l, x0h, x1l, x1h;
                td_box(a0, d0, &x0l, &x0h);
                td_box(a1, d1, &x1l, &x1h);
                SinCos s0, s1p, s1;
                isincos(x0l, x0h, &s0);      // sin, cos of X_1
                isincos(a1, a1, &s1p);       // of the point a~_2
                isincos(x1l, x1h, &s1);      // of X_2
                fiv h11, h21, h22;
                if (l == 0) {
                    h11 = td_negmul(s0.s, s1p.c);
                    h21 = td_negmul(s0.c, s1p.s);
                    h22 = td_negmul(s0.s, s1.c);
                } else {
                    h11 = td_negmul(s0.c, s1p.s);
                    h21 = td_negmul(s0.s, s1p.c);
                    h22 = td_negmul(s0.c, s1.s);
                }
                if (!td_zero(d0)) { acc_pos(acc, 0.5, mul_z(h11, sq_z(d0))); ++terms; }
                if (!td_zero(d0) && !td_zero(d1)) { acc_pos(acc, 1.0, mul_z(h21, mul_zz(d0, d1))); ++terms; }
                if (!td_zero(d1)) { acc_pos(acc, 0.5, mul_z(h22, sq_z(d1))); ++terms; }
            }
        }
        double lo, hi;
        if (fl & LEB_FLAG_BAD_INPUT) {
            lo = -INFINITY; hi = INFINITY;
        } else if (unbounded) {
            lo = -INFINITY; hi = INFINITY;
            fl |= LEB_FLAG_UNBOUNDED;
        } else {
            // at most 2080 same-sign FP64 roundings of 2^-53 each, relative to the sum
            lo = acc.lo - fabs(acc.lo) * 0x1p-40;
            hi = acc.hi + fabs(acc.hi) * 0x1p-40;
            if (terms == 0) { lo = 0.0; hi = 0.0; }
        }
        const int64_t o = u * A.nx + l;
        if (A.r_lo) { A.r_lo[o] = lo; A.r_hi[o] = hi; }
        if (A.c_bar) row_zono(lo, hi, A.pad, &A.c_bar[o], &A.rho_bar[o]);
    }
    if (A.flags) A.flags[u] = fl;
}

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

int launch_test_dyn(const leb_dynamics* dyn, int64_t units, const double* z, const double* v, const double* mu,
                    const double* sigma, double* r_lo, double* r_hi, double* c_bar, double* rho_bar, double pad,
                    uint32_t* flags, hipStream_t s) {
    if ((units + 255) / 256 > 0x7fffffff) return LEB_EINVAL;
    TestArgs A;
    A.z = z; A.v = v; A.mu = mu; A.sigma = sigma; A.Q = dyn->coeffs;
    A.r_lo = r_lo; A.r_hi = r_hi; A.c_bar = c_bar; A.rho_bar = rho_bar; A.flags = flags; A.pad = pad;
    A.units = units; A.nx = dyn->nx; A.nu = dyn->nu; A.kind = dyn->kind;
    hipLaunchKernelGGL(test_dyn_kernel, dim3((unsigned)((units + 255) / 256)), dim3(256), 0, s, A);
    return hipGetLastError() == hipSuccess ? LEB_OK : LEB_EDEVICE;
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
