// tube.hip -- tube map and the tube/LEB fixed point with its certificate.
//
// Tube update (eqs. tight_tube_center, tight_tube_width):
//   mu_k    = sum_{j<k} Phi_{k,j} c_bar_j
//   sigma_k = sum_{j<k} |Phi_{k,j}| (e + rho_bar_j)      (= ||Phi_{k,j} [E diag(rho_bar_j)]||_{1,r})
// Phi is decentralised and lag-invariant: one [8 x 6] block per lag d = k-j,
// shared by every node (rows 0..5 -> node state rows of the tube, rows 6..7
// -> node input rows; columns -> node residual rows).
//
// Fixed point: B -> LEB(B) -> (c_bar, rho_bar) -> tube map -> F(B).  F is
// inclusion-isotone, so a box with F(B) inside B contains the least fixed
// point and certifies the tube by induction over k (the argument of the
// Theorem 3 proof).  Jacobi sweeps update every k at once; causality (the
// tube at k uses steps j < k) bounds the number of sweeps to reach the
// exact fixed point by N.
//
// Certification.  Where the bounds grow faster than linearly in the tube
// radius and exceed the disturbance, F expands locally, so no uniform
// inflation of the least fixed point B* is a post-fixed point.  The causal
// structure (the Jacobian of F is nilpotent) still gives post-fixed points
// B* + (I - J)^-1 w for any w > 0, and the inflated Jacobi iteration
//   C <- F(C) (1 + tol) + abs
// converges to one of them, about tol above B*.  A trajectory is certified
// (and frozen) on the sweep that shows F(C) inside C.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <mutex>
#include <vector>

#include "leb.h"
#include "leb_internal.hpp"

namespace leb {

struct TubeArgs {
    const double* cbar; const double* rbar;   // [B][N][nx]
    const double* phi;                        // [N-1][8][6]
    double e[6];
    double* mu; double* sigma;                // [B][N][n]
    int B, N, U;
};

// one thread per (trajectory, node, step): 8 tube rows of that node
__global__ void __launch_bounds__(256) tube_map_kernel(TubeArgs A) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)A.B * A.U * A.N;
    if (gid >= total) return;
    const int k = (int)(gid % A.N);
    const int64_t bi = gid / A.N;
    const int i = (int)(bi % A.U);
    const int b = (int)(bi / A.U);
    const int nx = 6 * A.U, n = 8 * A.U;
    double m[8], s[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) { m[r] = 0.0; s[r] = 0.0; }
    const double* cb = A.cbar + ((int64_t)b * A.N) * nx + 6 * i;
    const double* rb = A.rbar + ((int64_t)b * A.N) * nx + 6 * i;
    for (int j = 0; j < k; ++j) {
        const double* P = A.phi + (int64_t)(k - j - 1) * 48;
        double c[6], w[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            c[q] = cb[(int64_t)j * nx + q];
            // residual radius plus the allowance for the rounding of the centre sum
            w[q] = A.e[q] + rb[(int64_t)j * nx + q] + fabs(c[q]) * 0x1p-44;
        }
#pragma unroll
        for (int r = 0; r < 8; ++r)
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                const double p = P[r * 6 + q];
                m[r] = __builtin_fma(p, c[q], m[r]);
                s[r] = __builtin_fma(fabs(p), w[q], s[r]);
            }
    }
    double* mo = A.mu + ((int64_t)b * A.N + k) * n;
    double* so = A.sigma + ((int64_t)b * A.N + k) * n;
#pragma unroll
    for (int r = 0; r < 6; ++r) { mo[6 * i + r] = m[r]; so[6 * i + r] = s[r] + s[r] * 0x1p-45; }
#pragma unroll
    for (int r = 0; r < 2; ++r) { mo[nx + 2 * i + r] = m[6 + r]; so[nx + 2 * i + r] = s[6 + r] + s[6 + r] * 0x1p-45; }
}

// Per trajectory: out[2b] = max over entries of max(|dsigma|, |dmu|) /
// max(sigma_new, floor) (relative change), out[2b+1] = 1 if box(new) lies in
// box(old) for every entry (containment), else 0.
__global__ void __launch_bounds__(256) tube_compare_kernel(const double* mu_old, const double* sg_old,
                                                          const double* mu_new, const double* sg_new,
                                                          int64_t per_traj, double floor_, double* out) {
    __shared__ double red[256];
    __shared__ int bad[256];
    const int b = blockIdx.x;
    const double* mo = mu_old + (int64_t)b * per_traj;
    const double* so = sg_old + (int64_t)b * per_traj;
    const double* mn = mu_new + (int64_t)b * per_traj;
    const double* sn = sg_new + (int64_t)b * per_traj;
    double acc = 0.0;
    int nok = 0;
    for (int64_t q = threadIdx.x; q < per_traj; q += 256) {
        const double d = fmax(fabs(sn[q] - so[q]), fabs(mn[q] - mo[q]));
        acc = fmax(acc, d / fmax(sn[q], floor_));
        if (!(isfinite(sn[q]) && isfinite(mn[q])) && !(sn[q] == so[q] && mn[q] == mo[q])) acc = INFINITY;
        const bool ok = (mn[q] - sn[q] >= mo[q] - so[q]) && (mn[q] + sn[q] <= mo[q] + so[q]);
        nok |= ok ? 0 : 1;
    }
    red[threadIdx.x] = acc;
    bad[threadIdx.x] = nok;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
            bad[threadIdx.x] |= bad[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) { out[2 * b] = red[0]; out[2 * b + 1] = bad[0] ? 0.0 : 1.0; }
}

// Next iterate of the inflated Jacobi map for trajectories not yet certified:
// mu <- mu_F, sigma <- sigma_F (1 + rel) + abs (rounded up).
__global__ void advance_kernel(const double* mu_f, const double* sg_f, double* mu, double* sg, const double* cmp,
                               int64_t per_traj, int64_t count, double rel, double abs_) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= count) return;
    const int64_t b = q / per_traj;
    if (cmp[2 * b + 1] != 0.0) return;        // certified: frozen
    const double s = sg_f[q] + sg_f[q] * rel + abs_;
    mu[q] = mu_f[q];
    sg[q] = s + s * 0x1p-50;
}

__global__ void cert_from_cmp(const double* cmp, uint32_t* out, int B) {
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < B) out[b] = cmp[2 * b + 1] != 0.0 ? 1u : 0u;
}

__global__ void fill_kernel(double* dst, int64_t count, double v) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < count) dst[q] = v;
}

// cmp[2b+1] |= cmpn[2b+1] (certified once contained); cmp[2b] = latest change
__global__ void merge_cert_kernel(double* cmp, const double* cmpn, int B) {
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    cmp[2 * b] = cmpn[2 * b];
    if (cmpn[2 * b + 1] != 0.0) cmp[2 * b + 1] = 1.0;
}

static unsigned nblk(int64_t count) { return (unsigned)((count + 255) / 256); }

int launch_tube_map(int B, int N, int U, const double* phi, const double* e, const double* cbar,
                    const double* rbar, double* mu, double* sigma, hipStream_t s) {
    TubeArgs a;
    a.cbar = cbar; a.rbar = rbar; a.phi = phi;
    for (int q = 0; q < 6; ++q) a.e[q] = e[q];
    a.mu = mu; a.sigma = sigma; a.B = B; a.N = N; a.U = U;
    const int64_t total = (int64_t)B * U * N;
    if (total == 0) return LEB_OK;
    hipLaunchKernelGGL(tube_map_kernel, dim3(nblk(total)), dim3(256), 0, s, a);
    return hipGetLastError() == hipSuccess ? LEB_OK : LEB_EDEVICE;
}

// ------------------------------------------------------------ workspace

struct Workspace {
    std::mutex mu;
    std::vector<void*> bufs;
    std::vector<size_t> sizes;
};
static Workspace g_ws;

// grow-only device buffers kept for the life of the process
static int ws_get(int slot, size_t bytes, void** out) {
    if ((int)g_ws.bufs.size() <= slot) { g_ws.bufs.resize(slot + 1, nullptr); g_ws.sizes.resize(slot + 1, 0); }
    if (g_ws.sizes[slot] < bytes) {
        if (g_ws.bufs[slot]) (void)hipFree(g_ws.bufs[slot]);
        g_ws.bufs[slot] = nullptr;
        g_ws.sizes[slot] = 0;
        if (getenv("LEB_TEST_FAIL_ALLOC")) return LEB_ENOMEM;
        if (hipMalloc(&g_ws.bufs[slot], bytes) != hipSuccess) return LEB_ENOMEM;
        g_ws.sizes[slot] = bytes;
    }
    *out = g_ws.bufs[slot];
    return LEB_OK;
}

}  // namespace leb

using namespace leb;

extern "C" int leb_tube_map(int32_t batch, int32_t N, int32_t n_units, const double* phi, const double* e,
                            const double* c_bar, const double* rho_bar, double* mu, double* sigma,
                            void* stream) {
    if (batch < 0 || N < 0 || n_units < 1 || n_units > 4096 || !e) return LEB_EINVAL;
    if ((int64_t)batch * N == 0) return LEB_OK;
    if (!c_bar || !rho_bar || !mu || !sigma || (N > 1 && !phi)) return LEB_EINVAL;
    const void* ptrs[] = {phi, c_bar, rho_bar, mu, sigma};
    for (const void* p : ptrs)
        if (p && !aligned8(p)) return LEB_EINVAL;
    for (int q = 0; q < 6; ++q)
        if (!(e[q] >= 0.0) || !isfinite(e[q])) return LEB_EINVAL;
    return launch_tube_map(batch, N, n_units, phi, e, c_bar, rho_bar, mu, sigma, (hipStream_t)stream);
}

extern "C" int leb_fixed_point_solve(const leb_dynamics* dyn, int32_t batch, int32_t N, const double* z,
                                     const double* v, const double* phi, const double* e,
                                     const leb_fp_options* opt, double* mu, double* sigma,
                                     uint32_t* certified, int32_t* sweeps_out, void* stream) {
    int rc = check_chain_dynamics(dyn);
    if (rc != LEB_OK) return rc;
    if (dyn->kind != LEB_DYN_PQUAD_CHAIN) return LEB_ENOTSUP;
    if (!opt || !e || !sweeps_out) return LEB_EINVAL;
    if (batch < 0 || N < 0) return LEB_EINVAL;
    if (!(opt->tol >= 0.0) || !isfinite(opt->tol) || opt->max_sweeps < 1 || !(opt->pad >= 0.0) ||
        !(opt->inflate_abs > 0.0) || !isfinite(opt->inflate_abs))
        return LEB_EINVAL;
    for (int q = 0; q < 6; ++q)
        if (!(e[q] >= 0.0) || !isfinite(e[q])) return LEB_EINVAL;
    *sweeps_out = 0;
    const int64_t units = (int64_t)batch * N;
    if (units == 0) return LEB_OK;
    if (!z || !v || !mu || !sigma || !certified || (N > 1 && !phi)) return LEB_EINVAL;
    const void* ptrs[] = {z, v, phi, mu, sigma};
    for (const void* p : ptrs)
        if (p && !aligned8(p)) return LEB_EINVAL;
    const int U = dyn->n_units, nx = dyn->nx, n = dyn->nx + dyn->nu;
    hipStream_t s = (hipStream_t)stream;

    std::lock_guard<std::mutex> lock(g_ws.mu);
    double *cb, *rb, *mu2, *sg2, *cmp, *cmpn;
    const size_t bx = (size_t)units * nx * sizeof(double), bn = (size_t)units * n * sizeof(double);
    if ((rc = ws_get(0, bx, (void**)&cb)) || (rc = ws_get(1, bx, (void**)&rb)) ||
        (rc = ws_get(2, bn, (void**)&mu2)) || (rc = ws_get(3, bn, (void**)&sg2)) ||
        (rc = ws_get(4, (size_t)batch * 2 * sizeof(double), (void**)&cmp)) ||
        (rc = ws_get(5, (size_t)batch * 2 * sizeof(double), (void**)&cmpn)))
        return rc;
    std::vector<double> host(2 * (size_t)batch);
    const int64_t cnt = units * n;
    auto ok = [](hipError_t e_) { return e_ == hipSuccess; };
    int sweeps = 0;
    // F: bound every unit of box (m_, s_) then map to (mo, so)
    auto F = [&](const double* m_, const double* s_, double* mo, double* so) -> int {
        int r = launch_pbh_chain(dyn, units, z, v, m_, s_, nullptr, nullptr, cb, rb, opt->pad, nullptr, s);
        if (r) return r;
        if ((r = launch_tube_map(batch, N, U, phi, e, cb, rb, mo, so, s))) return r;
        ++sweeps;
        return LEB_OK;
    };
    if (!opt->warm) {       // disturbance-only tube (LEB = 0): below the fixed point
        hipLaunchKernelGGL(fill_kernel, dim3(nblk(units * nx)), dim3(256), 0, s, cb, units * nx, 0.0);
        hipLaunchKernelGGL(fill_kernel, dim3(nblk(units * nx)), dim3(256), 0, s, rb, units * nx, opt->pad);
        if ((rc = launch_tube_map(batch, N, U, phi, e, cb, rb, mu, sigma, s))) return rc;
    }
    // Inflated Jacobi: C <- F(C) (1 + tol) + abs until F(C) lies inside C.
    // A trajectory is frozen (and certified) from the sweep that shows it.
    hipLaunchKernelGGL(fill_kernel, dim3(nblk(2 * (int64_t)batch)), dim3(256), 0, s, cmp, 2 * (int64_t)batch, 0.0);
    while (sweeps < opt->max_sweeps) {
        if ((rc = F(mu, sigma, mu2, sg2))) return rc;
        // containment per trajectory, accumulated (frozen trajectories stay certified)
        hipLaunchKernelGGL(tube_compare_kernel, dim3(batch), dim3(256), 0, s, mu, sigma, mu2, sg2, (int64_t)N * n,
                           opt->inflate_abs, cmpn);
        hipLaunchKernelGGL(merge_cert_kernel, dim3(nblk(batch)), dim3(256), 0, s, cmp, cmpn, batch);
        if (!ok(hipGetLastError())) return LEB_EDEVICE;
        if (!ok(hipMemcpyAsync(host.data(), cmp, 2 * (size_t)batch * sizeof(double), hipMemcpyDeviceToHost, s)) ||
            !ok(hipStreamSynchronize(s)))
            return LEB_EDEVICE;
        bool all = true;
        for (int b = 0; b < batch; ++b) all = all && host[2 * b + 1] != 0.0;
        if (all) {
            hipLaunchKernelGGL(cert_from_cmp, dim3(nblk(batch)), dim3(256), 0, s, cmp, certified, batch);
            *sweeps_out = sweeps;
            return ok(hipGetLastError()) ? LEB_OK : LEB_EDEVICE;
        }
        hipLaunchKernelGGL(advance_kernel, dim3(nblk(cnt)), dim3(256), 0, s, mu2, sg2, mu, sigma, cmp, (int64_t)N * n, cnt,
                           opt->tol, opt->inflate_abs);
    }
    // sweep budget exhausted: report which trajectories were certified
    hipLaunchKernelGGL(cert_from_cmp, dim3(nblk(batch)), dim3(256), 0, s, cmp, certified, batch);
    *sweeps_out = sweeps;
    return ok(hipGetLastError()) ? LEB_OK : LEB_EDEVICE;
}
