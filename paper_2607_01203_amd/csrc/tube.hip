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

// Fixed-point epilogue of the tube map (all NULL for the plain map).
struct TubeFP {
    const double* mu_in;  // C_t: the tube whose bounds produced (c_bar, rho_bar)
    const double* sg_in;
    uint32_t* state;      // [B]: bit 0 certified (frozen), bit 1 F(C_t) not inside C_t
    double tol, abs_;     // C_{t+1} = (mu_F, sigma_F (1 + tol) + abs_)
};

struct TubeArgs {
    const double* cbar; const double* rbar;   // [B][N][nx]
    double e[6];
    double* mu; double* sigma;                // [B][N][n] out
    int B, N, U;
    int groups;        // k-groups per column group (4 k-pairs each)
    int total;         // workgroups in the grid
};

// One wave per (64 columns, k-pair).  A column is one (trajectory, node);
// the wave computes the 8 tube rows of its node at steps k = p and
// k = N-1-p, so every wave performs N-1 block products.  Phi is indexed by
// the wave-uniform lag only, so its 48 entries come through scalar loads;
// the residual centres and radii come through vector loads shared in L2 by
// the waves of the same columns (the workgroup order is remapped so those
// land on one XCD).
__global__ void __launch_bounds__(256) tube_map_kernel(const double* __restrict__ phi, TubeArgs A, TubeFP P) {
    // XCD-aware order: workgroup ids are dealt round-robin over 8 XCDs;
    // give each XCD a contiguous range of (column group, k-group) tiles.
    const int id = blockIdx.x, x = id & 7, pos = id >> 3;
    const int q8 = A.total >> 3, r8 = A.total & 7;
    const int nid = x * q8 + min(x, r8) + pos;
    const int cg = nid / A.groups, g = nid - cg * A.groups;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int npairs = (A.N + 1) >> 1;
    const int p = g * 4 + wave;
    if (p >= npairs) return;
    const int cols = A.B * A.U;
    const int col = cg * 64 + lane;
    const bool valid = col < cols;
    const int cc = valid ? col : cols - 1;
    const int b = cc / A.U, i = cc - b * A.U;
    const int nx = 6 * A.U, n = 8 * A.U;
    const double* cb = A.cbar + ((int64_t)b * A.N) * nx + 6 * i;
    const double* rb = A.rbar + ((int64_t)b * A.N) * nx + 6 * i;
    const bool fp = P.state != nullptr;
    const bool frozen = fp && (P.state[b] & 1u);
    // first lane of this wave holding trajectory b (columns of one trajectory are contiguous)
    const int first = max(0, b * A.U - cg * 64);
    for (int half = 0; half < 2; ++half) {
        const int k = half ? A.N - 1 - p : p;
        if (half && k == p) break;
        double m[8], s[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) { m[r] = 0.0; s[r] = 0.0; }
#pragma unroll 2
        for (int j = 0; j < k; ++j) {
            const double* Pk = phi + (int64_t)(k - j - 1) * 48;
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
                    const double ph = Pk[r * 6 + q];
                    m[r] = __builtin_fma(ph, c[q], m[r]);
                    s[r] = __builtin_fma(fabs(ph), w[q], s[r]);
                }
        }
        // sums of at most 6 (N-1) rounded products: relative error below 2^-44 for N <= 2^7
        bool bad = false;
        const int64_t row0 = ((int64_t)b * A.N + k) * n;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int64_t o = row0 + (r < 6 ? 6 * i + r : nx + 2 * i + (r - 6));
            const double sF = s[r] + s[r] * 0x1p-44, mF = m[r];
            double mo = mF, so = sF;
            if (fp) {
                const double mi = P.mu_in[o], si = P.sg_in[o];
                if (frozen) {
                    mo = mi; so = si;
                } else {
                    // [mF - sF, mF + sF] inside [mi - si, mi + si], with the rounding of the test covered
                    bad |= !((fabs(mF - mi) + sF) * (1.0 + 0x1p-50) <= si);
                    so = sF + sF * P.tol + P.abs_;
                }
            }
            if (valid) { A.mu[o] = mo; A.sigma[o] = so; }
        }
        if (fp) {
            bad = bad && valid;
            const uint64_t mask = __ballot(bad);
            const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
            const uint64_t same = ~0ull << first;
            if (bad && !(mask & below & same)) atomicOr(&P.state[b], 2u);
        }
    }
}

// Per sweep, after the tube map: commit trajectories whose C_t was shown
// certified (state == 0: not frozen, contained) into the output tube.
// With final != 0: commit every trajectory not yet certified (sweep cap).
__global__ void fp_commit_kernel(const double* mu_in, const double* sg_in, double* mu, double* sg,
                                 const uint32_t* state, int64_t per_traj, int64_t count, int final_) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= count) return;
    const uint32_t st = state[q / per_traj];
    const bool go = final_ ? !(st & 1u) : st == 0u;
    if (go && mu_in != mu) { mu[q] = mu_in[q]; sg[q] = sg_in[q]; }
}

// state[b]: certified once contained; clear the per-sweep bit.  state[B]
// receives the number of trajectories not yet certified.
__global__ void __launch_bounds__(256) fp_state_kernel(uint32_t* state, int B) {
    __shared__ uint32_t cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    uint32_t open = 0;
    for (int b = threadIdx.x; b < B; b += 256) {
        const uint32_t st = state[b];
        const uint32_t ns = (st & 1u) | ((st & 2u) ? 0u : 1u);
        state[b] = ns;
        open += ns ? 0u : 1u;
    }
    atomicAdd(&cnt, open);
    __syncthreads();
    if (threadIdx.x == 0) state[B] = cnt;
}

__global__ void u32_fill_kernel(uint32_t* dst, int64_t count, uint32_t v) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < count) dst[q] = v;
}

__global__ void cert_out_kernel(const uint32_t* state, uint32_t* out, int B) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < B) out[b] = state[b] & 1u;
}

__global__ void fill_kernel(double* dst, int64_t count, double v) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < count) dst[q] = v;
}

static unsigned nblk(int64_t count) { return (unsigned)((count + 255) / 256); }

static int launch_tube(int B, int N, int U, const double* phi, const double* e, const double* cbar,
                       const double* rbar, double* mu, double* sigma, const TubeFP& fp, hipStream_t s) {
    TubeArgs a;
    a.cbar = cbar; a.rbar = rbar;
    for (int q = 0; q < 6; ++q) a.e[q] = e[q];
    a.mu = mu; a.sigma = sigma; a.B = B; a.N = N; a.U = U;
    const int64_t cols = (int64_t)B * U;
    if (cols == 0 || N == 0) return LEB_OK;
    const int64_t ncg = (cols + 63) / 64;
    a.groups = ((N + 1) / 2 + 3) / 4;
    const int64_t total = ncg * a.groups;
    if (total > 0x7fffffff) return LEB_EINVAL;
    a.total = (int)total;
    hipLaunchKernelGGL(tube_map_kernel, dim3((unsigned)total), dim3(256), 0, s, phi, a, fp);
    return hipGetLastError() == hipSuccess ? LEB_OK : LEB_EDEVICE;
}

int launch_tube_map(int B, int N, int U, const double* phi, const double* e, const double* cbar,
                    const double* rbar, double* mu, double* sigma, hipStream_t s) {
    TubeFP none{nullptr, nullptr, nullptr, 0.0, 0.0};
    return launch_tube(B, N, U, phi, e, cbar, rbar, mu, sigma, none, s);
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
    double *cb, *rb, *xm[2], *xs[2];
    uint32_t* state;
    const size_t bx = (size_t)units * nx * sizeof(double), bn = (size_t)units * n * sizeof(double);
    if ((rc = ws_get(0, bx, (void**)&cb)) || (rc = ws_get(1, bx, (void**)&rb)) ||
        (rc = ws_get(2, bn, (void**)&xm[0])) || (rc = ws_get(3, bn, (void**)&xs[0])) ||
        (rc = ws_get(4, bn, (void**)&xm[1])) || (rc = ws_get(5, bn, (void**)&xs[1])) ||
        (rc = ws_get(6, ((size_t)batch + 1) * sizeof(uint32_t), (void**)&state)))
        return rc;
    const int64_t cnt = units * n, per = (int64_t)N * n;
    auto ok = [](hipError_t e_) { return e_ == hipSuccess; };
    hipLaunchKernelGGL(u32_fill_kernel, dim3(nblk(batch + 1)), dim3(256), 0, s, state, (int64_t)batch + 1, 0u);
    // iterate C_t: the caller's tube (warm start) or the disturbance-only tube (LEB = 0, below the fixed point)
    const double *im = mu, *is = sigma;
    int nxt = 1;
    if (!opt->warm) {
        hipLaunchKernelGGL(fill_kernel, dim3(nblk(units * nx)), dim3(256), 0, s, cb, units * nx, 0.0);
        hipLaunchKernelGGL(fill_kernel, dim3(nblk(units * nx)), dim3(256), 0, s, rb, units * nx, opt->pad);
        if ((rc = launch_tube_map(batch, N, U, phi, e, cb, rb, xm[0], xs[0], s))) return rc;
        im = xm[0]; is = xs[0];
    }
    int sweeps = 0;
    uint32_t open = 0;
    while (sweeps < opt->max_sweeps) {
        // F(C_t): bound every unit of the tube, then the tube map; C_{t+1} = inflated F(C_t)
        if ((rc = launch_pbh_chain(dyn, units, z, v, im, is, nullptr, nullptr, cb, rb, opt->pad, nullptr, s)))
            return rc;
        const TubeFP fp{im, is, state, opt->tol, opt->inflate_abs};
        if ((rc = launch_tube(batch, N, U, phi, e, cb, rb, xm[nxt], xs[nxt], fp, s))) return rc;
        ++sweeps;
        hipLaunchKernelGGL(fp_commit_kernel, dim3(nblk(cnt)), dim3(256), 0, s, im, is, mu, sigma, state, per, cnt, 0);
        hipLaunchKernelGGL(fp_state_kernel, dim3(1), dim3(256), 0, s, state, batch);
        if (!ok(hipGetLastError()) ||
            !ok(hipMemcpyAsync(&open, state + batch, sizeof(uint32_t), hipMemcpyDeviceToHost, s)) ||
            !ok(hipStreamSynchronize(s)))
            return LEB_EDEVICE;
        im = xm[nxt]; is = xs[nxt];
        nxt ^= 1;
        if (open == 0) break;
    }
    // sweep cap: the latest iterate of every trajectory not certified
    if (open != 0)
        hipLaunchKernelGGL(fp_commit_kernel, dim3(nblk(cnt)), dim3(256), 0, s, im, is, mu, sigma, state, per, cnt, 1);
    hipLaunchKernelGGL(cert_out_kernel, dim3(nblk(batch)), dim3(256), 0, s, state, certified, batch);
    *sweeps_out = sweeps;
    return ok(hipGetLastError()) ? LEB_OK : LEB_EDEVICE;
}
