// tube.hip -- tube map and the tube/LEB fixed point with its certificate.
//
// Tube update (eqs. tight_tube_center, tight_tube_width):
//   mu_k    = sum_{j<k} Phi_{k,j} c_bar_j
//   sigma_k = sum_{j<k} |Phi_{k,j}| (e + rho_bar_j)      (= ||Phi_{k,j} [E diag(rho_bar_j)]||_{1,r})
// Phi is decentralised and lag-invariant: one [8 x 6] block per lag d = k-j,
// shared by every node (rows 0..5 -> node state rows of the tube, rows 6..7
// -> node input rows; columns -> node residual rows).
//
// Fixed point: C -> LEB(C) -> (c_bar, rho_bar) -> tube map -> F(C).  F is
// inclusion-isotone, so a tube with F(C) inside C contains the least fixed
// point and certifies the tube by induction over k (the argument of the
// Theorem 3 proof).  Jacobi sweeps update every k at once; causality (the
// tube at k uses steps j < k) bounds the number of sweeps to reach the
// fixed point by N.
//
// Certification.  Where the bounds grow faster than linearly in the tube
// radius and exceed the disturbance, F expands locally, so no uniform
// inflation of the least fixed point C* is a post-fixed point.  The causal
// structure (the Jacobian of F is nilpotent) still gives post-fixed points
// C* + (I - J)^-1 w for any w > 0, and the inflated Jacobi iteration
//   C <- F(C) (1 + tol) + abs
// converges to one of them, about tol above C*.  A trajectory is certified
// (and frozen) by the sweep that shows F(C) inside C.
#include <hip/hip_runtime.h>
#include <float.h>
#include <math.h>
#include <stdint.h>

#include <mutex>
#include <vector>

#include "leb.h"
#include "leb_internal.hpp"

namespace leb {

// Per-trajectory fixed-point state word.
constexpr uint32_t FP_CERT = 1u;          // certified (frozen)
constexpr uint32_t FP_OPEN = 1u << 31;    // this sweep: F(C) not inside C
constexpr int FP_SLOTS = 4096;            // host-visible open counts, one per sweep (mod FP_SLOTS)

// Fixed-point epilogue of the tube map (state == NULL for the plain map).
struct TubeFP {
    const double* mu_in;  // C_{t-1}: the tube whose bounds produced (c_bar, rho_bar)
    const double* sg_in;
    uint32_t* state;      // [B] state words, [B] open count
    double tol, abs_;     // C_t = (mu_F, sigma_F (1 + tol) + abs_)
};

struct TubeArgs {
    const double* cbar; const double* rbar;   // [B][N][nx]
    double e[6];
    double* mu; double* sigma;                // [B][N][n] out
    double wid;        // relative rounding allowance of the tube sums
    int B, N, U;
};

typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int TM_RT = 5;        // 16-row tiles per wave and row group

// The tube map as a contraction on FP64 MFMA (v_mfma_f64_16x16x4f64):
//   [mu; sigma][row (k, r)][col] = sum_{kk = (j, q)} T[row][kk] [c; w][kk][col],
//   T = Phi_{k-j-1}[r][q] for j < k (|Phi| for sigma), 0 otherwise,
//   c = c_bar_j[q], w = e_q + rho_bar_j[q] + |c| wid,
// with a column per (trajectory, node).  A workgroup owns 16 columns; wave w
// owns the row tiles w, w+4, ... (16 rows = 2 steps each) of its row group
// and skips the K range above the causal diagonal of each tile.  A
// fragments come from Phi in LDS, B fragments from the residual zonotopes
// (shared in L1 by the four waves).  Lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; element i of its accumulator is D[4i + l/16][l%16].
//
// Fixed-point form: frozen trajectories are not written; containment
// failures are or-ed into the state words (fp_state_kernel folds them).
__global__ void __launch_bounds__(256) tube_map_kernel(const double* __restrict__ phi, TubeArgs A, TubeFP P) {
    // LDS: Phi [(N-1)*48], e[6], then the B block of this workgroup's 16
    // columns: c [6(N-1)][16] and w [6(N-1)][16]
    extern __shared__ double sphi[];
    __shared__ uint32_t sbad[16];
    __shared__ int sjinf[16];
    const bool fp = P.state != nullptr;
    if (fp && P.state[A.B] == 0u) return;     // every trajectory certified by an earlier sweep
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int N = A.N, U = A.U, nx = 6 * U, n = 8 * U;
    const int nphi = (N - 1) * 48;
    const int kfull = 6 * (N - 1);
    double* se = sphi + nphi;
    double* sc = se + 8;
    double* sw = sc + (size_t)kfull * 16;
    for (int idx = tid; idx < nphi; idx += 256) sphi[idx] = phi[idx];
    if (tid < 6) se[tid] = A.e[tid];
    if (tid < 16) { sbad[tid] = 0u; sjinf[tid] = 0x7fffffff; }
    __syncthreads();
    const int cols = A.B * U;
    const int c0 = blockIdx.x * 16;
    // stage c_bar and w = e + rho_bar + |c_bar| wid: thread (kk-chunk, column), the 6 q of one
    // (column, step) are contiguous in HBM.  A residual that is not finite enters as 0, and
    // every later step of its column gets sigma = +inf (a product 0 * inf with the zero
    // entries of T would otherwise make earlier rows NaN).
    for (int idx = tid; idx < kfull * 16; idx += 256) {
        const int cl = idx / kfull, kk = idx - cl * kfull;
        const int j = kk / 6, q = kk - 6 * j;
        const int col = c0 + cl;
        double c = 0.0, w = 0.0;
        if (col < cols) {
            const int bb = col / U, nd = col - bb * U;
            const int64_t o = ((int64_t)bb * N + j) * nx + 6 * nd + q;
            c = A.cbar[o];
            w = se[q] + A.rbar[o] + fabs(c) * A.wid;
            if (!(fabs(c) <= DBL_MAX && w <= DBL_MAX)) {
                atomicMin(&sjinf[cl], j);
                c = 0.0;
                w = 0.0;
            }
        }
        sc[kk * 16 + cl] = c;
        sw[kk * 16 + cl] = w;
    }
    __syncthreads();
    const int col = c0 + (lane & 15);
    const bool cvalid = col < cols;
    const int cc = cvalid ? col : cols - 1;
    const int b = cc / U, node = cc - b * U;
    const int bfirst = c0 / U;
    const int nrt = (N + 1) >> 1;
    int kmax[TM_RT];
    int kw = 0;
#pragma unroll
    for (int s = 0; s < TM_RT; ++s) {
        const int rt = wave + 4 * (blockIdx.y * TM_RT + s);
        kmax[s] = rt < nrt ? 6 * min(N - 1, 2 * rt + 1) : 0;
        kw = max(kw, kmax[s]);
    }
    d4 am[TM_RT], as[TM_RT];
#pragma unroll
    for (int s = 0; s < TM_RT; ++s) { am[s] = d4{0.0, 0.0, 0.0, 0.0}; as[s] = d4{0.0, 0.0, 0.0, 0.0}; }
    const int lr = lane & 15, lq = lane >> 4;
    for (int k0 = 0; k0 < kw; k0 += 4) {
        const int kk = k0 + lq;
        const int j = kk / 6, q = kk - 6 * j;
        const bool kin = kk < kfull;
        const double c = kin ? sc[kk * 16 + lr] : 0.0;
        const double w = kin ? sw[kk * 16 + lr] : 0.0;
#pragma unroll
        for (int s = 0; s < TM_RT; ++s) {
            if (k0 >= kmax[s]) continue;       // wave-uniform
            const int rt = wave + 4 * (blockIdx.y * TM_RT + s);
            const int r = 16 * rt + lr, k = r >> 3, rr = r & 7;
            const int lag = k - j - 1;
            const double a = (lag >= 0 && lag < N - 1 && kin) ? sphi[lag * 48 + rr * 6 + q] : 0.0;
            am[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, c, am[s], 0, 0, 0);
            as[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(fabs(a), w, as[s], 0, 0, 0);
        }
    }
    const int jinf = sjinf[lr];
    const bool frozen = fp && (P.state[b] & FP_CERT);
    bool bad = false;
#pragma unroll
    for (int s = 0; s < TM_RT; ++s) {
        const int rt = wave + 4 * (blockIdx.y * TM_RT + s);
        if (rt >= nrt) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = 16 * rt + 4 * i + lq, k = r >> 3, rr = r & 7;
            if (k >= N || !cvalid) continue;
            const int64_t o = ((int64_t)b * N + k) * n + (rr < 6 ? 6 * node + rr : nx + 2 * node + (rr - 6));
            // sums of nonnegative terms, rounded upward; 2^-1000 covers any flushed subnormal part
            const double sF = k > jinf ? INFINITY : as[s][i] + as[s][i] * A.wid + 0x1p-1000, mF = am[s][i];
            double so = sF;
            if (fp) {
                const double mi = P.mu_in[o], si = P.sg_in[o];
                // [mF - sF, mF + sF] inside [mi - si, mi + si], with the rounding of the test
                // covered; a tube that is not finite is never accepted
                bad |= !(sF <= DBL_MAX && (fabs(mF - mi) + sF) * (1.0 + 0x1p-50) <= si);
                so = sF + sF * P.tol + P.abs_;
            }
            if (!frozen) { A.mu[o] = mF; A.sigma[o] = so; }
        }
    }
    if (!fp) return;
    if (bad && !frozen) sbad[b - bfirst] = 1u;
    __syncthreads();
    if (tid < 16 && sbad[tid] && bfirst + tid < A.B) atomicOr(&P.state[bfirst + tid], FP_OPEN);
}

// After the tube map of sweep t: fold this sweep's containment into the
// state words (certified at t, or open) and publish the open count to the
// device word and to host memory.  One workgroup.
__global__ void __launch_bounds__(256) fp_state_kernel(uint32_t* state, int B, uint32_t* host_open, int sweep) {
    if (state[B] == 0u) return;       // nothing open: this sweep was not needed
    __shared__ uint32_t cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    uint32_t open = 0;
    for (int t = threadIdx.x; t < B; t += 256) {
        const uint32_t st = state[t];
        uint32_t ns = st;
        if (!(st & FP_CERT)) {
            ns = (st & FP_OPEN) ? 0u : (FP_CERT | ((uint32_t)sweep << 1));
            state[t] = ns;
        }
        open += (ns & FP_CERT) ? 0u : 1u;
    }
    atomicAdd(&cnt, open);
    __syncthreads();
    if (threadIdx.x == 0) {
        state[B] = cnt;
        __hip_atomic_store(&host_open[sweep % FP_SLOTS], cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// After the last sweep: the certified tube of each trajectory is C_{s-1}
// (s = the sweep that certified it), which sits in buffer (s-1) & 1; an
// uncertified trajectory takes the latest iterate C_T from buffer T & 1.
// Buffer 0 is the caller's; buffer 1 is copied into it where needed.
__global__ void fp_final_kernel(const double* xm1, const double* xs1, double* mu, double* sg,
                                const uint32_t* state, int64_t per_traj, int64_t count, int last_sweep) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= count) return;
    const uint32_t st = state[q / per_traj];
    const int src = (st & FP_CERT) ? (int)(((st >> 1) - 1) & 1u) : (last_sweep & 1);
    if (src == 1) { mu[q] = xm1[q]; sg[q] = xs1[q]; }
}

__global__ void fp_init_kernel(uint32_t* state, int B) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < B) state[t] = 0u;
    if (t == B) state[B] = (uint32_t)B;     // open count
}

__global__ void cert_out_kernel(const uint32_t* state, uint32_t* out, int B) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < B) out[b] = state[b] & FP_CERT;
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
    // A sum of m rounded products (and the 3 operations forming a weight)
    // errs by at most gamma_{m+3} ~ (m+3) 2^-53 relative, in any order of
    // accumulation; twice that covers both the sigma sums and, through
    // |c_bar| wid in the weights, the rounding of the centre sums.
    a.wid = fmax(0x1p-44, (6.0 * (N > 0 ? N - 1 : 0) + 4.0) * 0x1p-52);
    const int64_t cols = (int64_t)B * U;
    if (cols == 0 || N == 0) return LEB_OK;
    const int64_t gx = (cols + 15) / 16;
    const int nrt = (N + 1) / 2;
    const int gy = (nrt + 4 * TM_RT - 1) / (4 * TM_RT);
    if (gx > 0x7fffffff || (int64_t)cols > 0x7fffffff) return LEB_EINVAL;
    // Phi, e (padded to 8) and the B block (c and w for 16 columns)
    const size_t nm1 = N > 1 ? N - 1 : 0;
    const size_t smem = (nm1 * 48 + 8 + 2 * 6 * nm1 * 16) * sizeof(double);
    if (smem > 160 * 1024 - 256) return LEB_ENOTSUP;     // N <= 86
    static bool lds_attr = false;      // the kernel may use up to 160 KB of LDS (set once)
    if (smem > 65536 && !lds_attr) {
        if (hipFuncSetAttribute((const void*)tube_map_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                160 * 1024 - 256) != hipSuccess)
            return LEB_EDEVICE;
        lds_attr = true;
    }
    hipLaunchKernelGGL(tube_map_kernel, dim3((unsigned)gx, gy), dim3(256), smem, s, phi, a, fp);
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
    uint32_t* host_open = nullptr;      // pinned, host-mapped
    uint32_t* host_open_dev = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
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

static int ws_host_and_events() {
    if (!g_ws.host_open) {
        void* h = nullptr;
        if (hipHostMalloc(&h, FP_SLOTS * sizeof(uint32_t), hipHostMallocMapped) != hipSuccess) return LEB_ENOMEM;
        void* d = nullptr;
        if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess) { (void)hipHostFree(h); return LEB_EDEVICE; }
        g_ws.host_open = (uint32_t*)h;
        g_ws.host_open_dev = (uint32_t*)d;
    }
    for (int q = 0; q < 2; ++q)
        if (!g_ws.ev[q] && hipEventCreateWithFlags(&g_ws.ev[q], hipEventDisableTiming) != hipSuccess)
            return LEB_EDEVICE;
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
    double *cb, *rb, *xm1, *xs1;
    uint32_t* state;
    const size_t bx = (size_t)units * nx * sizeof(double), bn = (size_t)units * n * sizeof(double);
    if ((rc = ws_get(0, bx, (void**)&cb)) || (rc = ws_get(1, bx, (void**)&rb)) ||
        (rc = ws_get(2, bn, (void**)&xm1)) || (rc = ws_get(3, bn, (void**)&xs1)) ||
        (rc = ws_get(4, ((size_t)batch + 1) * sizeof(uint32_t), (void**)&state)) || (rc = ws_host_and_events()))
        return rc;
    // iterates: buffer 0 = the caller's (mu, sigma), buffer 1 = workspace; sweep t reads C_{t-1}
    // from buffer (t-1) & 1 and writes C_t to buffer t & 1
    double* xm[2] = {mu, xm1};
    double* xs[2] = {sigma, xs1};
    const int64_t cnt = units * n, per = (int64_t)N * n;
    auto ok = [](hipError_t e_) { return e_ == hipSuccess; };
    hipLaunchKernelGGL(fp_init_kernel, dim3(nblk(batch + 1)), dim3(256), 0, s, state, batch);
    if (!opt->warm) {       // C_0: the disturbance-only tube (LEB = 0), below the fixed point
        hipLaunchKernelGGL(fill_kernel, dim3(nblk(units * nx)), dim3(256), 0, s, cb, units * nx, 0.0);
        hipLaunchKernelGGL(fill_kernel, dim3(nblk(units * nx)), dim3(256), 0, s, rb, units * nx, opt->pad);
        if ((rc = launch_tube_map(batch, N, U, phi, e, cb, rb, mu, sigma, s))) return rc;
    }
    volatile uint32_t* hopen = g_ws.host_open;
    auto sweep = [&](int t) -> int {
        const int a = (t - 1) & 1, w = t & 1;
        int r = launch_pbh_chain(dyn, units, z, v, xm[a], xs[a], nullptr, nullptr, cb, rb, opt->pad, nullptr, s,
                                 state + batch);
        if (r) return r;
        hopen[t % FP_SLOTS] = 0xffffffffu;
        const TubeFP fp{xm[a], xs[a], state, opt->tol, opt->inflate_abs};
        if ((r = launch_tube(batch, N, U, phi, e, cb, rb, xm[w], xs[w], fp, s))) return r;
        hipLaunchKernelGGL(fp_state_kernel, dim3(1), dim3(256), 0, s, state, batch, g_ws.host_open_dev, t);
        return ok(hipEventRecord(g_ws.ev[t & 1], s)) ? LEB_OK : LEB_EDEVICE;
    };
    // one sweep stays in flight while the host reads the previous sweep's
    // open count; a sweep enqueued after the last needed one exits at once
    if ((rc = sweep(1))) return rc;
    int t = 1;
    for (;;) {
        if (t < opt->max_sweeps && (rc = sweep(t + 1))) return rc;
        if (!ok(hipEventSynchronize(g_ws.ev[t & 1]))) return LEB_EDEVICE;
        const uint32_t open = hopen[t % FP_SLOTS];
        if (open == 0xffffffffu) return LEB_EDEVICE;     // the sweep did not publish its count
        if (open == 0 || t == opt->max_sweeps) break;
        ++t;
    }
    hipLaunchKernelGGL(fp_final_kernel, dim3(nblk(cnt)), dim3(256), 0, s, xm1, xs1, mu, sigma, state, per, cnt, t);
    hipLaunchKernelGGL(cert_out_kernel, dim3(nblk(batch)), dim3(256), 0, s, state, certified, batch);
    *sweeps_out = t;
    return ok(hipGetLastError()) ? LEB_OK : LEB_EDEVICE;
}
