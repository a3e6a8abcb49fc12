// surrogate.hip -- features, targets and decoding of the learned warm start,
// and the learned tube/LEB fixed point.
//
// The surrogate predicts, for node i of a chain at one timestep, the bound
// of its two non-linear rows (vx_i+, vz_i+) from the quantities the
// path-based bound of those rows depends on (Theorem 1 over the prefix
// boxes of node i's attitude block and of its two springs):
//   nominal theta_i, u1_i + u2_i, the spring separations to the
//   neighbours, and the displacement intervals
//   Delta_c = [min(mu_c - sigma_c, 0), max(mu_c + sigma_c, 0)]
//   of theta_i, u1_i, u2_i and of the positions of nodes i-1, i, i+1.
// Outputs (regression targets): log(max(hi, 1e-14)) and log(max(-lo, 1e-14))
// of the vx and vz rows (every term of the bound contains 0, so lo <= 0 <= hi).
//
// The second family covers ReLU-MLP dynamics: one box of the network's input
// (the nominal a~ = [z; v] and the half width of its displacement interval)
// maps to the log-bounds of every output row.
//
// The learned fixed point runs the tube iteration with surrogate bounds
// for a few sweeps (the initial tube), inflates it, and hands it to the
// certified iteration as a warm start; the result is certified by the
// plain bound exactly as from a cold start.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <mutex>

#include "leb.h"
#include "chain_features.hpp"
#include "leb_internal.hpp"

namespace leb {

constexpr float LOG_FLOOR = 1e-14f;
constexpr float NN_LOG_CEIL = 80.0f;

// one thread per (unit, node); rows of 32 floats written as 8 float4
__global__ void chain_features_kernel(const double* z, const double* v, const double* mu, const double* sigma,
                                      int nodes, int U, double L0, float* X) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nodes) return;
    const int u = q / U, i = q - u * U;
    const int nx = 6 * U, nu = 2 * U, n = nx + nu;
    float f[LEB_CHAIN_FEATURES];
    chain_node_features(z + (int64_t)u * nx, v + (int64_t)u * nu, mu ? mu + (int64_t)u * n : nullptr,
                        sigma + (int64_t)u * n, i, U, L0, f);
    float4* out = reinterpret_cast<float4*>(X + (int64_t)q * LEB_CHAIN_FEATURES);
#pragma unroll
    for (int t = 0; t < LEB_CHAIN_FEATURES / 4; ++t) out[t] = make_float4(f[4 * t], f[4 * t + 1], f[4 * t + 2], f[4 * t + 3]);
}

// targets from a bound: one thread per (unit, node)
__global__ void chain_targets_kernel(const double* r_lo, const double* r_hi, int nodes, int U, float* T) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nodes) return;
    const int u = q / U, i = q - u * U;
    const int64_t o = (int64_t)u * 6 * U + 6 * i;
    reinterpret_cast<float4*>(T)[q] = make_float4(logf(fmaxf((float)r_hi[o + 3], LOG_FLOOR)),
                                                  logf(fmaxf((float)-r_lo[o + 3], LOG_FLOOR)),
                                                  logf(fmaxf((float)r_hi[o + 4], LOG_FLOOR)),
                                                  logf(fmaxf((float)-r_lo[o + 4], LOG_FLOOR)));
}

// predicted bounds -> residual zonotope (c_bar, rho_bar): one thread per (unit, row)
__global__ void chain_decode_kernel(const float* Y, int64_t units, int U, double pad, double* cb, double* rb) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int nx = 6 * U;
    if (q >= units * nx) return;
    const int64_t u = q / nx;
    const int row = (int)(q - u * nx), i = row / 6, rc = row - 6 * i;
    double c = 0.0, r = 0.0;
    if (rc == 3 || rc == 4) {
        const float* y = Y + (u * U + i) * LEB_CHAIN_OUTPUTS + 2 * (rc - 3);
        chain_decode_row(y[0], y[1], &c, &r);
    }
    cb[q] = c;
    rb[q] = r + pad;
}

// NN surrogate inputs: one thread per (unit, network input c); row of 2n
// floats [a~ (n), 20 rho (n)], rho the half width of
// Delta = [fmin(mu - sigma, 0), fmax(mu + sigma, 0)]
__global__ void nn_features_kernel(const double* z, const double* v, const double* mu, const double* sigma,
                                   int64_t units, int nx, int nu, float* X) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int n = nx + nu;
    if (q >= units * n) return;
    const int64_t u = q / n;
    const int c = (int)(q - u * n);
    const double a = c < nx ? z[u * nx + c] : v[u * nu + (c - nx)];
    const double sg = sigma[q], m = mu ? mu[q] : 0.0;
    const double rho = 0.5 * (fmax(m + sg, 0.0) - fmin(m - sg, 0.0));
    X[u * 2 * n + c] = (float)a;
    X[u * 2 * n + n + c] = (float)(20.0 * rho);
}

// NN surrogate targets: one thread per (unit, output row r); row of 2m
// floats [log hi (m), log -lo (m)]
__global__ void nn_targets_kernel(const double* r_lo, const double* r_hi, int64_t units, int m, float* T) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= units * m) return;
    const int64_t u = q / m;
    const int r = (int)(q - u * m);
    T[u * 2 * m + r] = logf(fmaxf((float)r_hi[q], LOG_FLOOR));
    T[u * 2 * m + m + r] = logf(fmaxf((float)-r_lo[q], LOG_FLOOR));
}

// predicted log-bounds -> [lo, hi]: hi = exp(min(y_hi, 80)), lo = -exp(min(y_lo, 80));
// a prediction that is not finite gives 0
__global__ void nn_decode_kernel(const float* Y, int64_t units, int m, double* r_lo, double* r_hi) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= units * m) return;
    const int64_t u = q / m;
    const int r = (int)(q - u * m);
    const float yh = Y[u * 2 * m + r], yl = Y[u * 2 * m + m + r];
    r_hi[q] = isfinite(yh) ? exp((double)fminf(yh, NN_LOG_CEIL)) : 0.0;
    r_lo[q] = isfinite(yl) ? -exp((double)fminf(yl, NN_LOG_CEIL)) : 0.0;
}

__global__ void scale_sigma_kernel(double* sigma, int64_t count, double f, double a) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < count) sigma[q] = sigma[q] * f + a;
}

__global__ void fill64_kernel(double* dst, int64_t count, double v) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < count) dst[q] = v;
}

static unsigned nbk(int64_t n) { return (unsigned)((n + 255) / 256); }

struct SurWorkspace {
    std::mutex mu;
    float* X = nullptr; float* Y = nullptr; double* cb = nullptr; double* rb = nullptr;
    int64_t cap_nodes = 0, cap_rows = 0;
    float* nX = nullptr; float* nY = nullptr;   // NN family: features and predictions
    int64_t cap_nx = 0, cap_ny = 0;             // floats
    double* dist = nullptr;                     // one trajectory's disturbance-only tube (mu, sigma)
    int64_t cap_dist = 0;                       // doubles
    WsFence fence;
};
static SurWorkspace g_sw;

static int sw_get(int64_t nodes, int64_t rows) {
    if (nodes > g_sw.cap_nodes) {
        if (g_sw.X) (void)hipFree(g_sw.X);
        if (g_sw.Y) (void)hipFree(g_sw.Y);
        g_sw.X = nullptr; g_sw.Y = nullptr; g_sw.cap_nodes = 0;
        if (hipMalloc(&g_sw.X, (size_t)nodes * LEB_CHAIN_FEATURES * sizeof(float)) != hipSuccess ||
            hipMalloc(&g_sw.Y, (size_t)nodes * LEB_CHAIN_OUTPUTS * sizeof(float)) != hipSuccess)
            return LEB_ENOMEM;
        g_sw.cap_nodes = nodes;
    }
    if (rows > g_sw.cap_rows) {
        if (g_sw.cb) (void)hipFree(g_sw.cb);
        if (g_sw.rb) (void)hipFree(g_sw.rb);
        g_sw.cb = nullptr; g_sw.rb = nullptr; g_sw.cap_rows = 0;
        if (hipMalloc(&g_sw.cb, (size_t)rows * sizeof(double)) != hipSuccess ||
            hipMalloc(&g_sw.rb, (size_t)rows * sizeof(double)) != hipSuccess)
            return LEB_ENOMEM;
        g_sw.cap_rows = rows;
    }
    return LEB_OK;
}

static int grow_f32(float** p, int64_t* cap, int64_t count) {
    if (count <= *cap) return LEB_OK;
    if (*p) (void)hipFree(*p);
    *p = nullptr; *cap = 0;
    if (hipMalloc(p, (size_t)count * sizeof(float)) != hipSuccess) { *p = nullptr; return LEB_ENOMEM; }
    *cap = count;
    return LEB_OK;
}

static int grow_f64(double** p, int64_t* cap, int64_t count) {
    if (count <= *cap) return LEB_OK;
    if (*p) (void)hipFree(*p);
    *p = nullptr; *cap = 0;
    if (hipMalloc(p, (size_t)count * sizeof(double)) != hipSuccess) { *p = nullptr; return LEB_ENOMEM; }
    *cap = count;
    return LEB_OK;
}

}  // namespace leb

using namespace leb;

extern "C" int leb_chain_features(const leb_dynamics* dyn, int32_t batch, int32_t N, const double* z, const double* v,
                                  const double* mu, const double* sigma, float* x, void* stream) {
    int rc = check_chain_dynamics(dyn);
    if (rc != LEB_OK) return rc;
    if (dyn->kind != LEB_DYN_PQUAD_CHAIN || batch < 0 || N < 0) return LEB_EINVAL;
    const int64_t units = (int64_t)batch * N;
    if (units == 0) return LEB_OK;
    if (!z || !v || !sigma || !x || ((uintptr_t)x & 15)) return LEB_EINVAL;
    if (units * dyn->n_units > 0x7fffffff) return LEB_EINVAL;
    hipLaunchKernelGGL(chain_features_kernel, dim3(nbk(units * dyn->n_units)), dim3(256), 0, (hipStream_t)stream, z, v,
                       mu, sigma, (int)(units * dyn->n_units), dyn->n_units, dyn->rest_len, x);
    return hipGetLastError() == hipSuccess ? LEB_OK : LEB_EDEVICE;
}

extern "C" int leb_chain_targets(const leb_dynamics* dyn, int32_t batch, int32_t N, const double* r_lo,
                                 const double* r_hi, float* t, void* stream) {
    int rc = check_chain_dynamics(dyn);
    if (rc != LEB_OK) return rc;
    if (dyn->kind != LEB_DYN_PQUAD_CHAIN || batch < 0 || N < 0) return LEB_EINVAL;
    const int64_t units = (int64_t)batch * N;
    if (units == 0) return LEB_OK;
    if (!r_lo || !r_hi || !t || ((uintptr_t)t & 15)) return LEB_EINVAL;
    if (units * dyn->n_units > 0x7fffffff) return LEB_EINVAL;
    hipLaunchKernelGGL(chain_targets_kernel, dim3(nbk(units * dyn->n_units)), dim3(256), 0, (hipStream_t)stream, r_lo,
                       r_hi, (int)(units * dyn->n_units), dyn->n_units, t);
    return hipGetLastError() == hipSuccess ? LEB_OK : LEB_EDEVICE;
}

extern "C" int leb_chain_surrogate_bound(const leb_dynamics* dyn, int32_t batch, int32_t N, const double* z,
                                         const double* v, const double* mu, const double* sigma, leb_surrogate net,
                                         double* c_bar, double* rho_bar, double pad, void* stream) {
    int rc = check_chain_dynamics(dyn);
    if (rc != LEB_OK) return rc;
    if (dyn->kind != LEB_DYN_PQUAD_CHAIN || batch < 0 || N < 0 || !net || !(pad >= 0.0)) return LEB_EINVAL;
    int32_t din = 0, dout = 0;
    if (leb_surrogate_dims(net, &din, &dout) || din != LEB_CHAIN_FEATURES || dout != LEB_CHAIN_OUTPUTS)
        return LEB_EINVAL;
    const int64_t units = (int64_t)batch * N;
    if (units == 0) return LEB_OK;
    if (!z || !v || !sigma || !c_bar || !rho_bar) return LEB_EINVAL;
    if (units * dyn->n_units > 0x7fffffff) return LEB_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    return surrogate_chain_sweep(net, z, v, mu, sigma, (int)(units * dyn->n_units), dyn->n_units, dyn->rest_len, pad,
                                 c_bar, rho_bar, s);
}

extern "C" int leb_nn_features(int32_t nx, int32_t nu, int32_t batch, int32_t N, const double* z, const double* v,
                               const double* mu, const double* sigma, float* x, void* stream) {
    if (nx < 1 || nu < 0 || 2 * (nx + nu) > LEB_NN_MAX_FEATURES || batch < 0 || N < 0) return LEB_EINVAL;
    const int64_t units = (int64_t)batch * N;
    if (units == 0) return LEB_OK;
    if (!z || (nu > 0 && !v) || !sigma || !x || ((uintptr_t)x & 7)) return LEB_EINVAL;
    const int64_t cnt = units * (nx + nu);
    hipLaunchKernelGGL(nn_features_kernel, dim3(nbk(cnt)), dim3(256), 0, (hipStream_t)stream, z, v, mu, sigma, units,
                       (int)nx, (int)nu, x);
    return hipGetLastError() == hipSuccess ? LEB_OK : LEB_EDEVICE;
}

extern "C" int leb_nn_targets(int32_t m, int32_t batch, int32_t N, const double* r_lo, const double* r_hi, float* t,
                              void* stream) {
    if (m < 1 || 2 * m > LEB_NN_MAX_FEATURES || batch < 0 || N < 0) return LEB_EINVAL;
    const int64_t units = (int64_t)batch * N;
    if (units == 0) return LEB_OK;
    if (!r_lo || !r_hi || !t || ((uintptr_t)t & 7)) return LEB_EINVAL;
    hipLaunchKernelGGL(nn_targets_kernel, dim3(nbk(units * m)), dim3(256), 0, (hipStream_t)stream, r_lo, r_hi, units,
                       (int)m, t);
    return hipGetLastError() == hipSuccess ? LEB_OK : LEB_EDEVICE;
}

extern "C" int leb_nn_surrogate_bound(leb_surrogate net, int32_t nx, int32_t nu, int32_t batch, int32_t N,
                                      const double* z, const double* v, const double* mu, const double* sigma,
                                      double* r_lo, double* r_hi, void* stream) {
    if (!net || nx < 1 || nu < 0 || batch < 0 || N < 0) return LEB_EINVAL;
    int32_t din = 0, dout = 0;
    if (leb_surrogate_dims(net, &din, &dout) || din != 2 * (nx + nu) || dout < 2 || (dout & 1)) return LEB_EINVAL;
    const int64_t units = (int64_t)batch * N;
    if (units == 0) return LEB_OK;
    if (!z || (nu > 0 && !v) || !sigma || !r_lo || !r_hi) return LEB_EINVAL;
    if (units > 0x7fffffff) return LEB_EINVAL;
    const int m = dout / 2;
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lock(g_sw.mu);
    int rc;
    if ((rc = grow_f32(&g_sw.nX, &g_sw.cap_nx, units * din)) || (rc = grow_f32(&g_sw.nY, &g_sw.cap_ny, units * dout)))
        return rc;
    if ((rc = g_sw.fence.enter(s))) return rc;
    WsFenceScope leave{g_sw.fence, s};
    if ((rc = leb_nn_features(nx, nu, batch, N, z, v, mu, sigma, g_sw.nX, stream))) return rc;
    if ((rc = leb_mlp_fwd_bf16(net, (int32_t)units, g_sw.nX, g_sw.nY, stream))) return rc;
    hipLaunchKernelGGL(nn_decode_kernel, dim3(nbk(units * m)), dim3(256), 0, s, g_sw.nY, units, m, r_lo, r_hi);
    return hipGetLastError() == hipSuccess ? LEB_OK : LEB_EDEVICE;
}

extern "C" int leb_fixed_point_learned(const leb_dynamics* dyn, int32_t batch, int32_t N, const double* z,
                                       const double* v, const double* phi, const double* e, const leb_fp_options* opt,
                                       const leb_warm_start* ws, double* mu, double* sigma, uint32_t* certified,
                                       int32_t* sweeps_out, void* stream) {
    int rc = check_chain_dynamics(dyn);
    if (rc != LEB_OK) return rc;
    if (dyn->kind != LEB_DYN_PQUAD_CHAIN) return LEB_ENOTSUP;
    if (!ws || !ws->net || !sweeps_out || batch < 0 || N < 0) return LEB_EINVAL;
    if (ws->sweeps < 0 || !(ws->margin >= 0.0) || !isfinite(ws->margin)) return LEB_EINVAL;
    if ((rc = fp_check_args(opt, e, N))) return rc;      // before any launch
    int32_t din = 0, dout = 0;
    if (leb_surrogate_dims(ws->net, &din, &dout) || din != LEB_CHAIN_FEATURES || dout != LEB_CHAIN_OUTPUTS)
        return LEB_EINVAL;
    *sweeps_out = 0;
    const int64_t units = (int64_t)batch * N;
    if (units == 0) return LEB_OK;
    if (!z || !v || !mu || !sigma || !certified || (N > 1 && !phi)) return LEB_EINVAL;
    const void* ptrs[] = {z, v, phi, mu, sigma};
    for (const void* p : ptrs)
        if (p && ((uintptr_t)p & 7)) return LEB_EINVAL;
    const int U = dyn->n_units, nx = dyn->nx, n = dyn->nx + dyn->nu;
    const int64_t nodes = units * U;
    if (nodes > 0x7fffffff) return LEB_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    {
        std::lock_guard<std::mutex> lock(g_sw.mu);
        if ((rc = sw_get(nodes, units * nx))) return rc;
        if ((rc = g_sw.fence.enter(s))) return rc;
        WsFenceScope leave{g_sw.fence, s};
        // C_0: the disturbance-only tube (centre 0).  It is the same for every
        // trajectory, so the first surrogate sweep reads one trajectory's copy;
        // without surrogate sweeps it is written out whole and inflated below.
        if (ws->sweeps > 0) {
            if ((rc = grow_f64(&g_sw.dist, &g_sw.cap_dist, 2 * (int64_t)N * n))) return rc;
            if ((rc = launch_disturbance_tube(1, N, U, phi, e, opt->pad, g_sw.dist, g_sw.dist + (int64_t)N * n, s)))
                return rc;
        } else if ((rc = launch_disturbance_tube(batch, N, U, phi, e, opt->pad, mu, sigma, s))) {
            return rc;
        }
        // surrogate sweeps: C <- T(surrogate bound of C); the last one stores sigma
        // inflated, sigma (1 + margin) + inflate_abs: the warm start above the
        // surrogate's fixed point
        for (int t = 0; t < ws->sweeps; ++t) {
            rc = t == 0 ? surrogate_chain_sweep(ws->net, z, v, nullptr, g_sw.dist + (int64_t)N * n, (int)nodes, U,
                                                dyn->rest_len, opt->pad, g_sw.cb, g_sw.rb, s, true, N)
                        : surrogate_chain_sweep(ws->net, z, v, mu, sigma, (int)nodes, U, dyn->rest_len, opt->pad,
                                                g_sw.cb, g_sw.rb, s, true);
            if (rc) return rc;
            const bool last = t == ws->sweeps - 1;
            if ((rc = launch_tube_map_compact(batch, N, U, phi, e, opt->pad, g_sw.cb, g_sw.rb, mu, sigma, s,
                                              last ? 1.0 + ws->margin : 1.0, last ? opt->inflate_abs : 0.0)))
                return rc;
        }
        if (ws->sweeps == 0) {
            hipLaunchKernelGGL(scale_sigma_kernel, dim3(nbk(units * n)), dim3(256), 0, s, sigma, units * n,
                               1.0 + ws->margin, opt->inflate_abs);
            if (hipGetLastError() != hipSuccess) return LEB_EDEVICE;
        }
    }
    leb_fp_options o = *opt;
    o.warm = 1;
    return leb_fixed_point_solve(dyn, batch, N, z, v, phi, e, &o, mu, sigma, certified, sweeps_out, stream);
}
