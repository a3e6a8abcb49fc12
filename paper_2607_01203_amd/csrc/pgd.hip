// pgd.hip -- refinement of the nominal point by projected gradient descent
// on the bound's width (the nominal-point optimization of the results
// section, Table II): find the nominal (linearization) point a~ within
// a0 +/- radius sigma of the start a0 whose path-based bound is the narrowest,
//     W(a~) = sum_l (r_hi,l - r_lo,l),
// over either
//   * the travelling box a~ + mu0 +/- sigma (fixed perturbation radius, the
//     set centred on the nominal point): dW/da~ = dW/dz at fixed mu = mu0, or
//   * the fixed box (a0 + mu0) +/- sigma, written a~ + mu +/- sigma with
//     mu = a0 + mu0 - a~: dW/da~ = dW/dz - dW/dmu,
// the derivatives from the adjoint (leb_backward).  Each step moves every
// coordinate by a sign step, lr radius sigma (1 - s / steps), and projects
// back onto the search box; the narrowest iterate seen (the start included)
// is returned.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <mutex>

#include "leb.h"
#include "leb_internal.hpp"

namespace leb {

int launch_pbh_bwd(const leb_dynamics* dyn, int64_t units, const double* z, const double* v, const double* mu,
                   const double* sigma, const double* g_lo, const double* g_hi, double* gz, double* gv,
                   double* gmu, double* gsigma, hipStream_t stream);

struct PgdBufs {
    double *z, *v, *mu, *lo, *hi, *glo, *ghi, *gz, *gv, *gmu, *gsg, *best;
};

// start: a~ = a0, mu = mu0; outputs = a0; best width +inf; upstream adjoints -1 (lo), +1 (hi)
__global__ void pgd_init_kernel(const double* z0, const double* v0, const double* mu0, PgdBufs B, double* zo,
                                double* vo, int64_t units, int nx, int nu) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int n = nx + nu;
    if (q >= units * n) return;
    const int64_t u = q / n;
    const int i = (int)(q - u * n);
    const double a = i < nx ? z0[u * nx + i] : v0[u * nu + (i - nx)];
    if (i < nx) { B.z[u * nx + i] = a; zo[u * nx + i] = a; B.glo[u * nx + i] = -1.0; B.ghi[u * nx + i] = 1.0; }
    else { B.v[u * nu + i - nx] = a; vo[u * nu + i - nx] = a; }
    B.mu[q] = mu0 ? mu0[q] : 0.0;
    if (i == 0) B.best[u] = INFINITY;
}

// width of every unit's bound; keep the narrowest iterate (one thread per unit)
__global__ void pgd_width_kernel(PgdBufs B, double* zo, double* vo, double* width, double* width0, int64_t units,
                                 int nx, int nu, int first) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= units) return;
    double w = 0.0;
    for (int l = 0; l < nx; ++l) w += B.hi[u * nx + l] - B.lo[u * nx + l];
    if (first && width0) width0[u] = w;
    if (w < B.best[u]) {
        B.best[u] = w;
        for (int i = 0; i < nx; ++i) zo[u * nx + i] = B.z[u * nx + i];
        for (int i = 0; i < nu; ++i) vo[u * nu + i] = B.v[u * nu + i];
    }
    if (width) width[u] = B.best[u];
}

// a~ <- clamp(a~ - step sign(dW/da~), a0 +/- radius sigma); for the fixed box mu = a0 + mu0 - a~
// (one thread per coordinate)
__global__ void pgd_update_kernel(const double* z0, const double* v0, const double* mu0, const double* sigma,
                                  PgdBufs B, int64_t units, int nx, int nu, double radius, double frac,
                                  int fixed_box) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int n = nx + nu;
    if (q >= units * n) return;
    const int64_t u = q / n;
    const int i = (int)(q - u * n);
    const double a0 = i < nx ? z0[u * nx + i] : v0[u * nu + (i - nx)];
    double* ap = i < nx ? &B.z[u * nx + i] : &B.v[u * nu + (i - nx)];
    double g = i < nx ? B.gz[u * nx + i] : B.gv[u * nu + (i - nx)];
    if (fixed_box) g -= B.gmu[q];
    const double r = radius * sigma[q];
    double a = *ap;
    if (g > 0.0) a -= frac * r;
    else if (g < 0.0) a += frac * r;
    a = fmin(fmax(a, a0 - r), a0 + r);
    *ap = a;
    if (fixed_box) B.mu[q] = a0 + (mu0 ? mu0[q] : 0.0) - a;
}

struct PgdWorkspace {
    std::mutex mu;
    double* buf = nullptr;
    size_t cap = 0;
    WsFence fence;
};
static PgdWorkspace g_pgd;

}  // namespace leb

using namespace leb;

extern "C" int leb_pgd_nominal(const leb_dynamics* dyn, int32_t batch, int32_t N, const double* z0, const double* v0,
                               const double* mu0, const double* sigma, int32_t fixed_box, double radius,
                               int32_t steps, double lr, double* z, double* v, double* width, double* width0,
                               void* stream) {
    int rc = check_chain_dynamics(dyn);
    if (rc != LEB_OK) return rc;
    if (dyn->kind != LEB_DYN_PQUAD_CHAIN) return LEB_ENOTSUP;
    if (batch < 0 || N < 0 || steps < 0 || (fixed_box != 0 && fixed_box != 1) || !(radius >= 0.0 && radius <= 1.0) ||
        !(lr > 0.0) || !isfinite(lr))
        return LEB_EINVAL;
    const int64_t units = (int64_t)batch * N;
    if (units == 0) return LEB_OK;
    if (!z0 || !v0 || !sigma || !z || !v || !width) return LEB_EINVAL;
    const void* ptrs[] = {z0, v0, mu0, sigma, z, v, width, width0};
    for (const void* p : ptrs)
        if (p && !aligned8(p)) return LEB_EINVAL;
    const int nx = dyn->nx, nu = dyn->nu, n = nx + nu;
    if (units * n > ((int64_t)1 << 40)) return LEB_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lock(g_pgd.mu);
    // z, v, mu, lo, hi, glo, ghi, gz, gv, gmu, gsigma, best
    const size_t need = (size_t)units * (nx + nu + n + nx + nx + nx + nx + nx + nu + n + n + 1);
    if (need > g_pgd.cap) {
        if (g_pgd.buf) (void)hipFree(g_pgd.buf);
        g_pgd.buf = nullptr;
        g_pgd.cap = 0;
        if (hipMalloc(&g_pgd.buf, need * sizeof(double)) != hipSuccess) return LEB_ENOMEM;
        g_pgd.cap = need;
    }
    PgdBufs B;
    double* p = g_pgd.buf;
    auto take = [&](int64_t cnt) { double* q = p; p += cnt; return q; };
    B.z = take(units * nx); B.v = take(units * nu); B.mu = take(units * n); B.lo = take(units * nx);
    B.hi = take(units * nx); B.glo = take(units * nx); B.ghi = take(units * nx); B.gz = take(units * nx);
    B.gv = take(units * nu); B.gmu = take(units * n); B.gsg = take(units * n); B.best = take(units);
    if ((rc = g_pgd.fence.enter(s))) return rc;
    WsFenceScope leave{g_pgd.fence, s};
    const unsigned gc = (unsigned)((units * n + 255) / 256), gu = (unsigned)((units + 255) / 256);
    hipLaunchKernelGGL(pgd_init_kernel, dim3(gc), dim3(256), 0, s, z0, v0, mu0, B, z, v, units, nx, nu);
    for (int st = 0;; ++st) {
        if ((rc = launch_pbh_chain(dyn, units, B.z, B.v, B.mu, sigma, B.lo, B.hi, nullptr, nullptr, 0.0, nullptr, s)))
            return rc;
        hipLaunchKernelGGL(pgd_width_kernel, dim3(gu), dim3(256), 0, s, B, z, v, st == steps ? width : nullptr,
                           st == 0 ? width0 : nullptr, units, nx, nu, st == 0 ? 1 : 0);
        if (st == steps) break;
        if ((rc = launch_pbh_bwd(dyn, units, B.z, B.v, B.mu, sigma, B.glo, B.ghi, B.gz, B.gv,
                                 fixed_box ? B.gmu : nullptr, B.gsg, s)))
            return rc;
        const double frac = lr * (1.0 - (double)st / steps);
        hipLaunchKernelGGL(pgd_update_kernel, dim3(gc), dim3(256), 0, s, z0, v0, mu0, sigma, B, units, nx, nu,
                           radius, frac, fixed_box);
    }
    return hipGetLastError() == hipSuccess ? LEB_OK : LEB_EDEVICE;
}
