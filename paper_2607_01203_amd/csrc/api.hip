// api.hip -- C-ABI entry points: argument validation and dispatch.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "leb.h"
#include "leb_internal.hpp"

namespace leb {

bool aligned8(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }

int check_chain_dynamics(const leb_dynamics* dyn) {
    if (!dyn) return LEB_EINVAL;
    if (dyn->kind == LEB_DYN_LINEAR) return (dyn->nx >= 0 && dyn->nu >= 0) ? LEB_OK : LEB_EINVAL;
    if (dyn->kind != LEB_DYN_PQUAD_CHAIN) return LEB_ENOTSUP;
    if (dyn->n_units < 1) return LEB_EINVAL;
    if (dyn->n_units > 256) return LEB_ENOTSUP;
    if (dyn->nx != 6 * dyn->n_units || dyn->nu != 2 * dyn->n_units) return LEB_EINVAL;
    if (!(dyn->dt > 0.0) || !(dyn->m > 0.0) || !isfinite(dyn->dt) || !isfinite(dyn->m)) return LEB_EINVAL;
    if (!(dyn->k_spring >= 0.0) || !(dyn->rest_len >= 0.0) || !isfinite(dyn->k_spring) ||
        !isfinite(dyn->rest_len))
        return LEB_EINVAL;
    return LEB_OK;
}

int check_dynamics(const leb_dynamics* dyn) {
    if (!dyn) return LEB_EINVAL;
    switch (dyn->kind) {
    case LEB_DYN_LINEAR:
    case LEB_DYN_PQUAD_CHAIN: return check_chain_dynamics(dyn);
    case LEB_DYN_QUADRATIC:
        if (dyn->nx < 1 || dyn->nu < 0 || !dyn->coeffs || !aligned8(dyn->coeffs)) return LEB_EINVAL;
        return dyn->nx + dyn->nu <= 64 ? LEB_OK : LEB_ENOTSUP;
    case LEB_DYN_SINCOS: return (dyn->nx == 1 || dyn->nx == 2) && dyn->nu == 0 ? LEB_OK : LEB_EINVAL;
    case LEB_DYN_SATELLITE:
    case LEB_DYN_QUAD3D: {
        const bool sat = dyn->kind == LEB_DYN_SATELLITE;
        if (dyn->nx != (sat ? 7 : 12) || dyn->nu != (sat ? 3 : 4)) return LEB_EINVAL;
        if (!(dyn->dt > 0.0) || !isfinite(dyn->dt)) return LEB_EINVAL;
        if (!sat && (!(dyn->m > 0.0) || !isfinite(dyn->m))) return LEB_EINVAL;
        for (int i = 0; i < 3; ++i)
            if (!(dyn->J[i] > 0.0) || !isfinite(dyn->J[i])) return LEB_EINVAL;
        return LEB_OK;
    }
    }
    return LEB_ENOTSUP;
}

int WsFence::enter(hipStream_t s) {
    if (armed && hipStreamWaitEvent(s, ev, 0) != hipSuccess) return LEB_EDEVICE;
    return LEB_OK;
}

int WsFence::leave(hipStream_t s) {
    if (!ev && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        ev = nullptr;
        return LEB_EDEVICE;
    }
    if (hipEventRecord(ev, s) != hipSuccess) return LEB_EDEVICE;
    armed = true;
    return LEB_OK;
}

}  // namespace leb

using namespace leb;

extern "C" int leb_analytic_bound(const leb_dynamics* dyn, int32_t batch, int32_t N, const double* z,
                                  const double* v, const double* mu, const double* sigma, double* r_lo,
                                  double* r_hi, double* c_bar, double* rho_bar, double pad, uint32_t* flags,
                                  double* A, double* B, void* stream) {
    int rc = check_dynamics(dyn);
    if (rc != LEB_OK) return rc;
    if (batch < 0 || N < 0) return LEB_EINVAL;
    if (!(pad >= 0.0) || !isfinite(pad)) return LEB_EINVAL;
    if ((A || B) && dyn->kind != LEB_DYN_PQUAD_CHAIN) return LEB_EINVAL;
    const int64_t units = (int64_t)batch * (int64_t)N;
    if (units == 0) return LEB_OK;
    const int64_t nx = dyn->nx, nu = dyn->nu;
    // outputs come in pairs; at least one pair
    if (!r_lo != !r_hi || !c_bar != !rho_bar || !A != !B) return LEB_EINVAL;
    if (nx > 0 && !r_lo && !c_bar) return LEB_EINVAL;
    // every kind reads the nominal and the radii (the linear kind to validate them)
    if ((nx > 0 && !z) || (nu > 0 && !v) || (nx + nu > 0 && !sigma)) return LEB_EINVAL;
    const void* ptrs[] = {z, v, mu, sigma, r_lo, r_hi, c_bar, rho_bar, A, B};
    for (const void* p : ptrs)
        if (p && !aligned8(p)) return LEB_EINVAL;
    if (flags && (reinterpret_cast<uintptr_t>(flags) & 3u)) return LEB_EINVAL;
    if (units * (nx + nu) > ((int64_t)1 << 46)) return LEB_EINVAL;
    if (A && units * nx * (nx + nu) > ((int64_t)1 << 46)) return LEB_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (dyn->kind != LEB_DYN_PQUAD_CHAIN)
        return launch_small_dyn(dyn, LEB_IH_PATH, units, z, v, mu, sigma, r_lo, r_hi, c_bar, rho_bar, pad, flags,
                                s);
    if ((rc = launch_pbh_chain(dyn, units, z, v, mu, sigma, r_lo, r_hi, c_bar, rho_bar, pad, flags, s))) return rc;
    return A ? launch_chain_jacobians(dyn, units, z, v, A, B, s) : LEB_OK;
}

extern "C" const char* leb_strerror(int code) {
    switch (code) {
    case LEB_OK: return "ok";
    case LEB_EINVAL: return "invalid argument";
    case LEB_ENOMEM: return "device allocation failed";
    case LEB_EDEVICE: return "HIP runtime error";
    case LEB_ENOTSUP: return "not supported";
    case LEB_ESCRATCH: return "problem larger than the fixed scratch of the no-allocation entry point";
    }
    return "unknown status";
}

extern "C" const char* leb_version(void) { return "leb-mi355x 0.1 (gfx950)"; }
