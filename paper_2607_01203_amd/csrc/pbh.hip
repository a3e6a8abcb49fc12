// pbh.hip -- path-based Hessian (PBH) linearization-error bound on gfx950.
//
// Theorem 1 (eq. path_based_hessian): for each output row l,
//   R_l = sum_{j<k} [H_l,kj](X^(j)) (Delta_j Delta_k) + 1/2 sum_k [H_l,kk](X^(k)) Delta_k^2,
// where X^(p) frees the coordinates up to p and pins the rest at the nominal
// point (section IV.A, coordinate-wise path).
//
// Dynamics: a chain of U planar quadrotors with springs between neighbours
// (U = 1 is a single quadrotor).  Only the velocity rows vx_i+, vz_i+ are
// non-linear.  Their Hessian entries are
//   - attitude block over X^(theta_i) (inputs pinned):
//       vx: (theta,theta) c s~ sin(Theta), (u_a,theta) -c cos(Theta)
//       vz: (theta,theta) -c s~ cos(Theta), (u_a,theta) -c sin(Theta)
//     with c = dt/m, s~ = u1~ + u2~;
//   - spring block: the non-linear part of the spring force is
//     -k L0 grad|d|, so its Hessian in the separation d is the (fully
//     symmetric) third-derivative tensor of |d| times -k L0.  With
//     a = dx^2, b = dz^2, q = 1/(s2^2 sqrt(s2)), s2 = a + b, the canonical
//     inclusion functions are
//       Txxx = 3kL0 dx b q,  Txxz = -kL0 dz (2a - b) q,
//       Txzz =  kL0 dx (a - 2b) q,  Tzzz = 3kL0 dz a q,
//     evaluated over the four prefix boxes of a spring (free coordinates
//     px_i | + pz_i | + px_{i+1} | + pz_{i+1}).
// Point factors (c, kL0, s~, 1/2) are applied in FP64 when terms are
// accumulated; interval products are associative in exact arithmetic, so
// this leaves the enclosure of each canonical expression unchanged.
// Entries that two springs share (a node's own position pairs) are summed
// as intervals before the product with the displacement product.
//
// Work mapping: one workgroup of 256 lanes holds T = 256 / U timesteps.
// Lane (t, i) first evaluates spring i (between nodes i and i+1) of
// timestep t, then node i's two rows.  Spring i hands node i+1 its terms
// through LDS.  Inputs are staged with coalesced loads into LDS and the
// outputs leave through LDS with coalesced stores.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "ivl.hpp"
#include "leb.h"
#include "leb_internal.hpp"

namespace leb {

constexpr int PBH_BLOCK = 256;

struct SpringOut {      // what spring i passes to node i+1 (row i+1)
    double xlo, xhi, zlo, zhi;      // -(cross + own-of-node-i terms), already scaled
    fiv t_xxx3, t_xxz3, t_xzz3, t_xzz4, t_zzz4;   // node i+1's shared own-position entries
    uint32_t unbounded;
    uint32_t pad_;
};

struct RowOut { double xlo, xhi, zlo, zhi; };

struct ChainArgs {
    const double* z; const double* v; const double* mu; const double* sigma;
    double* r_lo; double* r_hi; double* c_bar; double* rho_bar; uint32_t* flags;
    int64_t units;
    int U, T;
    double c;        // dt / m
    double kL;       // k_spring * rest_len
    double L0;
    double pad;
};

__device__ __forceinline__ double wlo64(double x) { return x - fabs(x) * 0x1p-45; }
__device__ __forceinline__ double whi64(double x) { return x + fabs(x) * 0x1p-45; }

__device__ __forceinline__ double mask(fiv d) { return (d.lo != 0.0f || d.hi != 0.0f) ? 1.0 : 0.0; }

// FP64 value with absolute error allowance err -> outward FP32 interval
__device__ __forceinline__ fiv from64(double lo, double hi, double err) {
    return mk(rd32(lo - err), ru32(hi + err));
}

__global__ void __launch_bounds__(PBH_BLOCK) pbh_chain_fwd(ChainArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int U = A.U, T = A.T;
    const int nx = 6 * U, nu = 2 * U, n = nx + nu;
    double* s_nom = reinterpret_cast<double*>(smem);                       // [T][n]
    fiv* s_d = reinterpret_cast<fiv*>(s_nom + (size_t)T * n);              // [T][n]
    SpringOut* s_sp = reinterpret_cast<SpringOut*>(s_d + (size_t)T * n);   // [T][U]
    RowOut* s_row = reinterpret_cast<RowOut*>(s_sp + (size_t)T * U);       // [T][U]
    uint32_t* s_flag = reinterpret_cast<uint32_t*>(s_row + (size_t)T * U); // [T]

    const int tid = threadIdx.x;
    const int64_t u0 = (int64_t)blockIdx.x * T;
    const int64_t left = A.units - u0;
    const int nloc = left < T ? (int)left : T;

    for (int i = tid; i < T; i += PBH_BLOCK) s_flag[i] = 0u;
    __syncthreads();

    // ---- stage inputs (coalesced)
    for (int idx = tid; idx < nloc * nx; idx += PBH_BLOCK) {
        int lt = idx / nx, c = idx - lt * nx;
        double x = A.z[u0 * nx + idx];
        if (!isfinite(x)) atomicOr(&s_flag[lt], LEB_FLAG_BAD_INPUT);
        s_nom[lt * n + c] = x;
    }
    for (int idx = tid; idx < nloc * nu; idx += PBH_BLOCK) {
        int lt = idx / nu, c = idx - lt * nu;
        double x = A.v[u0 * nu + idx];
        if (!isfinite(x)) atomicOr(&s_flag[lt], LEB_FLAG_BAD_INPUT);
        s_nom[lt * n + nx + c] = x;
    }
    for (int idx = tid; idx < nloc * n; idx += PBH_BLOCK) {
        int lt = idx / n;
        double sg = A.sigma[u0 * n + idx];
        double m = A.mu ? A.mu[u0 * n + idx] : 0.0;
        uint32_t f = 0;
        if (!isfinite(sg) || !isfinite(m) || !(sg >= 0.0)) f |= LEB_FLAG_BAD_INPUT;
        if (fabs(m) > sg) f |= LEB_FLAG_HULL_EXTENDED;
        if (f) atomicOr(&s_flag[lt], f);
        // Delta = [min(mu - sigma, 0), max(mu + sigma, 0)]; the FP64
        // difference is widened by its rounding bound (exact zeros stay 0).
        double l = m - sg, h = m + sg;
        l = l - fabs(l) * 0x1p-52;
        h = h + fabs(h) * 0x1p-52;
        s_d[idx] = mk(rd32(fmin(l, 0.0)), ru32(fmax(h, 0.0)));
    }
    __syncthreads();

    const int lt = tid / U;
    const int i = tid - lt * U;
    const bool active = (lt < nloc);
    const double* nom = s_nom + lt * n;
    const fiv* D = s_d + lt * n;

    // constants with c folded in (all >= 0 for kL >= 0)
    const double K3 = 3.0 * A.kL * A.c, K15 = 1.5 * A.kL * A.c, K1 = A.kL * A.c, K05 = 0.5 * A.kL * A.c;

    // ---- spring i (nodes i, i+1)
    div_ rx = {0.0, 0.0}, rz = {0.0, 0.0};       // spring i's terms for row i
    fiv R_xxx = mk(0, 0), R_xxz = mk(0, 0), R_xzz1 = mk(0, 0), R_xzz2 = mk(0, 0), R_zzz = mk(0, 0);
    uint32_t unb = 0;
    if (active && i < U - 1) {
        const int pi_ = 6 * i, pj = 6 * (i + 1);
        const double pxi = nom[pi_], pzi = nom[pi_ + 1], pxj = nom[pj], pzj = nom[pj + 1];
        const fiv Dxi = D[pi_], Dzi = D[pi_ + 1], Dxj = D[pj], Dzj = D[pj + 1];
        const double dxn = A.L0 + pxj - pxi;
        const double dzn = pzj - pzi;
        const double sx = fabs(A.L0) + fabs(pxj) + fabs(pxi) + fabs(Dxi.lo) + fabs(Dxi.hi) + fabs(Dxj.lo) + fabs(Dxj.hi);
        const double sz = fabs(pzj) + fabs(pzi) + fabs(Dzi.lo) + fabs(Dzi.hi) + fabs(Dzj.lo) + fabs(Dzj.hi);
        const double ex = sx * 0x1p-50, ez = sz * 0x1p-50;
        // separations over the prefix boxes
        const fiv dxA = from64(dxn - (double)Dxi.hi, dxn - (double)Dxi.lo, ex);                       // V1, V2
        const fiv dxB = from64(dxn + (double)Dxj.lo - (double)Dxi.hi, dxn + (double)Dxj.hi - (double)Dxi.lo, ex); // V3, V4
        const fiv dz0 = from64(dzn, dzn, ez);                                                          // V1
        const fiv dz1 = from64(dzn - (double)Dzi.hi, dzn - (double)Dzi.lo, ez);                        // V2, V3
        const fiv dz2 = from64(dzn + (double)Dzj.lo - (double)Dzi.hi, dzn + (double)Dzj.hi - (double)Dzi.lo, ez); // V4
        const fiv aA = sq(dxA), aB = sq(dxB), b0 = sq(dz0), b1 = sq(dz1), b2 = sq(dz2);
        const fiv s1 = add(aA, b0), s2 = add(aA, b1), s3 = add(aB, b1), s4 = add(aB, b2);
        const float smin = fminf(fminf(s1.lo, s2.lo), fminf(s3.lo, s4.lo));
        unb = !(smin >= 0x1p-40f);
        if (!unb) {
            const fiv q1 = rcp_pos(mul_nn(mul_nn(s1, s1), sqrt_pos(s1)));
            const fiv q2 = rcp_pos(mul_nn(mul_nn(s2, s2), sqrt_pos(s2)));
            const fiv q3 = rcp_pos(mul_nn(mul_nn(s3, s3), sqrt_pos(s3)));
            const fiv q4 = rcp_pos(mul_nn(mul_nn(s4, s4), sqrt_pos(s4)));
            // unit-coefficient third-derivative enclosures per prefix box
            const fiv Txxx1 = mul_nonneg(dxA, mul_nn(b0, q1));
            const fiv Txxz1 = mul(dz0, mul_nonneg(twoa_minus_b(aA, b0), q1));
            const fiv Txzz1 = mul(dxA, mul_nonneg(a_minus_twob(aA, b0), q1));
            const fiv Txxz2 = mul(dz1, mul_nonneg(twoa_minus_b(aA, b1), q2));
            const fiv Txzz2 = mul(dxA, mul_nonneg(a_minus_twob(aA, b1), q2));
            const fiv Tzzz2 = mul_nonneg(dz1, mul_nn(aA, q2));
            const fiv Txxx3 = mul_nonneg(dxB, mul_nn(b1, q3));
            const fiv Txxz3 = mul(dz1, mul_nonneg(twoa_minus_b(aB, b1), q3));
            const fiv Txzz3 = mul(dxB, mul_nonneg(a_minus_twob(aB, b1), q3));
            const fiv Txzz4 = mul(dxB, mul_nonneg(a_minus_twob(aB, b2), q4));
            const fiv Tzzz4 = mul_nonneg(dz2, mul_nn(aB, q4));
            // displacement products (all contain 0) and zero masks
            const double mxi = mask(Dxi), mzi = mask(Dzi), mxj = mask(Dxj), mzj = mask(Dzj);
            const fiv C1 = mul_zz(Dxi, Dxj), C2 = mul_zz(Dxi, Dzj), C3 = mul_zz(Dzi, Dxj), C4 = mul_zz(Dzi, Dzj);
            const fiv Pxxi = sq_z(Dxi), Pxzi = mul_zz(Dxi, Dzi), Pzzi = sq_z(Dzi);
            const fiv Pxxj = sq_z(Dxj), Pxzj = mul_zz(Dxj, Dzj), Pzzj = sq_z(Dzj);
            // cross entries (node i x node i+1): +row i, -row i+1
            div_ cx = {0.0, 0.0}, cz = {0.0, 0.0};
            acc_neg(cx, -K3 * mxi * mxj, mul_z(Txxx1, C1));
            acc_pos(cx, K1 * mxi * mzj, mul_z(Txxz1, C2));
            acc_pos(cx, K1 * mzi * mxj, mul_z(Txxz2, C3));
            acc_neg(cx, -K1 * mzi * mzj, mul_z(Txzz2, C4));
            acc_pos(cz, K1 * mxi * mxj, mul_z(Txxz1, C1));
            acc_neg(cz, -K1 * mxi * mzj, mul_z(Txzz1, C2));
            acc_neg(cz, -K1 * mzi * mxj, mul_z(Txzz2, C3));
            acc_neg(cz, -K3 * mzi * mzj, mul_z(Tzzz2, C4));
            // row i: node i+1's own position pairs (only spring i touches them in row i)
            rx = cx; rz = cz;
            acc_pos(rx, K15 * mxj, mul_z(Txxx3, Pxxj));
            acc_neg(rx, -K1 * mxj * mzj, mul_z(Txxz3, Pxzj));
            acc_pos(rx, K05 * mzj, mul_z(Txzz4, Pzzj));
            acc_neg(rz, -K05 * mxj, mul_z(Txxz3, Pxxj));
            acc_pos(rz, K1 * mxj * mzj, mul_z(Txzz3, Pxzj));
            acc_pos(rz, K15 * mzj, mul_z(Tzzz4, Pzzj));
            // row i+1 (force -F): -(cross + node i's own position pairs)
            div_ ax = cx, az = cz;
            acc_pos(ax, K15 * mxi, mul_z(Txxx1, Pxxi));
            acc_neg(ax, -K1 * mxi * mzi, mul_z(Txxz1, Pxzi));
            acc_pos(ax, K05 * mzi, mul_z(Txzz2, Pzzi));
            acc_neg(az, -K05 * mxi, mul_z(Txxz1, Pxxi));
            acc_pos(az, K1 * mxi * mzi, mul_z(Txzz1, Pxzi));
            acc_pos(az, K15 * mzi, mul_z(Tzzz2, Pzzi));
            SpringOut o;
            o.xlo = -ax.hi; o.xhi = -ax.lo; o.zlo = -az.hi; o.zhi = -az.lo;
            o.t_xxx3 = Txxx3; o.t_xxz3 = Txxz3; o.t_xzz3 = Txzz3; o.t_xzz4 = Txzz4; o.t_zzz4 = Tzzz4;
            o.unbounded = 0;
            s_sp[lt * U + i] = o;
            R_xxx = Txxx1; R_xxz = Txxz1; R_xzz1 = Txzz1; R_xzz2 = Txzz2; R_zzz = Tzzz2;
        } else {
            SpringOut o = {};
            o.unbounded = 1;
            s_sp[lt * U + i] = o;
            atomicOr(&s_flag[lt], LEB_FLAG_UNBOUNDED);
        }
    }
    __syncthreads();

    // ---- node i: attitude block, shared position pairs, totals
    if (active) {
        const int th = 6 * i + 2, pxc = 6 * i, pzc = 6 * i + 1;
        const int u1 = nx + 2 * i, u2 = u1 + 1;
        const fiv Dth = D[th], Du1 = D[u1], Du2 = D[u2], Dx = D[pxc], Dz = D[pzc];
        const double mth = mask(Dth), mu1 = mask(Du1), mu2 = mask(Du2), mx = mask(Dx), mz = mask(Dz);
        const double thn = nom[th];
        const double sn = nom[u1] + nom[u2];
        double tlo = thn + (double)Dth.lo, thi = thn + (double)Dth.hi;
        const double et = (fabs(thn) + fabs(Dth.lo) + fabs(Dth.hi)) * 0x1p-51;
        fiv S, Cs;
        isincos(tlo - et, thi + et, &S, &Cs);
        const fiv Ptt = sq_z(Dth), Ptu1 = mul_zz(Dth, Du1), Ptu2 = mul_zz(Dth, Du2);
        div_ ox = rx, oz = rz;
        const double kth = 0.5 * A.c * sn * mth;
        acc_any(ox, kth, mul_z(S, Ptt));                 //  1/2 c s~ sin(Theta) Dth^2
        acc_neg(ox, -A.c * mth * mu1, mul_z(Cs, Ptu1));  // -c cos(Theta) Dth Du1
        acc_neg(ox, -A.c * mth * mu2, mul_z(Cs, Ptu2));
        acc_any(oz, -kth, mul_z(Cs, Ptt));               // -1/2 c s~ cos(Theta) Dth^2
        acc_neg(oz, -A.c * mth * mu1, mul_z(S, Ptu1));   // -c sin(Theta) Dth Du1
        acc_neg(oz, -A.c * mth * mu2, mul_z(S, Ptu2));
        uint32_t row_unb = unb;
        if (U > 1) {
            fiv L_xxx = mk(0, 0), L_xxz = mk(0, 0), L_xzz3 = mk(0, 0), L_xzz4 = mk(0, 0), L_zzz = mk(0, 0);
            if (i > 0) {
                const SpringOut& o = s_sp[lt * U + i - 1];
                row_unb |= o.unbounded;
                ox.lo += o.xlo; ox.hi += o.xhi; oz.lo += o.zlo; oz.hi += o.zhi;
                L_xxx = o.t_xxx3; L_xxz = o.t_xxz3; L_xzz3 = o.t_xzz3; L_xzz4 = o.t_xzz4; L_zzz = o.t_zzz4;
            }
            if (!row_unb) {
                // own position pairs: right spring (+F) minus left spring (-F), summed before the product
                const fiv Pxx = sq_z(Dx), Pxz = mul_zz(Dx, Dz), Pzz = sq_z(Dz);
                const fiv Gxxx = sub(R_xxx, L_xxx), Gxxz = sub(R_xxz, L_xxz);
                const fiv Gxzz_xz = sub(R_xzz1, L_xzz3), Gxzz_zz = sub(R_xzz2, L_xzz4), Gzzz = sub(R_zzz, L_zzz);
                acc_pos(ox, K15 * mx, mul_z(Gxxx, Pxx));
                acc_neg(ox, -K1 * mx * mz, mul_z(Gxxz, Pxz));
                acc_pos(ox, K05 * mz, mul_z(Gxzz_zz, Pzz));
                acc_neg(oz, -K05 * mx, mul_z(Gxxz, Pxx));
                acc_pos(oz, K1 * mx * mz, mul_z(Gxzz_xz, Pxz));
                acc_pos(oz, K15 * mz, mul_z(Gzzz, Pzz));
            }
        }
        RowOut r;
        if (row_unb) {
            r.xlo = r.zlo = -INFINITY; r.xhi = r.zhi = INFINITY;
        } else {
            // all lower-end summands are <= 0 and all upper-end summands >= 0,
            // so 2^-45 relative covers every FP64 rounding in the sums
            r.xlo = wlo64(ox.lo); r.xhi = whi64(ox.hi); r.zlo = wlo64(oz.lo); r.zhi = whi64(oz.hi);
        }
        s_row[lt * U + i] = r;
    }
    __syncthreads();

    // ---- store (coalesced), zeros on the affine rows
    for (int idx = tid; idx < nloc * nx; idx += PBH_BLOCK) {
        int t = idx / nx, row = idx - t * nx;
        int node = row / 6, rc = row - node * 6;
        uint32_t f = s_flag[t];
        double lo = 0.0, hi = 0.0;
        if (f & LEB_FLAG_BAD_INPUT) { lo = -INFINITY; hi = INFINITY; }
        else if (rc == 3) { lo = s_row[t * U + node].xlo; hi = s_row[t * U + node].xhi; }
        else if (rc == 4) { lo = s_row[t * U + node].zlo; hi = s_row[t * U + node].zhi; }
        const int64_t o = u0 * nx + idx;
        if (A.r_lo) {
            A.r_lo[o] = lo;
            A.r_hi[o] = hi;
        }
        if (A.c_bar) {
            double cb, rb;
            if (isfinite(lo) && isfinite(hi)) {
                cb = 0.5 * (lo + hi);
                rb = fmax(hi - cb, cb - lo);
                rb = rb + fabs(rb) * 0x1p-50 + A.pad;
            } else { cb = 0.0; rb = INFINITY; }
            A.c_bar[o] = cb;
            A.rho_bar[o] = rb;
        }
    }
    if (A.flags)
        for (int t = tid; t < nloc; t += PBH_BLOCK) {
            uint32_t f = s_flag[t];
            A.flags[u0 + t] = (f & LEB_FLAG_BAD_INPUT) ? (f & ~LEB_FLAG_UNBOUNDED) : f;
        }
}

__global__ void fill_zero_kernel(double* a, double* b, double* c, double* d, double pad, uint32_t* flags,
                                 int64_t count, int64_t nflags) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = idx; k < count; k += stride) {
        a[k] = 0.0; b[k] = 0.0;
        if (c) { c[k] = 0.0; d[k] = pad; }
    }
    if (flags)
        for (int64_t k = idx; k < nflags; k += stride) flags[k] = 0u;
}

size_t pbh_smem_bytes(int U) {
    int T = PBH_BLOCK / U, n = 8 * U;
    return (size_t)T * n * sizeof(double) + (size_t)T * n * sizeof(fiv) + (size_t)T * U * sizeof(SpringOut)
         + (size_t)T * U * sizeof(RowOut) + (size_t)T * sizeof(uint32_t) + 16;
}

int launch_pbh_chain(const leb_dynamics* dyn, int64_t units, const double* z, const double* v,
                     const double* mu, const double* sigma, double* r_lo, double* r_hi, double* c_bar,
                     double* rho_bar, double pad, uint32_t* flags, hipStream_t stream) {
    ChainArgs a;
    a.z = z; a.v = v; a.mu = mu; a.sigma = sigma;
    a.r_lo = r_lo; a.r_hi = r_hi; a.c_bar = c_bar; a.rho_bar = rho_bar; a.flags = flags;
    a.units = units;
    a.U = dyn->n_units;
    a.T = PBH_BLOCK / a.U;
    a.c = dyn->dt / dyn->m;
    a.kL = dyn->k_spring * dyn->rest_len;
    a.L0 = dyn->rest_len;
    a.pad = pad;
    int64_t blocks = (units + a.T - 1) / a.T;
    if (blocks > 0x7fffffff) return LEB_EINVAL;
    size_t smem = pbh_smem_bytes(a.U);
    hipLaunchKernelGGL(pbh_chain_fwd, dim3((unsigned)blocks), dim3(PBH_BLOCK), smem, stream, a);
    return hipGetLastError() == hipSuccess ? LEB_OK : LEB_EDEVICE;
}

int launch_fill_zero(int64_t count, double* r_lo, double* r_hi, double* c_bar, double* rho_bar, double pad,
                     uint32_t* flags, int64_t nflags, hipStream_t stream) {
    int64_t blocks = (count + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 65535) blocks = 65535;
    hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, r_lo, r_hi, c_bar,
                       rho_bar, pad, flags, count, nflags);
    return hipGetLastError() == hipSuccess ? LEB_OK : LEB_EDEVICE;
}

}  // namespace leb
