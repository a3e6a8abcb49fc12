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
#include "node.hpp"
#include "pbh_common.hpp"

namespace leb {

constexpr int PBH_BLOCK = 256;

struct SpringOut {      // what spring i passes to node i+1 (row i+1)
    double xlo, xhi, zlo, zhi;      // -(cross + own-of-node-i terms), already scaled
    IV<float> L[5];                 // node i+1's shared own-position entries
    uint32_t unbounded;
    uint32_t pad_;
};

struct RowOut { double xlo, xhi, zlo, zhi; };

struct ChainArgs {
    const double* z; const double* v; const double* mu; const double* sigma;
    double* r_lo; double* r_hi; double* c_bar; double* rho_bar; uint32_t* flags;
    const uint32_t* open;   // optional: return at once when *open == 0 (fixed point already certified)
    const PbhTile* tiles;   // optional: one tile (its own pointers, <= T units) per workgroup
    int64_t units;
    int U, T;
    double c;        // dt / m
    double kL;       // k_spring * rest_len
    double L0;
    double pad;
};


__global__ void __launch_bounds__(PBH_BLOCK) pbh_chain_fwd(ChainArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int U = A.U, T = A.T;
    const int nx = 6 * U, nu = 2 * U, n = nx + nu;
    double* s_nom = reinterpret_cast<double*>(smem);                       // [T][n]
    IV<float>* s_d = reinterpret_cast<IV<float>*>(s_nom + (size_t)T * n);  // [T][n]
    SpringOut* s_sp = reinterpret_cast<SpringOut*>(s_d + (size_t)T * n);   // [T][U]
    RowOut* s_row = reinterpret_cast<RowOut*>(s_sp + (size_t)T * U);       // [T][U]
    uint32_t* s_flag = reinterpret_cast<uint32_t*>(s_row + (size_t)T * U); // [T]

    if (A.open && *A.open == 0u) return;
    const int tid = threadIdx.x;
    const double *Z, *V, *MU, *SG;
    double *RLO, *RHI, *CB, *RB;
    uint32_t* FL;
    int nloc;
    if (A.tiles) {
        const PbhTile& tl = A.tiles[blockIdx.x];
        Z = tl.z; V = tl.v; MU = tl.mu; SG = tl.sigma;
        RLO = tl.r_lo; RHI = tl.r_hi; CB = tl.c_bar; RB = tl.rho_bar; FL = tl.flags;
        nloc = tl.n;
    } else {
        const int64_t u0 = (int64_t)blockIdx.x * T;
        const int64_t left = A.units - u0;
        nloc = left < T ? (int)left : T;
        Z = A.z + u0 * nx; V = A.v ? A.v + u0 * nu : nullptr; MU = A.mu ? A.mu + u0 * n : nullptr;
        SG = A.sigma + u0 * n;
        RLO = A.r_lo ? A.r_lo + u0 * nx : nullptr; RHI = A.r_hi ? A.r_hi + u0 * nx : nullptr;
        CB = A.c_bar ? A.c_bar + u0 * nx : nullptr; RB = A.rho_bar ? A.rho_bar + u0 * nx : nullptr;
        FL = A.flags ? A.flags + u0 : nullptr;
    }

    for (int i = tid; i < T; i += PBH_BLOCK) s_flag[i] = 0u;
    __syncthreads();

    // ---- stage inputs (coalesced, 8 loads in flight per thread)
    for (int i0 = tid; i0 < nloc * nx; i0 += 8 * PBH_BLOCK) {
        double x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int idx = i0 + u * PBH_BLOCK;
            x[u] = idx < nloc * nx ? Z[idx] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int idx = i0 + u * PBH_BLOCK;
            if (idx >= nloc * nx) break;
            const int lt = idx / nx, c = idx - lt * nx;
            if (!isfinite(x[u])) atomicOr(&s_flag[lt], LEB_FLAG_BAD_INPUT);
            s_nom[lt * n + c] = x[u];
        }
    }
    for (int i0 = tid; i0 < nloc * nu; i0 += 8 * PBH_BLOCK) {
        double x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int idx = i0 + u * PBH_BLOCK;
            x[u] = idx < nloc * nu ? V[idx] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int idx = i0 + u * PBH_BLOCK;
            if (idx >= nloc * nu) break;
            const int lt = idx / nu, c = idx - lt * nu;
            if (!isfinite(x[u])) atomicOr(&s_flag[lt], LEB_FLAG_BAD_INPUT);
            s_nom[lt * n + nx + c] = x[u];
        }
    }
    for (int i0 = tid; i0 < nloc * n; i0 += 8 * PBH_BLOCK) {
        double sgv[8], mv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int idx = i0 + u * PBH_BLOCK;
            const bool in = idx < nloc * n;
            sgv[u] = in ? SG[idx] : 0.0;
            mv[u] = (in && MU) ? MU[idx] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int idx = i0 + u * PBH_BLOCK;
            if (idx >= nloc * n) break;
            const int lt = idx / n;
            const double sg = sgv[u], m = mv[u];
            uint32_t f = 0;
            if (!isfinite(sg) || !isfinite(m) || !(sg >= 0.0)) f |= LEB_FLAG_BAD_INPUT;
            if (fabs(m) > sg) f |= LEB_FLAG_HULL_EXTENDED;
            if (f) atomicOr(&s_flag[lt], f);
            // Delta = [min(mu - sigma, 0), max(mu + sigma, 0)]; the FP64
            // difference is widened by its rounding bound (exact zeros stay 0).
            double l = m - sg, h = m + sg;
            l = l - fabs(l) * 0x1p-52;
            h = h + fabs(h) * 0x1p-52;
            s_d[idx] = iv(rd32(fmin(l, 0.0)), ru32(fmax(h, 0.0)));
        }
    }
    __syncthreads();

    const int lt = tid / U;
    const int i = tid - lt * U;
    const bool active = (lt < nloc);
    const double* nom = s_nom + lt * n;
    const IV<float>* D = s_d + lt * n;

    // constants with c folded in (all >= 0 for kL >= 0)
    const double K3 = 3.0 * A.kL * A.c, K15 = 1.5 * A.kL * A.c, K1 = A.kL * A.c, K05 = 0.5 * A.kL * A.c;

    // ---- spring i (nodes i, i+1)
    div_ rx = {0.0, 0.0}, rz = {0.0, 0.0};       // spring i's terms for row i
    IV<float> R[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) R[q] = iv(0.0f, 0.0f);
    uint32_t unb = 0;
    if (active && i < U - 1) {
        SpringSetup st;
        spring_setup(nom, D, i, A.L0, st);
        AccPrimal acc;
        SpringPieces<float> pc;
        const bool ok = spring_core<float, AccPrimal>(st.dxA, st.dxB, st.dz0, st.dz1, st.dz2, st.Dxi, st.Dzi,
                                                      st.Dxj, st.Dzj, maskv(st.Dxi), maskv(st.Dzi),
                                                      maskv(st.Dxj), maskv(st.Dzj), K3, K15, K1, K05, acc, pc);
        SpringOut o = {};
        if (ok) {
            rx.lo = acc.a[S_CX].lo + acc.a[S_BX].lo; rx.hi = acc.a[S_CX].hi + acc.a[S_BX].hi;
            rz.lo = acc.a[S_CZ].lo + acc.a[S_BZ].lo; rz.hi = acc.a[S_CZ].hi + acc.a[S_BZ].hi;
            // row i+1 receives -(cross + node i's own pairs)
            o.xlo = -(acc.a[S_CX].hi + acc.a[S_AX].hi); o.xhi = -(acc.a[S_CX].lo + acc.a[S_AX].lo);
            o.zlo = -(acc.a[S_CZ].hi + acc.a[S_AZ].hi); o.zhi = -(acc.a[S_CZ].lo + acc.a[S_AZ].lo);
#pragma unroll
            for (int q = 0; q < 5; ++q) { o.L[q] = pc.L[q]; R[q] = pc.R[q]; }
            o.unbounded = 0;
        } else {
            unb = 1;
            o.unbounded = 1;
            atomicOr(&s_flag[lt], LEB_FLAG_UNBOUNDED);
        }
        s_sp[lt * U + i] = o;
    }
    __syncthreads();

    // ---- node i: attitude block, shared position pairs, totals
    if (active) {
        const int th = 6 * i + 2, pxc = 6 * i, pzc = 6 * i + 1;
        const int u1 = nx + 2 * i, u2 = u1 + 1;
        IV<float> L[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) L[q] = iv(0.0f, 0.0f);
        div_ ox = rx, oz = rz;
        uint32_t row_unb = unb;
        if (i > 0) {
            const SpringOut& o = s_sp[lt * U + i - 1];
            row_unb |= o.unbounded;
            ox.lo += o.xlo; ox.hi += o.xhi; oz.lo += o.zlo; oz.hi += o.zhi;
#pragma unroll
            for (int q = 0; q < 5; ++q) L[q] = o.L[q];
        }
        NodeTerms nt;
        const IV<float> Dth = D[th], Du1 = D[u1], Du2 = D[u2], Dx = D[pxc], Dz = D[pzc];
        node_terms(nom[th], nom[u1] + nom[u2], Dth, Du1, Du2, Dx, Dz, R, L, U > 1 && !row_unb, A.c, K15, K1,
                   K05, maskv(Dth), maskv(Du1), maskv(Du2), maskv(Dx), maskv(Dz), nt);
#pragma unroll
        for (int q = 0; q < 12; ++q) {
            div_& acc = node_term_row(q) == 0 ? ox : oz;
            const float a = nt.neg[q] ? nt.T[q].hi : nt.T[q].lo;
            const float b = nt.neg[q] ? nt.T[q].lo : nt.T[q].hi;
            acc.lo = __builtin_fma(nt.k[q], (double)a, acc.lo);
            acc.hi = __builtin_fma(nt.k[q], (double)b, acc.hi);
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
        const int o = idx;
        if (RLO) {
            RLO[o] = lo;
            RHI[o] = hi;
        }
        if (CB) {
            double cb, rb;
            if (isfinite(lo) && isfinite(hi)) {
                cb = 0.5 * (lo + hi);
                rb = fmax(hi - cb, cb - lo);
                rb = rb + fabs(rb) * 0x1p-50 + A.pad;
            } else { cb = 0.0; rb = INFINITY; }
            CB[o] = cb;
            RB[o] = rb;
        }
    }
    if (FL)
        for (int t = tid; t < nloc; t += PBH_BLOCK) {
            uint32_t f = s_flag[t];
            FL[t] = (f & LEB_FLAG_BAD_INPUT) ? (f & ~LEB_FLAG_UNBOUNDED) : f;
        }
}

__global__ void fill_zero_kernel(double* a, double* b, double* c, double* d, double pad, uint32_t* flags,
                                 int64_t count, int64_t nflags) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = idx; k < count; k += stride) {
        if (a) { a[k] = 0.0; b[k] = 0.0; }
        if (c) { c[k] = 0.0; d[k] = pad; }
    }
    if (flags)
        for (int64_t k = idx; k < nflags; k += stride) flags[k] = 0u;
}

size_t pbh_smem_bytes(int U) { return pbh_smem_bytes_T(U, PBH_BLOCK / U); }

size_t pbh_smem_bytes_T(int U, int T) {
    const int n = 8 * U;
    return (size_t)T * n * sizeof(double) + (size_t)T * n * sizeof(IV<float>) + (size_t)T * U * sizeof(SpringOut)
         + (size_t)T * U * sizeof(RowOut) + (size_t)T * sizeof(uint32_t) + 16;
}

int launch_pbh_chain(const leb_dynamics* dyn, int64_t units, const double* z, const double* v,
                     const double* mu, const double* sigma, double* r_lo, double* r_hi, double* c_bar,
                     double* rho_bar, double pad, uint32_t* flags, hipStream_t stream, const uint32_t* open) {
    ChainArgs a;
    a.z = z; a.v = v; a.mu = mu; a.sigma = sigma;
    a.r_lo = r_lo; a.r_hi = r_hi; a.c_bar = c_bar; a.rho_bar = rho_bar; a.flags = flags;
    a.open = open;
    a.tiles = nullptr;
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

int launch_pbh_tiles(const leb_dynamics* dyn, const PbhTile* tiles, int n_tiles, int T, hipStream_t stream) {
    if (n_tiles == 0) return LEB_OK;
    ChainArgs a = {};
    a.tiles = tiles;
    a.U = dyn->n_units;
    if (T < 1 || T * a.U > PBH_BLOCK) return LEB_EINVAL;
    a.T = T;
    a.c = dyn->dt / dyn->m;
    a.kL = dyn->k_spring * dyn->rest_len;
    a.L0 = dyn->rest_len;
    a.pad = 0.0;
    hipLaunchKernelGGL(pbh_chain_fwd, dim3((unsigned)n_tiles), dim3(PBH_BLOCK), pbh_smem_bytes_T(a.U, T), stream, a);
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
