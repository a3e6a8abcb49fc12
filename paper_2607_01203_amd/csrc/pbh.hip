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
// Lane (t, i) = t U + i loads the coordinates of node i at timestep t (and
// the two positions of node i+1 that spring i needs) straight into
// registers: the offset of node i's rows is linear in the lane index, so
// the loads and the stores of the node's six output rows are coalesced.
// The lane evaluates spring i (between nodes i and i+1), hands node i+1
// its terms through LDS, then evaluates node i's two rows.
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


// T timesteps with their own pointers (nloc <= T of them present).
struct TileRef {
    const double *Z, *V, *MU, *SG;
    double *RLO, *RHI, *CB, *RB;
    uint32_t* FL;
    int nloc;
};

// Coordinates of node i at one timestep (state rows 6i.., inputs 2i..) and
// the positions of node i+1 that spring i needs.
struct NodeIn { double zs[6], vs[2], ms[8], ss[8], zj[2], mj[2], sj[2]; };

__device__ __forceinline__ void node_load(const TileRef& t, int U, int lt, int i, NodeIn& d) {
    const int nx = 6 * U, nu = 2 * U, n = nx + nu;
#pragma unroll
    for (int c = 0; c < 6; ++c) d.zs[c] = 0.0;
    d.vs[0] = d.vs[1] = 0.0;
#pragma unroll
    for (int c = 0; c < 8; ++c) { d.ms[c] = 0.0; d.ss[c] = 0.0; }
    d.zj[0] = d.zj[1] = d.mj[0] = d.mj[1] = d.sj[0] = d.sj[1] = 0.0;
    if (lt >= t.nloc) return;
    const bool right = i < U - 1;
    const double* zp = t.Z + (int64_t)lt * nx + 6 * i;
    const double* vp = t.V + (int64_t)lt * nu + 2 * i;
    const double* sp = t.SG + (int64_t)lt * n;
#pragma unroll
    for (int c = 0; c < 6; ++c) { d.zs[c] = zp[c]; d.ss[c] = sp[6 * i + c]; }
    d.vs[0] = vp[0]; d.vs[1] = vp[1];
    d.ss[6] = sp[nx + 2 * i]; d.ss[7] = sp[nx + 2 * i + 1];
    if (t.MU) {
        const double* mp = t.MU + (int64_t)lt * n;
#pragma unroll
        for (int c = 0; c < 6; ++c) d.ms[c] = mp[6 * i + c];
        d.ms[6] = mp[nx + 2 * i]; d.ms[7] = mp[nx + 2 * i + 1];
        if (right) { d.mj[0] = mp[6 * i + 6]; d.mj[1] = mp[6 * i + 7]; }
    }
    if (right) { d.zj[0] = zp[6]; d.zj[1] = zp[7]; d.sj[0] = sp[6 * i + 6]; d.sj[1] = sp[6 * i + 7]; }
}

// Spring i and node i of timestep lt; s_sp [T][U], s_flag [T] (cleared).
// Contains one workgroup barrier.
__device__ __forceinline__ void node_pass(const ChainArgs& A, const TileRef& t, const NodeIn& d, int lt, int i,
                                          SpringOut* s_sp, uint32_t* s_flag) {
    const int U = A.U, nx = 6 * U;
    const bool active = lt < t.nloc;
    const bool right = active && i < U - 1;      // spring i exists
    if (active) {
        uint32_t f = 0;
#pragma unroll
        for (int c = 0; c < 6; ++c)
            if (!isfinite(d.zs[c])) f |= LEB_FLAG_BAD_INPUT;
        if (!isfinite(d.vs[0]) || !isfinite(d.vs[1])) f |= LEB_FLAG_BAD_INPUT;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            if (!isfinite(d.ss[c]) || !isfinite(d.ms[c]) || !(d.ss[c] >= 0.0)) f |= LEB_FLAG_BAD_INPUT;
            if (fabs(d.ms[c]) > d.ss[c]) f |= LEB_FLAG_HULL_EXTENDED;
        }
        if (f) atomicOr(&s_flag[lt], f);
    }
    const IV<float> Dx = disp_interval(d.ms[0], d.ss[0]), Dz = disp_interval(d.ms[1], d.ss[1]);
    const IV<float> Dth = disp_interval(d.ms[2], d.ss[2]);
    const IV<float> Du1 = disp_interval(d.ms[6], d.ss[6]), Du2 = disp_interval(d.ms[7], d.ss[7]);

    // constants with c folded in (all >= 0 for kL >= 0)
    const double K3 = 3.0 * A.kL * A.c, K15 = 1.5 * A.kL * A.c, K1 = A.kL * A.c, K05 = 0.5 * A.kL * A.c;

    // ---- spring i (nodes i, i+1)
    div_ rx = {0.0, 0.0}, rz = {0.0, 0.0};       // spring i's terms for row i
    IV<float> R[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) R[q] = iv(0.0f, 0.0f);
    uint32_t unb = 0;
    if (right) {
        SpringSetup st;
        spring_setup_v(d.zs[0], d.zs[1], d.zj[0], d.zj[1], Dx, Dz, disp_interval(d.mj[0], d.sj[0]),
                       disp_interval(d.mj[1], d.sj[1]), A.L0, st);
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
    __syncthreads();      // spring terms and flags complete

    // ---- node i: attitude block, shared position pairs, totals; the node's six rows out
    if (!active) return;
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
    node_terms(d.zs[2], d.vs[0] + d.vs[1], Dth, Du1, Du2, Dx, Dz, R, L, U > 1 && !row_unb, A.c, K15, K1, K05,
               maskv(Dth), maskv(Du1), maskv(Du2), maskv(Dx), maskv(Dz), nt);
#pragma unroll
    for (int q = 0; q < 12; ++q) {
        div_& acc = node_term_row(q) == 0 ? ox : oz;
        const float a = nt.neg[q] ? nt.T[q].hi : nt.T[q].lo;
        const float b = nt.neg[q] ? nt.T[q].lo : nt.T[q].hi;
        acc.lo = __builtin_fma(nt.k[q], (double)a, acc.lo);
        acc.hi = __builtin_fma(nt.k[q], (double)b, acc.hi);
    }
    const uint32_t ft = s_flag[lt];
    double lo[6], hi[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) { lo[c] = 0.0; hi[c] = 0.0; }
    if (ft & LEB_FLAG_BAD_INPUT) {
#pragma unroll
        for (int c = 0; c < 6; ++c) { lo[c] = -INFINITY; hi[c] = INFINITY; }
    } else if (row_unb) {
        lo[3] = lo[4] = -INFINITY; hi[3] = hi[4] = INFINITY;
    } else {
        // all lower-end summands are <= 0 and all upper-end summands >= 0,
        // so 2^-45 relative covers every FP64 rounding in the sums
        lo[3] = wlo64(ox.lo); hi[3] = whi64(ox.hi); lo[4] = wlo64(oz.lo); hi[4] = whi64(oz.hi);
    }
    const int64_t o = (int64_t)lt * nx + 6 * i;
    if (t.RLO) {
#pragma unroll
        for (int c = 0; c < 6; ++c) { t.RLO[o + c] = lo[c]; t.RHI[o + c] = hi[c]; }
    }
    if (t.CB) {
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            double cb, rb;
            if (isfinite(lo[c]) && isfinite(hi[c])) {
                cb = 0.5 * (lo[c] + hi[c]);
                rb = fmax(hi[c] - cb, cb - lo[c]);
                rb = rb + fabs(rb) * 0x1p-50 + A.pad;
            } else { cb = 0.0; rb = INFINITY; }
            t.CB[o + c] = cb;
            t.RB[o + c] = rb;
        }
    }
    if (t.FL && i == 0) t.FL[lt] = (ft & LEB_FLAG_BAD_INPUT) ? (ft & ~LEB_FLAG_UNBOUNDED) : ft;
}

__global__ void __launch_bounds__(PBH_BLOCK) pbh_chain_fwd(ChainArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int U = A.U, T = A.T;
    const int nx = 6 * U, nu = 2 * U, n = nx + nu;
    SpringOut* s_sp = reinterpret_cast<SpringOut*>(smem);                  // [T][U]
    uint32_t* s_flag = reinterpret_cast<uint32_t*>(s_sp + (size_t)T * U);   // [T]

    if (A.open && *A.open == 0u) return;
    const int tid = threadIdx.x;
    TileRef t0;
    if (A.tiles) {
        const PbhTile& pt = A.tiles[blockIdx.x];
        t0 = TileRef{pt.z, pt.v, pt.mu, pt.sigma, pt.r_lo, pt.r_hi, pt.c_bar, pt.rho_bar, pt.flags, pt.n};
    } else {
        const int64_t u0 = (int64_t)blockIdx.x * T;
        const int64_t left = A.units - u0;
        t0.nloc = left < T ? (int)left : T;
        t0.Z = A.z + u0 * nx; t0.V = A.v + u0 * nu; t0.MU = A.mu ? A.mu + u0 * n : nullptr;
        t0.SG = A.sigma + u0 * n;
        t0.RLO = A.r_lo ? A.r_lo + u0 * nx : nullptr; t0.RHI = A.r_hi ? A.r_hi + u0 * nx : nullptr;
        t0.CB = A.c_bar ? A.c_bar + u0 * nx : nullptr; t0.RB = A.rho_bar ? A.rho_bar + u0 * nx : nullptr;
        t0.FL = A.flags ? A.flags + u0 : nullptr;
    }
    for (int q = tid; q < T; q += PBH_BLOCK) s_flag[q] = 0u;
    const int lt = tid / U;
    const int i = tid - lt * U;
    NodeIn d0;
    node_load(t0, U, lt, i, d0);
    __syncthreads();      // s_flag cleared
    node_pass(A, t0, d0, lt, i, s_sp, s_flag);
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

size_t pbh_smem_bytes_T(int U, int T) {
    return (size_t)T * U * sizeof(SpringOut) + (size_t)T * sizeof(uint32_t) + 16;
}
size_t pbh_smem_bytes(int U) { return pbh_smem_bytes_T(U, PBH_BLOCK / U); }

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
    hipLaunchKernelGGL(pbh_chain_fwd, dim3((unsigned)blocks), dim3(PBH_BLOCK), pbh_smem_bytes(a.U), stream, a);
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
