// pbh_node.hpp -- one node of one timestep of the chain in the path-based
// Hessian bound (Theorem 1): its coordinates loaded into registers, spring
// i (to node i+1) and the node's two non-linear rows.  Shared by the bound
// kernel and the fused fixed-point sweep, so both evaluate the same
// expressions in the same order.
//
// A lane holds node i of timestep t.  spring_step evaluates spring i and
// hands node i+1 its terms (a SpringOut in LDS); after a barrier that
// covers the lanes of the timestep, node_step adds the left spring's terms
// and the attitude block and returns the node's rows 3 (vx) and 4 (vz).
#pragma once
#include "ivl.hpp"
#include "node.hpp"
#include "pbh_common.hpp"

namespace leb {

struct SpringOut {      // what spring i passes to node i+1 (row i+1)
    double xlo, xhi, zlo, zhi;      // -(cross + own-of-node-i terms), already scaled
    IV<float> L[5];                 // node i+1's shared own-position entries
    uint32_t unbounded;
    uint32_t pad_;
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

// input flags of the node's coordinates (bad input, hull extended)
__device__ __forceinline__ uint32_t node_flags(const NodeIn& d) {
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
    return f;
}

struct NodeConsts {
    double c;        // dt / m
    double L0;       // spring rest length
    double K3, K15, K1, K05;   // 3, 1.5, 1, 0.5 times k_spring rest_len c (all >= 0 for k_spring >= 0)
};
__device__ __forceinline__ NodeConsts node_consts(double c, double kL, double L0) {
    NodeConsts k;
    k.c = c; k.L0 = L0;
    k.K3 = 3.0 * kL * c; k.K15 = 1.5 * kL * c; k.K1 = kL * c; k.K05 = 0.5 * kL * c;
    return k;
}

// what a lane keeps from spring_step for node_step
struct SpringKeep {
    IV<float> Dx, Dz, Dth, Du1, Du2;
    div_ rx, rz;          // spring i's terms for row i
    IV<float> R[5];       // node i's shared own-position entries (right spring)
    uint32_t unb;         // spring i has no finite bound
};

// Spring i (nodes i, i+1) when right; writes *out (right only) and returns
// whether the spring is unbounded through k.unb.
__device__ __forceinline__ void spring_step(const NodeConsts& K, const NodeIn& d, bool right, SpringKeep& k,
                                            SpringOut* out) {
    k.Dx = disp_interval(d.ms[0], d.ss[0]); k.Dz = disp_interval(d.ms[1], d.ss[1]);
    k.Dth = disp_interval(d.ms[2], d.ss[2]);
    k.Du1 = disp_interval(d.ms[6], d.ss[6]); k.Du2 = disp_interval(d.ms[7], d.ss[7]);
    k.rx = {0.0, 0.0}; k.rz = {0.0, 0.0};
#pragma unroll
    for (int q = 0; q < 5; ++q) k.R[q] = iv(0.0f, 0.0f);
    k.unb = 0;
    if (!right) return;
    SpringSetup st;
    spring_setup_v(d.zs[0], d.zs[1], d.zj[0], d.zj[1], k.Dx, k.Dz, disp_interval(d.mj[0], d.sj[0]),
                   disp_interval(d.mj[1], d.sj[1]), K.L0, st);
    AccPrimal acc;
    SpringPieces<float> pc;
    const bool ok = spring_core<float, AccPrimal>(st.dxA, st.dxB, st.dz0, st.dz1, st.dz2, st.Dxi, st.Dzi, st.Dxj,
                                                  st.Dzj, maskv(st.Dxi), maskv(st.Dzi), maskv(st.Dxj),
                                                  maskv(st.Dzj), K.K3, K.K15, K.K1, K.K05, acc, pc);
    SpringOut o = {};
    if (ok) {
        k.rx.lo = acc.a[S_CX].lo + acc.a[S_BX].lo; k.rx.hi = acc.a[S_CX].hi + acc.a[S_BX].hi;
        k.rz.lo = acc.a[S_CZ].lo + acc.a[S_BZ].lo; k.rz.hi = acc.a[S_CZ].hi + acc.a[S_BZ].hi;
        // row i+1 receives -(cross + node i's own pairs)
        o.xlo = -(acc.a[S_CX].hi + acc.a[S_AX].hi); o.xhi = -(acc.a[S_CX].lo + acc.a[S_AX].lo);
        o.zlo = -(acc.a[S_CZ].hi + acc.a[S_AZ].hi); o.zhi = -(acc.a[S_CZ].lo + acc.a[S_AZ].lo);
#pragma unroll
        for (int q = 0; q < 5; ++q) { o.L[q] = pc.L[q]; k.R[q] = pc.R[q]; }
        o.unbounded = 0;
    } else {
        k.unb = 1;
        o.unbounded = 1;
    }
    *out = o;
}

// Node i: attitude block, the left spring's terms (left == NULL for node 0),
// shared position pairs.  ft: the timestep's flags.  Rows 3 and 4 of the
// node as [lo3, hi3], [lo4, hi4]; a bad input makes every row of the node
// (-inf, inf) (*all_inf = true), an unbounded spring rows 3 and 4.
__device__ __forceinline__ void node_step(const NodeConsts& K, int U, const NodeIn& d, const SpringKeep& k,
                                          const SpringOut* left, uint32_t ft, double* lo34, double* hi34,
                                          bool* all_inf) {
    IV<float> L[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) L[q] = iv(0.0f, 0.0f);
    div_ ox = k.rx, oz = k.rz;
    uint32_t row_unb = k.unb;
    if (left) {
        row_unb |= left->unbounded;
        ox.lo += left->xlo; ox.hi += left->xhi; oz.lo += left->zlo; oz.hi += left->zhi;
#pragma unroll
        for (int q = 0; q < 5; ++q) L[q] = left->L[q];
    }
    NodeTerms nt;
    node_terms(d.zs[2], d.vs[0] + d.vs[1], k.Dth, k.Du1, k.Du2, k.Dx, k.Dz, k.R, L, U > 1 && !row_unb, K.c, K.K15,
               K.K1, K.K05, maskv(k.Dth), maskv(k.Du1), maskv(k.Du2), maskv(k.Dx), maskv(k.Dz), nt);
#pragma unroll
    for (int q = 0; q < 12; ++q) {
        div_& acc = node_term_row(q) == 0 ? ox : oz;
        const float a = nt.neg[q] ? nt.T[q].hi : nt.T[q].lo;
        const float b = nt.neg[q] ? nt.T[q].lo : nt.T[q].hi;
        acc.lo = __builtin_fma(nt.k[q], (double)a, acc.lo);
        acc.hi = __builtin_fma(nt.k[q], (double)b, acc.hi);
    }
    *all_inf = (ft & LEB_FLAG_BAD_INPUT) != 0u;
    if (*all_inf || row_unb) {
        lo34[0] = lo34[1] = -INFINITY; hi34[0] = hi34[1] = INFINITY;
    } else {
        // all lower-end summands are <= 0 and all upper-end summands >= 0,
        // so 2^-45 relative covers every FP64 rounding in the sums
        lo34[0] = wlo64(ox.lo); hi34[0] = whi64(ox.hi); lo34[1] = wlo64(oz.lo); hi34[1] = whi64(oz.hi);
    }
}

// zonotope packaging of a row [lo, hi] (eq. zono_map): centre, radius + pad
__device__ __forceinline__ void row_zono(double lo, double hi, double pad, double* cb, double* rb) {
    if (isfinite(lo) && isfinite(hi)) {
        *cb = 0.5 * (lo + hi);
        double r = fmax(hi - *cb, *cb - lo);
        *rb = r + fabs(r) * 0x1p-50 + pad;
    } else {
        *cb = 0.0;
        *rb = INFINITY;
    }
}

// Spring i and node i of timestep lt; s_sp [T][U], s_flag [T] (cleared).
// Contains one workgroup barrier.  Args supplies U, c (dt/m), kL, L0, pad and
// compact (1: c_bar, rho_bar hold rows 3 and 4 of each node only).
template <class Args>
__device__ __forceinline__ void node_pass(const Args& A, const TileRef& t, const NodeIn& d, int lt, int i,
                                          SpringOut* s_sp, uint32_t* s_flag) {
    const int U = A.U, nx = 6 * U;
    const bool active = lt < t.nloc;
    const bool right = active && i < U - 1;      // spring i exists
    if (active) {
        const uint32_t f = node_flags(d);
        if (f) atomicOr(&s_flag[lt], f);
    }
    const NodeConsts K = node_consts(A.c, A.kL, A.L0);
    SpringKeep k;
    spring_step(K, d, right, k, &s_sp[lt * U + i]);
    if (k.unb) atomicOr(&s_flag[lt], LEB_FLAG_UNBOUNDED);
    __syncthreads();      // spring terms and flags complete
    if (!active) return;
    const uint32_t ft = s_flag[lt];
    double lo34[2], hi34[2];
    bool all_inf;
    node_step(K, U, d, k, i > 0 ? &s_sp[lt * U + i - 1] : nullptr, ft, lo34, hi34, &all_inf);
    double lo[6], hi[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        lo[c] = all_inf ? -INFINITY : 0.0;
        hi[c] = all_inf ? INFINITY : 0.0;
    }
    lo[3] = lo34[0]; hi[3] = hi34[0]; lo[4] = lo34[1]; hi[4] = hi34[1];
    const int64_t o = (int64_t)lt * nx + 6 * i;
    if (t.RLO) {
#pragma unroll
        for (int c = 0; c < 6; ++c) { t.RLO[o + c] = lo[c]; t.RHI[o + c] = hi[c]; }
    }
    if (t.CB && A.compact) {
        // the four affine rows are exactly (0, pad) unless the unit is bad, and then
        // rows 3 and 4 are not finite either
        const int64_t o2 = 2 * ((int64_t)lt * U + i);
        row_zono(lo[3], hi[3], A.pad, &t.CB[o2], &t.RB[o2]);
        row_zono(lo[4], hi[4], A.pad, &t.CB[o2 + 1], &t.RB[o2 + 1]);
    } else if (t.CB) {
#pragma unroll
        for (int c = 0; c < 6; ++c) row_zono(lo[c], hi[c], A.pad, &t.CB[o + c], &t.RB[o + c]);
    }
    if (t.FL && i == 0) t.FL[lt] = (ft & LEB_FLAG_BAD_INPUT) ? (ft & ~LEB_FLAG_UNBOUNDED) : ft;
}

}  // namespace leb
