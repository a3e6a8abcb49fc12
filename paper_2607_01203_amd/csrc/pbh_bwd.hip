// pbh_bwd.hip -- adjoint of the path-based Hessian bound (leb_backward).
//
// Gradient of L = sum_{unit,row} g_lo r_lo + g_hi r_hi with respect to the
// nominal trajectory (z, v) and the tube (sigma, mu), for the exact-
// arithmetic bound of Theorem 1 (rounding steps are the identity; every
// selection follows the primal values and takes the first candidate in the
// order lo*lo, lo*hi, hi*lo, hi*hi on a tie).  The paper uses these
// gradients to refine the nominal point (Table II) and to penalise the
// propagated error (eq. linearization_error_cost_penalty).
//
// Interval intermediates are recomputed, never stored:
//   1. spring i primal (the bound kernel's own code, F = float): pieces of
//      node i+1's shared entries go to LDS;
//   2. node i primal and its hand-written reverse: adjoints of the node's
//      displacements, nominal attitude and thrust sum, and of the shared
//      spring pieces (the left spring's go to LDS);
//   3. spring i tangent passes: the same spring code with a forward-mode
//      dual type, one pass per spring input (2 separations, 8 displacement
//      endpoints); each pass contracts the tangents with the adjoints;
//   4. per-coordinate sums in a fixed order (deterministic), then the
//      chain rule through Delta = [min(mu - sigma, 0), max(mu + sigma, 0)].
// Rows that are unbounded, and units with invalid data, contribute nothing.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "leb.h"
#include "leb_internal.hpp"
#include "node.hpp"
#include "pbh_common.hpp"

namespace leb {

constexpr int BWD_BLOCK = 128;

struct BwdArgs {
    const double* z; const double* v; const double* mu; const double* sigma;
    const double* g_lo; const double* g_hi;
    double* gz; double* gv; double* gmu; double* gsigma;
    int64_t units;
    int U, T;
    double c, kL, L0;
};

struct BSpring { IV<float> L[5]; uint32_t unbounded; uint32_t pad_; };
struct RowAdj { double xlo, xhi, zlo, zhi; };
struct NodeGrad { double th, s, dth[2], du1[2], du2[2], dx[2], dz[2]; };
struct SpringGrad { double d[10]; };     // dxn, dzn, Dxi lo/hi, Dzi lo/hi, Dxj lo/hi, Dzj lo/hi
struct PieceAdj { double lo[5], hi[5]; };

// reverse of t_mul_z(a, p) for F = float (first-on-tie selections)
__device__ __forceinline__ void bwd_mul_z(IV<float> a, IV<float> p, double tlo, double thi, double* alo,
                                          double* ahi, double* plo, double* phi) {
    const float c1 = a.lo * p.hi, c2 = a.hi * p.lo;
    if (c1 <= c2) { *alo += tlo * p.hi; *phi += tlo * a.lo; }
    else { *ahi += tlo * p.lo; *plo += tlo * a.hi; }
    const float c0 = a.lo * p.lo, c3 = a.hi * p.hi;
    if (c0 >= c3) { *alo += thi * p.lo; *plo += thi * a.lo; }
    else { *ahi += thi * p.hi; *phi += thi * a.hi; }
}
// reverse of t_sq_z(a) = [0, max(a.lo^2, a.hi^2)]
__device__ __forceinline__ void bwd_sq_z(IV<float> a, double thi, double* alo, double* ahi) {
    const float l2 = a.lo * a.lo, h2 = a.hi * a.hi;
    if (l2 >= h2) *alo += thi * 2.0 * a.lo;
    else *ahi += thi * 2.0 * a.hi;
}

__device__ __forceinline__ double sc_deriv(const SinCos& sc, bool is_sin, int sel, double a64, double b64, bool at_b) {
    // derivative of the selected endpoint value; 0 when the bound is a clamped extremum
    if (sel == 2) return 0.0;
    if (sc.wide) {
        const double x = sel == 0 ? a64 : b64;
        return is_sin ? cos(x) : -sin(x);
    }
    const float x = sel == 0 ? sc.fa : sc.fb;
    (void)at_b;
    return is_sin ? (double)cos_poly(x) : -(double)sin_poly(x);
}

__global__ void __launch_bounds__(BWD_BLOCK) pbh_chain_bwd(BwdArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int U = A.U, T = A.T;
    const int nx = 6 * U, nu = 2 * U, n = nx + nu;
    double* s_nom = reinterpret_cast<double*>(smem);                                 // [T][n]
    IV<float>* s_d = reinterpret_cast<IV<float>*>(s_nom + (size_t)T * n);            // [T][n]
    RowAdj* s_g = reinterpret_cast<RowAdj*>(s_d + (size_t)T * n);                    // [T][U]
    unsigned char* region = reinterpret_cast<unsigned char*>(s_g + (size_t)T * U);
    const size_t region_bytes = (size_t)T * U * (sizeof(BSpring) > sizeof(SpringGrad) ? sizeof(BSpring) : sizeof(SpringGrad));
    BSpring* s_sp = reinterpret_cast<BSpring*>(region);                              // phases 1-2
    SpringGrad* s_gs = reinterpret_cast<SpringGrad*>(region);                        // phases 3-4
    PieceAdj* s_lbar = reinterpret_cast<PieceAdj*>(region + region_bytes);           // [T][U]
    NodeGrad* s_gn = reinterpret_cast<NodeGrad*>(s_lbar + (size_t)T * U);            // [T][U]
    uint32_t* s_unb = reinterpret_cast<uint32_t*>(s_gn + (size_t)T * U);             // [T][U] row unbounded
    uint32_t* s_flag = s_unb + (size_t)T * U;                                        // [T]

    const int tid = threadIdx.x;
    const int64_t u0 = (int64_t)blockIdx.x * T;
    const int64_t left = A.units - u0;
    const int nloc = left < T ? (int)left : T;

    for (int q = tid; q < T; q += BWD_BLOCK) s_flag[q] = 0u;
    __syncthreads();
    for (int idx = tid; idx < nloc * nx; idx += BWD_BLOCK) {
        const int lt = idx / nx, c = idx - lt * nx;
        const double x = A.z[u0 * nx + idx];
        if (!isfinite(x)) atomicOr(&s_flag[lt], LEB_FLAG_BAD_INPUT);
        s_nom[lt * n + c] = x;
        const int rc = c % 6;
        if (rc == 3 || rc == 4) {
            RowAdj& g = s_g[lt * U + c / 6];
            const double gl = A.g_lo[u0 * nx + idx], gh = A.g_hi[u0 * nx + idx];
            if (rc == 3) { g.xlo = gl; g.xhi = gh; } else { g.zlo = gl; g.zhi = gh; }
        }
    }
    for (int idx = tid; idx < nloc * nu; idx += BWD_BLOCK) {
        const int lt = idx / nu, c = idx - lt * nu;
        const double x = A.v[u0 * nu + idx];
        if (!isfinite(x)) atomicOr(&s_flag[lt], LEB_FLAG_BAD_INPUT);
        s_nom[lt * n + nx + c] = x;
    }
    for (int idx = tid; idx < nloc * n; idx += BWD_BLOCK) {
        const int lt = idx / n;
        const double sg = A.sigma[u0 * n + idx];
        const double m = A.mu ? A.mu[u0 * n + idx] : 0.0;
        if (!isfinite(sg) || !isfinite(m) || !(sg >= 0.0)) atomicOr(&s_flag[lt], LEB_FLAG_BAD_INPUT);
        double l = m - sg, h = m + sg;
        l = l - fabs(l) * 0x1p-52;
        h = h + fabs(h) * 0x1p-52;
        s_d[idx] = iv(rd32(fmin(l, 0.0)), ru32(fmax(h, 0.0)));
    }
    __syncthreads();

    const int lt = tid / U;
    const int i = tid - lt * U;
    const bool active = (lt < nloc);
    const double* nom = s_nom + lt * n;
    const IV<float>* D = s_d + lt * n;
    const double K3 = 3.0 * A.kL * A.c, K15 = 1.5 * A.kL * A.c, K1 = A.kL * A.c, K05 = 0.5 * A.kL * A.c;
    const bool bad = active && (s_flag[lt] & LEB_FLAG_BAD_INPUT);

    // ---- 1. spring i primal
    IV<float> R[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) R[q] = iv(0.0f, 0.0f);
    bool spring_ok = false;
    SpringSetup st;
    if (active && i < U - 1) {
        spring_setup(nom, D, i, A.L0, st);
        AccPrimal acc;
        SpringPieces<float> pc;
        spring_ok = spring_core<float, AccPrimal>(st.dxA, st.dxB, st.dz0, st.dz1, st.dz2, st.Dxi, st.Dzi, st.Dxj,
                                                  st.Dzj, 1.0, 1.0, 1.0, 1.0, K3, K15, K1, K05, acc, pc);
        BSpring o;
#pragma unroll
        for (int q = 0; q < 5; ++q) { o.L[q] = spring_ok ? pc.L[q] : iv(0.0f, 0.0f); R[q] = spring_ok ? pc.R[q] : iv(0.0f, 0.0f); }
        o.unbounded = spring_ok ? 0u : 1u;
        o.pad_ = 0;
        s_sp[lt * U + i] = o;
    }
    __syncthreads();

    // ---- 2. node i primal + reverse
    PieceAdj rbar;
#pragma unroll
    for (int q = 0; q < 5; ++q) { rbar.lo[q] = 0.0; rbar.hi[q] = 0.0; }
    if (active) {
        const int th = 6 * i + 2, pxc = 6 * i, pzc = 6 * i + 1;
        const int u1 = nx + 2 * i, u2 = u1 + 1;
        IV<float> L[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) L[q] = iv(0.0f, 0.0f);
        uint32_t row_unb = (i < U - 1 && !spring_ok) ? 1u : 0u;
        if (i > 0) {
            const BSpring& o = s_sp[lt * U + i - 1];
            row_unb |= o.unbounded;
#pragma unroll
            for (int q = 0; q < 5; ++q) L[q] = o.L[q];
        }
        s_unb[lt * U + i] = row_unb;
        RowAdj g = s_g[lt * U + i];
        if (row_unb || bad) { g.xlo = g.xhi = g.zlo = g.zhi = 0.0; }
        const bool own = U > 1 && !row_unb;
        NodeTerms nt;
        const IV<float> Dth = D[th], Du1 = D[u1], Du2 = D[u2], Dx = D[pxc], Dz = D[pzc];
        const double sn = nom[u1] + nom[u2];
        node_terms(nom[th], sn, Dth, Du1, Du2, Dx, Dz, R, L, own, A.c, K15, K1, K05, 1.0, 1.0, 1.0, 1.0, 1.0, nt);
        // term adjoints
        double tlo[12], thi[12];
        double sbar = 0.0;
#pragma unroll
        for (int q = 0; q < 12; ++q) {
            const int row = node_term_row(q);
            const double alo = row == 0 ? g.xlo : g.zlo, ahi = row == 0 ? g.xhi : g.zhi;
            const double k = nt.k[q];
            tlo[q] = k * (nt.neg[q] ? ahi : alo);
            thi[q] = k * (nt.neg[q] ? alo : ahi);
            if (q == 0 || q == 3) {
                // d kappa / d s~ = +-c/2 ; kappa enters through the selected endpoints
                const float a = nt.neg[q] ? nt.T[q].hi : nt.T[q].lo;
                const float b = nt.neg[q] ? nt.T[q].lo : nt.T[q].hi;
                const double dk = (q == 0 ? 0.5 : -0.5) * A.c;
                sbar += dk * (alo * (double)a + ahi * (double)b);
            }
        }
        NodeGrad ng = {};
        ng.s = sbar;
        double Sb_lo = 0, Sb_hi = 0, Cb_lo = 0, Cb_hi = 0;
        double Ptt_lo = 0, Ptt_hi = 0, Pu1_lo = 0, Pu1_hi = 0, Pu2_lo = 0, Pu2_hi = 0;
        const IV<float> S = iv(nt.sc.s.lo, nt.sc.s.hi), Cs = iv(nt.sc.c.lo, nt.sc.c.hi);
        bwd_mul_z(S, nt.Ptt, tlo[0], thi[0], &Sb_lo, &Sb_hi, &Ptt_lo, &Ptt_hi);
        bwd_mul_z(Cs, nt.Ptu1, tlo[1], thi[1], &Cb_lo, &Cb_hi, &Pu1_lo, &Pu1_hi);
        bwd_mul_z(Cs, nt.Ptu2, tlo[2], thi[2], &Cb_lo, &Cb_hi, &Pu2_lo, &Pu2_hi);
        bwd_mul_z(Cs, nt.Ptt, tlo[3], thi[3], &Cb_lo, &Cb_hi, &Ptt_lo, &Ptt_hi);
        bwd_mul_z(S, nt.Ptu1, tlo[4], thi[4], &Sb_lo, &Sb_hi, &Pu1_lo, &Pu1_hi);
        bwd_mul_z(S, nt.Ptu2, tlo[5], thi[5], &Sb_lo, &Sb_hi, &Pu2_lo, &Pu2_hi);
        // displacement products of the attitude block
        bwd_sq_z(Dth, Ptt_hi, &ng.dth[0], &ng.dth[1]);
        bwd_mul_z(Dth, Du1, Pu1_lo, Pu1_hi, &ng.dth[0], &ng.dth[1], &ng.du1[0], &ng.du1[1]);
        bwd_mul_z(Dth, Du2, Pu2_lo, Pu2_hi, &ng.dth[0], &ng.dth[1], &ng.du2[0], &ng.du2[1]);
        // sin / cos bounds -> Theta endpoints -> nominal theta and Dth
        const double a64 = nom[th] + (double)Dth.lo, b64 = nom[th] + (double)Dth.hi;
        double Th_lo = 0.0, Th_hi = 0.0;
        {
            const SinCos& sc = nt.sc;
            const double dslo = sc_deriv(sc, true, sc.s_lo, a64, b64, false);
            const double dshi = sc_deriv(sc, true, sc.s_hi, a64, b64, true);
            const double dclo = sc_deriv(sc, false, sc.c_lo, a64, b64, false);
            const double dchi = sc_deriv(sc, false, sc.c_hi, a64, b64, true);
            if (sc.s_lo == 0) Th_lo += Sb_lo * dslo; else if (sc.s_lo == 1) Th_hi += Sb_lo * dslo;
            if (sc.s_hi == 0) Th_lo += Sb_hi * dshi; else if (sc.s_hi == 1) Th_hi += Sb_hi * dshi;
            if (sc.c_lo == 0) Th_lo += Cb_lo * dclo; else if (sc.c_lo == 1) Th_hi += Cb_lo * dclo;
            if (sc.c_hi == 0) Th_lo += Cb_hi * dchi; else if (sc.c_hi == 1) Th_hi += Cb_hi * dchi;
        }
        ng.th = Th_lo + Th_hi;
        ng.dth[0] += Th_lo;
        ng.dth[1] += Th_hi;
        // own position pairs
        PieceAdj lbar;
#pragma unroll
        for (int q = 0; q < 5; ++q) { lbar.lo[q] = 0.0; lbar.hi[q] = 0.0; }
        if (own) {
            double Gb_lo[5] = {0, 0, 0, 0, 0}, Gb_hi[5] = {0, 0, 0, 0, 0};
            double Pxx_lo = 0, Pxx_hi = 0, Pxz_lo = 0, Pxz_hi = 0, Pzz_lo = 0, Pzz_hi = 0;
            bwd_mul_z(nt.G[0], nt.Pxx, tlo[6], thi[6], &Gb_lo[0], &Gb_hi[0], &Pxx_lo, &Pxx_hi);
            bwd_mul_z(nt.G[1], nt.Pxz, tlo[7], thi[7], &Gb_lo[1], &Gb_hi[1], &Pxz_lo, &Pxz_hi);
            bwd_mul_z(nt.G[3], nt.Pzz, tlo[8], thi[8], &Gb_lo[3], &Gb_hi[3], &Pzz_lo, &Pzz_hi);
            bwd_mul_z(nt.G[1], nt.Pxx, tlo[9], thi[9], &Gb_lo[1], &Gb_hi[1], &Pxx_lo, &Pxx_hi);
            bwd_mul_z(nt.G[2], nt.Pxz, tlo[10], thi[10], &Gb_lo[2], &Gb_hi[2], &Pxz_lo, &Pxz_hi);
            bwd_mul_z(nt.G[4], nt.Pzz, tlo[11], thi[11], &Gb_lo[4], &Gb_hi[4], &Pzz_lo, &Pzz_hi);
            bwd_sq_z(Dx, Pxx_hi, &ng.dx[0], &ng.dx[1]);
            bwd_mul_z(Dx, Dz, Pxz_lo, Pxz_hi, &ng.dx[0], &ng.dx[1], &ng.dz[0], &ng.dz[1]);
            bwd_sq_z(Dz, Pzz_hi, &ng.dz[0], &ng.dz[1]);
            // G = R - L: [R.lo - L.hi, R.hi - L.lo]
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                rbar.lo[q] = Gb_lo[q]; rbar.hi[q] = Gb_hi[q];
                lbar.hi[q] = -Gb_lo[q]; lbar.lo[q] = -Gb_hi[q];
            }
        }
        if (i > 0) s_lbar[lt * U + i - 1] = lbar;
        s_gn[lt * U + i] = ng;
    }
    __syncthreads();

    // ---- 3. spring i tangent passes
    if (active && spring_ok) {
        const RowAdj gi0 = s_g[lt * U + i], gj0 = s_g[lt * U + i + 1];
        const bool ui = bad || s_unb[lt * U + i], uj = bad || s_unb[lt * U + i + 1];
        const double xli = ui ? 0.0 : gi0.xlo, xhi_ = ui ? 0.0 : gi0.xhi, zli = ui ? 0.0 : gi0.zlo, zhi_ = ui ? 0.0 : gi0.zhi;
        const double xlj = uj ? 0.0 : gj0.xlo, xhj = uj ? 0.0 : gj0.xhi, zlj = uj ? 0.0 : gj0.zlo, zhj = uj ? 0.0 : gj0.zhi;
        const PieceAdj lb = s_lbar[lt * U + i];
        AccTangent acc;
        // slot adjoints: row i takes C + B, row i+1 takes -(C + A)
        acc.alo[S_CX] = xli - xhj; acc.ahi[S_CX] = xhi_ - xlj;
        acc.alo[S_CZ] = zli - zhj; acc.ahi[S_CZ] = zhi_ - zlj;
        acc.alo[S_BX] = xli;       acc.ahi[S_BX] = xhi_;
        acc.alo[S_BZ] = zli;       acc.ahi[S_BZ] = zhi_;
        acc.alo[S_AX] = -xhj;      acc.ahi[S_AX] = -xlj;
        acc.alo[S_AZ] = -zhj;      acc.ahi[S_AZ] = -zlj;
        SpringGrad sgr;
        for (int dir = 0; dir < 10; ++dir) {
            // tangents of the spring inputs for this direction
            const float tdx = dir == 0, tdz = dir == 1;
            const float txil = dir == 2, txih = dir == 3, tzil = dir == 4, tzih = dir == 5;
            const float txjl = dir == 6, txjh = dir == 7, tzjl = dir == 8, tzjh = dir == 9;
            const IV<DF> dxA = iv(dfm(st.dxA.lo, tdx - txih), dfm(st.dxA.hi, tdx - txil));
            const IV<DF> dxB = iv(dfm(st.dxB.lo, tdx + txjl - txih), dfm(st.dxB.hi, tdx + txjh - txil));
            const IV<DF> dz0 = iv(dfm(st.dz0.lo, tdz), dfm(st.dz0.hi, tdz));
            const IV<DF> dz1 = iv(dfm(st.dz1.lo, tdz - tzih), dfm(st.dz1.hi, tdz - tzil));
            const IV<DF> dz2 = iv(dfm(st.dz2.lo, tdz + tzjl - tzih), dfm(st.dz2.hi, tdz + tzjh - tzil));
            const IV<DF> Dxi = iv(dfm(st.Dxi.lo, txil), dfm(st.Dxi.hi, txih));
            const IV<DF> Dzi = iv(dfm(st.Dzi.lo, tzil), dfm(st.Dzi.hi, tzih));
            const IV<DF> Dxj = iv(dfm(st.Dxj.lo, txjl), dfm(st.Dxj.hi, txjh));
            const IV<DF> Dzj = iv(dfm(st.Dzj.lo, tzjl), dfm(st.Dzj.hi, tzjh));
            acc.g = 0.0;
            SpringPieces<DF> pc;
            spring_core<DF, AccTangent>(dxA, dxB, dz0, dz1, dz2, Dxi, Dzi, Dxj, Dzj, 1.0, 1.0, 1.0, 1.0, K3, K15, K1,
                                        K05, acc, pc);
            double g = acc.g;
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                g += rbar.lo[q] * (double)pc.R[q].lo.d + rbar.hi[q] * (double)pc.R[q].hi.d;
                g += lb.lo[q] * (double)pc.L[q].lo.d + lb.hi[q] * (double)pc.L[q].hi.d;
            }
            sgr.d[dir] = g;
        }
        s_gs[lt * U + i] = sgr;
    } else if (active && i < U - 1) {
        SpringGrad z = {};
        s_gs[lt * U + i] = z;
    }
    __syncthreads();

    // ---- 4. per-coordinate sums (fixed order) and the box chain rule
    for (int idx = tid; idx < nloc * n; idx += BWD_BLOCK) {
        const int t = idx / n, c = idx - t * n;
        const bool tbad = s_flag[t] & LEB_FLAG_BAD_INPUT;
        double gnom = 0.0, glo = 0.0, ghi = 0.0;
        if (!tbad) {
            if (c < nx) {
                const int m = c / 6, rc = c - 6 * m;
                if (rc == 0 || rc == 1) {
                    const NodeGrad& ng = s_gn[t * U + m];
                    glo = rc == 0 ? ng.dx[0] : ng.dz[0];
                    ghi = rc == 0 ? ng.dx[1] : ng.dz[1];
                    if (m < U - 1) {        // spring m: node m is its first node
                        const SpringGrad& sg = s_gs[t * U + m];
                        gnom -= sg.d[rc];
                        glo += sg.d[rc == 0 ? 2 : 4];
                        ghi += sg.d[rc == 0 ? 3 : 5];
                    }
                    if (m > 0) {            // spring m-1: node m is its second node
                        const SpringGrad& sg = s_gs[t * U + m - 1];
                        gnom += sg.d[rc];
                        glo += sg.d[rc == 0 ? 6 : 8];
                        ghi += sg.d[rc == 0 ? 7 : 9];
                    }
                } else if (rc == 2) {
                    const NodeGrad& ng = s_gn[t * U + m];
                    gnom = ng.th; glo = ng.dth[0]; ghi = ng.dth[1];
                }
            } else {
                const int m = (c - nx) / 2, a = (c - nx) & 1;
                const NodeGrad& ng = s_gn[t * U + m];
                gnom = ng.s;
                glo = a == 0 ? ng.du1[0] : ng.du2[0];
                ghi = a == 0 ? ng.du1[1] : ng.du2[1];
            }
        }
        const int64_t o = u0 * n + idx;
        const double sg = A.sigma[o];
        const double mu = A.mu ? A.mu[o] : 0.0;
        // Delta_lo = min(mu - sigma, 0), Delta_hi = max(mu + sigma, 0); first candidate on a tie
        const double alo = (mu - sg <= 0.0) ? glo : 0.0;
        const double ahi = (mu + sg >= 0.0) ? ghi : 0.0;
        A.gsigma[o] = ahi - alo;
        if (A.gmu) A.gmu[o] = alo + ahi;
        if (c < nx) A.gz[(u0 + t) * nx + c] = gnom;
        else A.gv[(u0 + t) * nu + (c - nx)] = gnom;
    }
}

size_t bwd_smem_bytes(int U) {
    const int T = BWD_BLOCK / U, n = 8 * U;
    const size_t region = (size_t)T * U * (sizeof(BSpring) > sizeof(SpringGrad) ? sizeof(BSpring) : sizeof(SpringGrad));
    return (size_t)T * n * (sizeof(double) + sizeof(IV<float>)) + (size_t)T * U * sizeof(RowAdj) + region +
           (size_t)T * U * (sizeof(PieceAdj) + sizeof(NodeGrad) + sizeof(uint32_t)) + (size_t)T * sizeof(uint32_t) + 16;
}

int launch_pbh_bwd(const leb_dynamics* dyn, int64_t units, const double* z, const double* v, const double* mu,
                   const double* sigma, const double* g_lo, const double* g_hi, double* gz, double* gv,
                   double* gmu, double* gsigma, hipStream_t stream) {
    if (dyn->n_units > BWD_BLOCK) return LEB_ENOTSUP;
    BwdArgs a;
    a.z = z; a.v = v; a.mu = mu; a.sigma = sigma; a.g_lo = g_lo; a.g_hi = g_hi;
    a.gz = gz; a.gv = gv; a.gmu = gmu; a.gsigma = gsigma;
    a.units = units;
    a.U = dyn->n_units;
    a.T = BWD_BLOCK / a.U;
    a.c = dyn->dt / dyn->m;
    a.kL = dyn->k_spring * dyn->rest_len;
    a.L0 = dyn->rest_len;
    const int64_t blocks = (units + a.T - 1) / a.T;
    if (blocks > 0x7fffffff) return LEB_EINVAL;
    const size_t smem = bwd_smem_bytes(a.U);
    if (smem > 65536) return LEB_ENOTSUP;
    hipLaunchKernelGGL(pbh_chain_bwd, dim3((unsigned)blocks), dim3(BWD_BLOCK), smem, stream, a);
    return hipGetLastError() == hipSuccess ? LEB_OK : LEB_EDEVICE;
}

}  // namespace leb

using namespace leb;

extern "C" int leb_backward(const leb_dynamics* dyn, int32_t batch, int32_t N, const double* z, const double* v,
                            const double* mu, const double* sigma, const double* g_lo, const double* g_hi,
                            double* gz, double* gv, double* gmu, double* gsigma, void* stream) {
    int rc = check_chain_dynamics(dyn);
    if (rc != LEB_OK) return rc;
    if (dyn->kind != LEB_DYN_PQUAD_CHAIN) return LEB_ENOTSUP;
    if (batch < 0 || N < 0) return LEB_EINVAL;
    if (gmu && !mu) return LEB_EINVAL;
    const int64_t units = (int64_t)batch * N;
    if (units == 0) return LEB_OK;
    if (!z || !v || !sigma || !g_lo || !g_hi || !gz || !gv || !gsigma) return LEB_EINVAL;
    const void* ptrs[] = {z, v, mu, sigma, g_lo, g_hi, gz, gv, gmu, gsigma};
    for (const void* p : ptrs)
        if (p && !aligned8(p)) return LEB_EINVAL;
    return launch_pbh_bwd(dyn, units, z, v, mu, sigma, g_lo, g_hi, gz, gv, gmu, gsigma, (hipStream_t)stream);
}
