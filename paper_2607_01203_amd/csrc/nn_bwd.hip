// nn_bwd.hip -- adjoint of the ReLU-MLP remainder bound (sections IV.B and IV.D).
//
// The bound of nn.hip (CROWN with a full pass for every hidden layer's
// pre-activation bounds, Theorem 2 with J = J_g(a~)) is piecewise smooth in
// the nominal a~, the radii sigma and the offset mu; the paper differentiates
// it to shape the nominal trajectory.  This file computes, for
//     L = sum_rows g_hi r_hi + g_lo r_lo,
// dL/da~, dL/dsigma and dL/dmu of the exact-arithmetic bound (rounding
// allowances of the forward kernels are not part of it), by reverse mode.
//
// Forward quantities.  Box c = a~ + (dlo + dhi)/2, rho = (dhi - dlo)/2 with
// dlo = min(mu - sigma, 0), dhi = max(mu + sigma, 0).  Layer-1 bounds
// W_1 c + b_1 -/+ |W_1| rho.  The pass of target layer k (2 <= k <= L) runs
//     Lambda^(k-1) = rows of W_k,  for j = k-1 .. 1:
//       sel = (Lambda >= 0) for the upper pass, (Lambda < 0) for the lower one
//       Omega_j = Lambda^(j) (.) S_j,  S_j = sel ? s_j : a_j
//       beta += sum sel Lambda^(j) t_j + Omega_j b_j,  Lambda^(j-1) = Omega_j W_j
// with the relaxation s = u/(u-l), t = -s l, a = [u >= -l] of each unstable
// neuron (identity / zero for stable ones), and concretises
// Lambda^(0) c +/- |Lambda^(0)| rho + beta (k < L: bounds of layer k; k = L:
// Theorem 2 with Lambda^(0) - J in place of Lambda^(0)).
//
// Reverse.  With the row seeds y (g_hi / g_lo for k = L, the adjoints of the
// bounds u_k / l_k otherwise), the adjoint of one pass is
//     Lambda-bar^(0) = y (c +/- sign(D) rho),  c-bar += D^T y,  rho-bar +/-= |D|^T y
//     for j = 1 .. k-1:
//       Omega-bar_j = Lambda-bar^(j-1) W_j^T + y b_j^T
//       s-bar_j += sum_rows sel Omega-bar_j Lambda^(j),  t-bar_j += sum_rows sel y Lambda^(j)
//       Lambda-bar^(j) = Omega-bar_j (.) S_j + sel y t_j      (j < k-1)
// (D = Lambda^(0) - J for k = L, Lambda^(0) otherwise), and the relaxation
// adjoint of an unstable neuron is
//     u-bar = (-l s-bar + l^2 t-bar) / (u-l)^2,  l-bar = (u s-bar - u^2 t-bar) / (u-l)^2.
// Passes run from k = L down to 2: the bounds of layer j receive adjoints
// only from passes with k > j, so each layer's adjoint is complete when its
// own pass is reversed.  J a~ - g(a~) has derivative 0 (J is locally constant).
//
// GPU design.  One workgroup of 256 lanes per (box, pass direction); lane q
// owns neuron column q of every level, applies the relaxation selection to
// it and keeps the per-neuron sums s-bar, t-bar, c-bar, rho-bar of its column
// across row blocks; later passes add to them in launch order, so the result
// is deterministic.  The operand of each row-block product is staged in LDS
// as [neuron][row]; the weights come from L2 (W_j forward, W_j^T in reverse,
// both row-major, coalesced).  Two forms:
//  * MFMA (at most three hidden layers, the usual case): 16-row blocks on
//    FP64 MFMA; every pass has a forward launch that stores its levels and the
//    reverse launch reads them back; the k range of each product runs over
//    the neurons that are not stably inactive (see the MFMA section below).
//  * VALU (deeper networks): 8-row blocks, Lambda^(j) of the lane's column
//    kept in registers for the reverse sweep; hidden-layer passes store their
//    levels, the output pass recomputes its chain; narrow outputs (the input
//    layer) split the sum over lane slices added in a fixed order.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "leb.h"
#include "leb_internal.hpp"
#include "nn_net.hpp"

namespace leb {

constexpr int NB_R = 8;          // target rows per block
constexpr int NB_T = 256;        // lanes per workgroup
constexpr int NB_CHUNK = 4096;   // most boxes per chunk of the workspace
constexpr int NB_CHUNK_MIN = 32; // fewest (deep, wide networks)
constexpr size_t NB_LV_BUDGET = (size_t)8 << 30;   // workspace bytes that set the chunk size

struct NbArgs {
    int L;
    int w[NN_MAXL + 1];
    const double* W[NN_MAXL];
    const double* WT[NN_MAXL];
    const double* b[NN_MAXL];
    int nx, nu;
    int k;                         // target layer of a pass; layer of a relaxation adjoint
    int64_t u0;                    // first unit of the chunk
    const double* z; const double* v; const double* mu; const double* sigma;
    const double* g_lo; const double* g_hi;
    double* gz; double* gv; double* gmu; double* gsigma;
    // chunk workspace (box-major)
    double* cr;                    // [box][2][NN_MAXW]          c, rho
    double* zn;                    // [box][NN_MAXL][NN_MAXW]    nominal pre-activations of hidden layer j (index j-1)
    double* bd;                    // [box][NN_MAXL][2][NN_MAXW] lo, hi of hidden layer j
    double* st;                    // [box][2][NN_MAXL][2][NN_MAXW] s-bar, t-bar per pass direction
    double* ub;                    // [box][NN_MAXL][2][NN_MAXW] u-bar, l-bar of hidden layer j
    double* cg;                    // [box][2][2][NN_MAXW]       c-bar, rho-bar per pass direction
    uint32_t* ok;                  // [box] 1: valid input
    double* lv;                    // [box][2][lv_bm] levels Lambda^(j) of the hidden-layer passes
    size_t lv_bm;                  // doubles per (box, direction)
    int lv_off[NN_MAXL][NN_MAXL];  // offset of level j of pass k: [row][column], w[k] x w[j]
};

__device__ __forceinline__ size_t ix_cr(int box, int which) { return ((size_t)box * 2 + which) * NN_MAXW; }
__device__ __forceinline__ size_t ix_zn(int box, int j) { return ((size_t)box * NN_MAXL + j - 1) * NN_MAXW; }
__device__ __forceinline__ size_t ix_bd(int box, int j, int hi) {
    return (((size_t)box * NN_MAXL + j - 1) * 2 + hi) * NN_MAXW;
}
__device__ __forceinline__ size_t ix_st(int box, int mode, int j, int which) {
    return ((((size_t)box * 2 + mode) * NN_MAXL + j - 1) * 2 + which) * NN_MAXW;
}
__device__ __forceinline__ size_t ix_ub(int box, int j, int which) {
    return (((size_t)box * NN_MAXL + j - 1) * 2 + which) * NN_MAXW;
}
__device__ __forceinline__ size_t ix_cg(int box, int mode, int which) {
    return (((size_t)box * 2 + mode) * 2 + which) * NN_MAXW;
}

// ReLU relaxation of a neuron with pre-activation bounds [lo, hi]: upper
// line s z + t, lower line a z
__device__ __forceinline__ void nb_relax(double lo, double hi, double& s, double& t, double& a) {
    if (lo >= 0.0) { s = 1.0; t = 0.0; a = 1.0; }
    else if (hi > 0.0) { s = hi / (hi - lo); t = -s * lo; a = hi >= -lo ? 1.0 : 0.0; }
    else { s = 0.0; t = 0.0; a = 0.0; }
}

// out[r][i] = sum_{p < len} X[p][r] M[p nc + i] for i < nc, X in LDS as [p][NB_R];
// lane q < nc receives column q.  Narrow outputs split p over 256 / nc lane
// slices, added in slice order.  Every lane must call it (it may hold a barrier).
__device__ __forceinline__ void nb_rowmat(const double* __restrict__ M, int nc, int len, const double* sX,
                                          double* sP, int q, double acc[NB_R]) {
    const int S = nc >= NB_T ? 1 : NB_T / nc;
    const int i = q % nc, sl = q / nc;
#pragma unroll
    for (int r = 0; r < NB_R; ++r) acc[r] = 0.0;
    if (sl < S) {
        const int p0 = (int)(((int64_t)sl * len) / S), p1 = (int)(((int64_t)(sl + 1) * len) / S);
        const double* Mi = M + i;
#pragma unroll 4
        for (int p = p0; p < p1; ++p) {
            const double w = Mi[(size_t)p * nc];
            const double* x = sX + p * NB_R;
#pragma unroll
            for (int r = 0; r < NB_R; ++r) acc[r] = __builtin_fma(x[r], w, acc[r]);
        }
    }
    if (S > 1) {
        if (sl >= 1 && sl < S) {
#pragma unroll
            for (int r = 0; r < NB_R; ++r) sP[((sl - 1) * nc + i) * NB_R + r] = acc[r];
        }
        lds_barrier();
        if (q < nc) {
            for (int s2 = 1; s2 < S; ++s2) {
#pragma unroll
                for (int r = 0; r < NB_R; ++r) acc[r] += sP[((s2 - 1) * nc + q) * NB_R + r];
            }
        }
    }
}

// per box: validity, the box (c, rho), nominal pre-activations, layer-1
// bounds, and zeroed adjoint sums
__global__ void __launch_bounds__(NB_T) nb_box_kernel(NbArgs A) {
    __shared__ double s_a[NN_MAXW], s_c[NN_MAXW], s_r[NN_MAXW];
    __shared__ uint32_t s_bad;
    const int box = blockIdx.x, q = threadIdx.x;
    const int64_t unit = A.u0 + box;
    const int n0 = A.w[0], L = A.L;
    if (q == 0) s_bad = 0;
    __syncthreads();
    if (q < n0) {
        const double x = q < A.nx ? A.z[unit * A.nx + q] : A.v[unit * A.nu + (q - A.nx)];
        const double sg = A.sigma[unit * n0 + q];
        const double mu = A.mu ? A.mu[unit * n0 + q] : 0.0;
        if (!isfinite(x) || !isfinite(sg) || !isfinite(mu) || !(sg >= 0.0)) atomicOr(&s_bad, 1u);
        const double dlo = fmin(mu - sg, 0.0), dhi = fmax(mu + sg, 0.0);
        s_a[q] = x;
        s_c[q] = x + 0.5 * (dlo + dhi);
        s_r[q] = 0.5 * (dhi - dlo);
        A.cr[ix_cr(box, 0) + q] = s_c[q];
        A.cr[ix_cr(box, 1) + q] = s_r[q];
    }
    // zero the adjoint sums of this box
    for (int j = 1; j < L; ++j)
        for (int md = 0; md < 2; ++md)
            for (int wh = 0; wh < 2; ++wh) A.st[ix_st(box, md, j, wh) + q] = 0.0;
    for (int md = 0; md < 2; ++md)
        for (int wh = 0; wh < 2; ++wh) A.cg[ix_cg(box, md, wh) + q] = 0.0;
    __syncthreads();
    if (q == 0) A.ok[box] = s_bad ? 0u : 1u;
    const int n1 = A.w[1];
    if (q < n1) {
        const double* Wr = A.W[0] + (size_t)q * n0;
        double lin = A.b[0][q], mag = 0.0;
        for (int p = 0; p < n0; ++p) {
            lin = __builtin_fma(Wr[p], s_c[p], lin);
            mag = __builtin_fma(fabs(Wr[p]), s_r[p], mag);
        }
        A.bd[ix_bd(box, 1, 0) + q] = lin - mag;
        A.bd[ix_bd(box, 1, 1) + q] = lin + mag;
    }
    // nominal pre-activations of the hidden layers (the masks of J)
    for (int l = 0; l < L - 1; ++l) {
        const int in = A.w[l], out = A.w[l + 1];
        double zz = 0.0;
        if (q < out) {
            zz = A.b[l][q];
            const double* WT = A.WT[l];
            for (int p = 0; p < in; ++p) zz = __builtin_fma(WT[(size_t)p * out + q], s_a[p], zz);
        }
        __syncthreads();
        if (q < out) {
            A.zn[ix_zn(box, l + 1) + q] = zz;
            s_a[q] = zz > 0.0 ? zz : 0.0;
        }
        __syncthreads();
    }
}

// One CROWN pass of target layer A.k for one box (blockIdx.x) and direction
// (blockIdx.y: 0 upper, 1 lower).  REV = false: the bounds of layer k
// (hi for the upper pass, lo for the lower one).  REV = true: the adjoint of
// the pass, added to the per-neuron sums.  LV >= k - 1: levels kept per lane.
template <bool REV, int LV>
__global__ void __launch_bounds__(NB_T) nb_pass_kernel(NbArgs A) {
    __shared__ __attribute__((aligned(16))) double sX[NN_MAXW * NB_R];
    __shared__ __attribute__((aligned(16))) double sP[NN_MAXW * NB_R];
    __shared__ double sRed[NB_T / 64][NB_R];
    const int box = blockIdx.x, mode = blockIdx.y, q = threadIdx.x;
    if (!A.ok[box]) return;
    const bool upper = mode == 0;
    const double sgn = upper ? 1.0 : -1.0;
    const int k = A.k, L = A.L, n0 = A.w[0];
    const int rows = A.w[k], nk1 = A.w[k - 1];
    const double* Wk = A.W[k - 1];
    const double cq = q < n0 ? A.cr[ix_cr(box, 0) + q] : 0.0;
    const double rq = q < n0 ? A.cr[ix_cr(box, 1) + q] : 0.0;
    double sacc[LV], tacc[LV];
#pragma unroll
    for (int j = 0; j < LV; ++j) { sacc[j] = 0.0; tacc[j] = 0.0; }
    double cacc = 0.0, racc = 0.0;

    for (int r0 = 0; r0 < rows; r0 += NB_R) {
        const int nr = min(NB_R, rows - r0);
        double lam[LV][NB_R];                   // Lambda^(j) of column q, j = 0 .. k-2
        double bpart[NB_R];
#pragma unroll
        for (int r = 0; r < NB_R; ++r) bpart[r] = 0.0;
        double* lvb = A.lv + ((size_t)box * 2 + mode) * A.lv_bm;
        if (REV && k < L) {
            // the levels stored by this layer's forward pass
#pragma unroll
            for (int j = 0; j < LV; ++j) {
                if (j > k - 2 || q >= A.w[j]) continue;
                const double* src = lvb + A.lv_off[k][j] + (size_t)r0 * A.w[j] + q;
#pragma unroll
                for (int r = 0; r < NB_R; ++r) lam[j][r] = r < nr ? src[(size_t)r * A.w[j]] : 0.0;
            }
        }
        // ---- forward chain of the block, j = k-1 .. 1 (every pass but the
        // reverse of a hidden layer's)
#pragma unroll
        for (int j = LV; j >= 1; --j) {
            if (j > k - 1 || (REV && k < L)) continue;
            const int nj = A.w[j];
            if (q < nj) {
                double s, t, a;
                nb_relax(A.bd[ix_bd(box, j, 0) + q], A.bd[ix_bd(box, j, 1) + q], s, t, a);
                const double bj = A.b[j - 1][q];
#pragma unroll
                for (int r = 0; r < NB_R; ++r) {
                    double lm;
                    if (j == k - 1) lm = r < nr ? Wk[(size_t)(r0 + r) * nk1 + q] : 0.0;
                    else lm = lam[j < LV ? j : 0][r];     // j < LV whenever j < k - 1
                    const bool sel = upper ? lm >= 0.0 : lm < 0.0;
                    const double om = lm * (sel ? s : a);
                    if (!REV) bpart[r] += (sel ? lm * t : 0.0) + om * bj;
                    sX[q * NB_R + r] = om;
                }
            }
            lds_barrier();
            double acc[NB_R];
            nb_rowmat(A.W[j - 1], A.w[j - 1], nj, sX, sP, q, acc);
            if (q < A.w[j - 1]) {
#pragma unroll
                for (int r = 0; r < NB_R; ++r) lam[j - 1][r] = acc[r];
                if (!REV) {
                    double* dst = lvb + A.lv_off[k][j - 1] + (size_t)r0 * A.w[j - 1] + q;
#pragma unroll
                    for (int r = 0; r < NB_R; ++r)
                        if (r < nr) dst[(size_t)r * A.w[j - 1]] = acc[r];
                }
            }
            lds_barrier();
        }
        if (!REV) {
            // concretise: row value = b_k + beta parts + Lambda^(0) c +/- |Lambda^(0)| rho
            if (q < n0) {
#pragma unroll
                for (int r = 0; r < NB_R; ++r) bpart[r] += lam[0][r] * cq + sgn * fabs(lam[0][r]) * rq;
            }
            const int wv = q >> 6;
#pragma unroll
            for (int r = 0; r < NB_R; ++r) {
                double x = bpart[r];
#pragma unroll
                for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o);
                if ((q & 63) == 0) sRed[wv][r] = x;
            }
            lds_barrier();
            if (q < nr) {
                double x = A.b[k - 1][r0 + q];
                for (int w2 = 0; w2 < NB_T / 64; ++w2) x += sRed[w2][q];
                A.bd[ix_bd(box, k, upper ? 1 : 0) + r0 + q] = x;
            }
            lds_barrier();
            continue;
        }
        // ---- reverse sweep of the block
        double y[NB_R];
#pragma unroll
        for (int r = 0; r < NB_R; ++r) {
            double yy = 0.0;
            if (r < nr) {
                if (k == L) yy = (upper ? A.g_hi : A.g_lo)[(A.u0 + box) * rows + r0 + r];
                else yy = A.ub[ix_ub(box, k, upper ? 0 : 1) + r0 + r];
            }
            y[r] = yy;
        }
        double jv[NB_R];
#pragma unroll
        for (int r = 0; r < NB_R; ++r) jv[r] = 0.0;
        if (k == L) {
            // the rows of J = W_L D_{L-1} W_{L-1} ... D_1 W_1 (D = [z^ > 0]) for this block
#pragma unroll
            for (int r = 0; r < NB_R; ++r) jv[r] = (q < nk1 && r < nr) ? Wk[(size_t)(r0 + r) * nk1 + q] : 0.0;
            for (int j = L - 1; j >= 1; --j) {
                const int nj = A.w[j];
                if (q < nj) {
                    const double on = A.zn[ix_zn(box, j) + q] > 0.0 ? 1.0 : 0.0;
#pragma unroll
                    for (int r = 0; r < NB_R; ++r) sX[q * NB_R + r] = jv[r] * on;
                }
                lds_barrier();
                nb_rowmat(A.W[j - 1], A.w[j - 1], nj, sX, sP, q, jv);
                lds_barrier();
            }
        }
        // seeds of Lambda^(0) and the direct c / rho terms
        if (q < n0) {
#pragma unroll
            for (int r = 0; r < NB_R; ++r) {
                const double d = lam[0][r] - jv[r];
                const double sd = d > 0.0 ? 1.0 : (d < 0.0 ? -1.0 : 0.0);
                cacc += y[r] * d;
                racc += sgn * y[r] * fabs(d);
                sX[q * NB_R + r] = y[r] * (cq + sgn * sd * rq);
            }
        }
        lds_barrier();
#pragma unroll
        for (int j = 1; j <= LV; ++j) {
            if (j > k - 1) continue;
            const int nj = A.w[j];
            double ob[NB_R];
            nb_rowmat(A.WT[j - 1], nj, A.w[j - 1], sX, sP, q, ob);
            lds_barrier();                      // sX is rewritten below
            if (q < nj) {
                double s, t, a;
                nb_relax(A.bd[ix_bd(box, j, 0) + q], A.bd[ix_bd(box, j, 1) + q], s, t, a);
                const double bj = A.b[j - 1][q];
                double sa = 0.0, ta = 0.0;
#pragma unroll
                for (int r = 0; r < NB_R; ++r) {
                    double lm;
                    if (j == k - 1) lm = r < nr ? Wk[(size_t)(r0 + r) * nk1 + q] : 0.0;
                    else lm = lam[j < LV ? j : 0][r];     // j < LV whenever j < k - 1
                    const bool sel = upper ? lm >= 0.0 : lm < 0.0;
                    const double obr = ob[r] + y[r] * bj;
                    if (sel) {
                        sa += obr * lm;
                        ta += y[r] * lm;
                    }
                    if (j < k - 1) sX[q * NB_R + r] = obr * (sel ? s : a) + (sel ? y[r] * t : 0.0);
                }
                sacc[j - 1] += sa;
                tacc[j - 1] += ta;
            }
            lds_barrier();
        }
    }
    if (REV) {
#pragma unroll
        for (int j = 1; j <= LV; ++j) {
            if (j > k - 1) continue;
            if (q < A.w[j]) {
                A.st[ix_st(box, mode, j, 0) + q] += sacc[j - 1];
                A.st[ix_st(box, mode, j, 1) + q] += tacc[j - 1];
            }
        }
        if (q < n0) {
            A.cg[ix_cg(box, mode, 0) + q] += cacc;
            A.cg[ix_cg(box, mode, 1) + q] += racc;
        }
    }
}

// ---------------------------------------------------------------- MFMA form
//
// Networks with at most three hidden layers: the row-block products run on
// FP64 MFMA (v_mfma_f64_16x16x4f64) with 16-row blocks.  The operand (16 rows
// x len) and the product (16 rows x nc) sit in LDS as [neuron][row] with a
// row stride of 17 doubles, so the A-operand reads (lane l: row l % 16 of
// k-step 4 kk + l / 16) are consecutive and the owner lanes' column reads
// spread over the banks.  B operands (the weights) come from L2, one per lane
// and tile per k-step, the next k-step's loaded before this one's MFMAs.
// Every pass, the output pass included, has a forward launch that stores its
// levels; the reverse launches read them back, so no level lives in
// registers across a product.
typedef double nbd4 __attribute__((ext_vector_type(4)));
constexpr int NBM_R = 16;        // rows per block
constexpr int NBM_RS = 17;       // LDS row stride of operand and product

// sD[col][row] = sum_{p < len} sA[p][row] M[kl[p] ld + cl[col]], col < nc,
// 16 rows; kl = NULL: kl[p] = p, cl = NULL: cl[c] = c.  len a multiple of 4
// (possibly 0), nc of 16.  Every lane calls it; it ends with a barrier after
// which sD is complete (and sA no longer read).
__device__ __forceinline__ void nbm_mm(const double* __restrict__ M, int ld, int nc, int len, const int* kl,
                                       const int* cl, const double* sA, double* sD, int q) {
    const int w = q >> 6, l = q & 63, lr = l & 15, lq = l >> 4;
    const int nt = nc >> 4, nk = len >> 2;
    auto krow = [&](int p) { return (size_t)(kl ? kl[p] : p) * ld; };
    auto kcol = [&](int t) { return (size_t)(cl ? cl[16 * t + lr] : 16 * t + lr); };
    if (nt >= 4) {
        // column tiles t = w, w + 4, ... of this wave over the whole k range
        nbd4 acc[4];
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) acc[s2] = nbd4{0.0, 0.0, 0.0, 0.0};
        double bn[4];
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) {
            const int t = w + 4 * s2;
            bn[s2] = (t < nt && nk > 0) ? M[krow(lq) + kcol(t)] : 0.0;
        }
        for (int kk = 0; kk < nk; ++kk) {
            double b[4];
#pragma unroll
            for (int s2 = 0; s2 < 4; ++s2) b[s2] = bn[s2];
            if (kk + 1 < nk) {
#pragma unroll
                for (int s2 = 0; s2 < 4; ++s2) {
                    const int t = w + 4 * s2;
                    bn[s2] = t < nt ? M[krow(4 * kk + 4 + lq) + kcol(t)] : 0.0;
                }
            }
            const double av = sA[(4 * kk + lq) * NBM_RS + lr];
#pragma unroll
            for (int s2 = 0; s2 < 4; ++s2)
                if (w + 4 * s2 < nt) acc[s2] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b[s2], acc[s2], 0, 0, 0);
        }
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) {
            const int t = w + 4 * s2;
            if (t < nt) {
#pragma unroll
                for (int i = 0; i < 4; ++i) sD[(16 * t + lr) * NBM_RS + 4 * i + lq] = acc[s2][i];
            }
        }
        lds_barrier();
        return;
    }
    // narrow output (1 to 3 tiles): the k range in four quarters, one per
    // wave, partials added in wave order
    // two k-steps per trip into two accumulators (their loads issued
    // together, two independent MFMA chains), added at the end
    nbd4 acc[3], acc2[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) { acc[t] = nbd4{0.0, 0.0, 0.0, 0.0}; acc2[t] = nbd4{0.0, 0.0, 0.0, 0.0}; }
    const int k0 = (w * nk) >> 2, k1 = ((w + 1) * nk) >> 2;
    int kk = k0;
    for (; kk + 1 < k1; kk += 2) {
        const double av0 = sA[(4 * kk + lq) * NBM_RS + lr];
        const double av1 = sA[(4 * kk + 4 + lq) * NBM_RS + lr];
        double b0[3], b1[3];
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            b0[t] = t < nt ? M[krow(4 * kk + lq) + kcol(t)] : 0.0;
            b1[t] = t < nt ? M[krow(4 * kk + 4 + lq) + kcol(t)] : 0.0;
        }
#pragma unroll
        for (int t = 0; t < 3; ++t)
            if (t < nt) {
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av0, b0[t], acc[t], 0, 0, 0);
                acc2[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av1, b1[t], acc2[t], 0, 0, 0);
            }
    }
    if (kk < k1) {
        const double av = sA[(4 * kk + lq) * NBM_RS + lr];
#pragma unroll
        for (int t = 0; t < 3; ++t)
            if (t < nt) {
                const double bv = M[krow(4 * kk + lq) + kcol(t)];
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[t], 0, 0, 0);
            }
    }
#pragma unroll
    for (int t = 0; t < 3; ++t) acc[t] += acc2[t];
    double* part = sD + 1024;            // [wave][tile][i][lane], past the product's 3 tiles
#pragma unroll
    for (int t = 0; t < 3; ++t)
        if (t < nt) {
#pragma unroll
            for (int i = 0; i < 4; ++i) part[((w * 3 + t) * 4 + i) * 64 + l] = acc[t][i];
        }
    lds_barrier();
    for (int e = q; e < nc * NBM_R; e += NB_T) {
        const int col = e >> 4, row = e & 15;
        const int t = col >> 4, li = (row & 3) * 16 + (col & 15), i = row >> 2;
        double x = 0.0;
        for (int w2 = 0; w2 < 4; ++w2) x += part[((w2 * 3 + t) * 4 + i) * 64 + li];
        sD[col * NBM_RS + row] = x;
    }
    lds_barrier();
}

// zero the operand rows tot .. len-1 (the padding of a neuron list)
__device__ __forceinline__ void nbm_pad(double* sA, int tot, int len, int q) {
    for (int e = q; e < (len - tot) * NBM_R; e += NB_T) sA[(tot + e / NBM_R) * NBM_RS + e % NBM_R] = 0.0;
}

// One CROWN pass of target layer A.k (2 <= k <= L) for one box and direction,
// MFMA form.  FWD: the levels of every 16-row block into lv, and for a
// hidden layer its bounds.  REV: the adjoint of the pass from the stored levels.
template <bool REV>
__global__ void __launch_bounds__(NB_T) __attribute__((amdgpu_waves_per_eu(2))) nbm_pass_kernel(NbArgs A) {
    __shared__ __attribute__((aligned(16))) double sA[NN_MAXW * NBM_RS];
    __shared__ __attribute__((aligned(16))) double sD[NN_MAXW * NBM_RS];
    // per hidden layer j (index j-1): the neurons that are not stably inactive
    // (an inactive neuron's column of Omega, and of Lambda-bar, is exactly 0,
    // and its own columns of Lambda and Omega-bar are never used), padded with
    // entry 0 to a multiple of 4 (k range) and of 16 (output columns); pos: a
    // neuron's place in the list.  Products over a hidden layer's neurons, in
    // k or in output columns, run over its list; their outputs sit at list
    // positions.
    __shared__ int sList[3][NN_MAXW], sPos[3][NN_MAXW], sLen[3], sLen16[3], sTot[3];
    __shared__ int sCnt[NB_T / 64];
    const int box = blockIdx.x, mode = blockIdx.y, q = threadIdx.x;
    if (!A.ok[box]) return;
    for (int j = 1; j <= A.k - 1; ++j) {
        const int nj = A.w[j];
        const bool keep = q < nj && (A.bd[ix_bd(box, j, 0) + q] >= 0.0 || A.bd[ix_bd(box, j, 1) + q] > 0.0);
        const uint64_t bal = __ballot(keep);
        if ((q & 63) == 0) sCnt[q >> 6] = __popcll(bal);
        lds_barrier();
        int off = 0, tot = 0;
        for (int w2 = 0; w2 < NB_T / 64; ++w2) {
            if (w2 < (q >> 6)) off += sCnt[w2];
            tot += sCnt[w2];
        }
        const int pos = off + __popcll(bal & ((1ull << (q & 63)) - 1ull));
        if (keep) sList[j - 1][pos] = q;
        if (q < nj) sPos[j - 1][q] = keep ? pos : -1;
        const int padded = (tot + 3) & ~3, padded16 = (tot + 15) & ~15;
        if (q >= tot && q < padded16) sList[j - 1][q] = 0;
        if (q == 0) { sLen[j - 1] = padded; sLen16[j - 1] = padded16; sTot[j - 1] = tot; }
        lds_barrier();
    }
    const bool upper = mode == 0;
    const double sgn = upper ? 1.0 : -1.0;
    const int k = A.k, L = A.L, n0 = A.w[0];
    const int rows = A.w[k], nk1 = A.w[k - 1];
    const double* Wk = A.W[k - 1];
    const double cq = q < n0 ? A.cr[ix_cr(box, 0) + q] : 0.0;
    const double rq = q < n0 ? A.cr[ix_cr(box, 1) + q] : 0.0;
    double* lvb = A.lv + ((size_t)box * 2 + mode) * A.lv_bm;
    double sacc[3] = {0.0, 0.0, 0.0}, tacc[3] = {0.0, 0.0, 0.0};
    double cacc = 0.0, racc = 0.0;
    // forward launches: the relaxation and bias of the lane's neuron in each
    // layer j < k (loaded once), and the rows of W_k of the next block (loaded
    // while the current block computes)
    double fs[3] = {0.0, 0.0, 0.0}, ft[3] = {0.0, 0.0, 0.0}, fa[3] = {0.0, 0.0, 0.0}, fb[3] = {0.0, 0.0, 0.0};
    double wk[NBM_R];
    // reverse launches: Lambda^(0) rows of the block (lanes q < n0), loaded a block ahead
    double l0n[NBM_R];
    if (REV) {
#pragma unroll
        for (int r = 0; r < NBM_R; ++r)
            l0n[r] = (q < n0 && r < rows) ? lvb[A.lv_off[k][0] + (size_t)r * n0 + q] : 0.0;
    }
    if (!REV) {
#pragma unroll
        for (int j = 1; j <= 3; ++j) {
            if (j <= k - 1 && q < A.w[j]) {
                nb_relax(A.bd[ix_bd(box, j, 0) + q], A.bd[ix_bd(box, j, 1) + q], fs[j - 1], ft[j - 1], fa[j - 1]);
                fb[j - 1] = A.b[j - 1][q];
            }
        }
#pragma unroll
        for (int r = 0; r < NBM_R; ++r) wk[r] = (q < nk1 && r < rows) ? Wk[(size_t)r * nk1 + q] : 0.0;
    }

    for (int r0 = 0; r0 < rows; r0 += NBM_R) {
        const int nr = min(NBM_R, rows - r0);
        if (!REV) {
            double bpart[NBM_R];
#pragma unroll
            for (int r = 0; r < NBM_R; ++r) bpart[r] = 0.0;
            for (int j = k - 1; j >= 1; --j) {
                const int nj = A.w[j];
                const int pq = q < nj ? sPos[j - 1][q] : -1;
                if (pq >= 0) {
                    const double s = j == 1 ? fs[0] : (j == 2 ? fs[1] : fs[2]);
                    const double t = j == 1 ? ft[0] : (j == 2 ? ft[1] : ft[2]);
                    const double a = j == 1 ? fa[0] : (j == 2 ? fa[1] : fa[2]);
                    const double bj = j == 1 ? fb[0] : (j == 2 ? fb[1] : fb[2]);
#pragma unroll
                    for (int r = 0; r < NBM_R; ++r) {
                        const double lm = j == k - 1 ? wk[r] : sD[pq * NBM_RS + r];
                        const bool sel = upper ? lm >= 0.0 : lm < 0.0;
                        const double om = lm * (sel ? s : a);
                        bpart[r] += (sel ? lm * t : 0.0) + om * bj;
                        sA[pq * NBM_RS + r] = om;
                    }
                }
                if (j == k - 1) {
                    // the next block's rows of W_k
                    const int r1 = r0 + NBM_R;
#pragma unroll
                    for (int r = 0; r < NBM_R; ++r)
                        wk[r] = (q < nk1 && r1 + r < rows) ? Wk[(size_t)(r1 + r) * nk1 + q] : 0.0;
                }
                const int len = sLen[j - 1];
                nbm_pad(sA, sTot[j - 1], len, q);
                lds_barrier();
                const int nj1 = A.w[j - 1];
                if (j == 1) nbm_mm(A.W[0], nj1, nj1, len, sList[0], nullptr, sA, sD, q);
                else nbm_mm(A.W[j - 1], nj1, sLen16[j - 2], len, sList[j - 1], sList[j - 2], sA, sD, q);
                if (q < nj1) {
                    // Lambda^(j-1) column q (0 for a stably inactive neuron: never used)
                    const int pc = j == 1 ? q : sPos[j - 2][q];
                    double* dst = lvb + A.lv_off[k][j - 1] + (size_t)r0 * nj1 + q;
                    for (int r = 0; r < nr; ++r) dst[(size_t)r * nj1] = pc >= 0 ? sD[pc * NBM_RS + r] : 0.0;
                }
            }
            if (k < L) {
                // concretise the rows: b_k + beta parts + Lambda^(0) c +/- |Lambda^(0)| rho
                if (q < n0) {
#pragma unroll
                    for (int r = 0; r < NBM_R; ++r) {
                        const double l0 = sD[q * NBM_RS + r];
                        bpart[r] += l0 * cq + sgn * fabs(l0) * rq;
                    }
                }
                const int wv = q >> 6;
#pragma unroll
                for (int r = 0; r < NBM_R; ++r) {
                    double x = bpart[r];
#pragma unroll
                    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o);
                    if ((q & 63) == 0) sA[wv * NBM_R + r] = x;
                }
                lds_barrier();
                if (q < nr) {
                    double x = A.b[k - 1][r0 + q];
                    for (int w2 = 0; w2 < NB_T / 64; ++w2) x += sA[w2 * NBM_R + q];
                    A.bd[ix_bd(box, k, upper ? 1 : 0) + r0 + q] = x;
                }
            }
            lds_barrier();
            continue;
        }
        // ---- reverse sweep of the block from the stored levels
        double y[NBM_R];
#pragma unroll
        for (int r = 0; r < NBM_R; ++r) {
            double yy = 0.0;
            if (r < nr) {
                if (k == L) yy = (upper ? A.g_hi : A.g_lo)[(A.u0 + box) * rows + r0 + r];
                else yy = A.ub[ix_ub(box, k, upper ? 0 : 1) + r0 + r];
            }
            y[r] = yy;
        }
        double jv[NBM_R];
#pragma unroll
        for (int r = 0; r < NBM_R; ++r) jv[r] = 0.0;
        if (k == L) {
            // rows of J = W_L D_{L-1} W_{L-1} ... D_1 W_1 (D = [z^ > 0]) for this block
            for (int j = L - 1; j >= 1; --j) {
                const int nj = A.w[j];
                if (q < nj) {
                    const double on = A.zn[ix_zn(box, j) + q] > 0.0 ? 1.0 : 0.0;
#pragma unroll
                    for (int r = 0; r < NBM_R; ++r) {
                        double x;
                        if (j == L - 1) x = r < nr ? Wk[(size_t)(r0 + r) * nk1 + q] : 0.0;
                        else x = sD[q * NBM_RS + r];
                        sA[q * NBM_RS + r] = x * on;
                    }
                }
                lds_barrier();
                nbm_mm(A.W[j - 1], A.w[j - 1], A.w[j - 1], nj, nullptr, nullptr, sA, sD, q);
            }
            if (q < n0) {
#pragma unroll
                for (int r = 0; r < NBM_R; ++r) jv[r] = sD[q * NBM_RS + r];
            }
            lds_barrier();
        }
        if (q < n0) {
#pragma unroll
            for (int r = 0; r < NBM_R; ++r) {
                const double d = l0n[r] - jv[r];
                const double sd = d > 0.0 ? 1.0 : (d < 0.0 ? -1.0 : 0.0);
                cacc += y[r] * d;
                racc += sgn * y[r] * fabs(d);
                sA[q * NBM_RS + r] = y[r] * (cq + sgn * sd * rq);
            }
            // the next block's Lambda^(0) rows, in flight while this block runs
            const int r1 = r0 + NBM_R;
            const double* src = lvb + A.lv_off[k][0] + (size_t)r1 * n0 + q;
#pragma unroll
            for (int r = 0; r < NBM_R; ++r) l0n[r] = r1 + r < rows ? src[(size_t)r * n0] : 0.0;
        }
        lds_barrier();
        for (int j = 1; j <= k - 1; ++j) {
            const int nj = A.w[j];
            // this level's Lambda^(j) column, relaxation and bias, loaded before
            // the product so their latency overlaps it
            double lmv[NBM_R];
            double lo_j = 0.0, hi_j = 0.0, bj = 0.0;
            if (q < nj) {
                const double* src = j == k - 1 ? Wk + (size_t)r0 * nk1 + q
                                               : lvb + A.lv_off[k][j] + (size_t)r0 * nj + q;
                const size_t ld = j == k - 1 ? (size_t)nk1 : (size_t)nj;
#pragma unroll
                for (int r = 0; r < NBM_R; ++r) lmv[r] = r < nr ? src[(size_t)r * ld] : 0.0;
                lo_j = A.bd[ix_bd(box, j, 0) + q];
                hi_j = A.bd[ix_bd(box, j, 1) + q];
                bj = A.b[j - 1][q];
            }
            // k over layer j-1: the inputs (all) or the listed neurons of a hidden layer
            // output columns over layer j's list
            if (j == 1) nbm_mm(A.WT[0], nj, sLen16[0], n0, nullptr, sList[0], sA, sD, q);
            else nbm_mm(A.WT[j - 1], nj, sLen16[j - 1], sLen[j - 2], sList[j - 2], sList[j - 1], sA, sD, q);
            const int pq = q < nj ? sPos[j - 1][q] : -1;
            if (j < k - 1) nbm_pad(sA, sTot[j - 1], sLen[j - 1], q);
            if (pq >= 0) {
                double s, t, a;
                nb_relax(lo_j, hi_j, s, t, a);
                double sa = 0.0, ta = 0.0;
#pragma unroll
                for (int r = 0; r < NBM_R; ++r) {
                    const double lm = lmv[r];
                    const bool sel = upper ? lm >= 0.0 : lm < 0.0;
                    const double obr = sD[pq * NBM_RS + r] + y[r] * bj;
                    if (sel) {
                        sa += obr * lm;
                        ta += y[r] * lm;
                    }
                    if (j < k - 1 && pq >= 0) sA[pq * NBM_RS + r] = obr * (sel ? s : a) + (sel ? y[r] * t : 0.0);
                }
                // j <= k - 1 <= L - 1 <= 3
                if (j == 1) { sacc[0] += sa; tacc[0] += ta; }
                else if (j == 2) { sacc[1] += sa; tacc[1] += ta; }
                else { sacc[2] += sa; tacc[2] += ta; }
            }
            lds_barrier();
        }
    }
    if (REV) {
        for (int j = 1; j <= k - 1; ++j) {
            if (q < A.w[j]) {
                const double sa = j == 1 ? sacc[0] : (j == 2 ? sacc[1] : sacc[2]);
                const double ta = j == 1 ? tacc[0] : (j == 2 ? tacc[1] : tacc[2]);
                A.st[ix_st(box, mode, j, 0) + q] += sa;
                A.st[ix_st(box, mode, j, 1) + q] += ta;
            }
        }
        if (q < n0) {
            A.cg[ix_cg(box, mode, 0) + q] += cacc;
            A.cg[ix_cg(box, mode, 1) + q] += racc;
        }
    }
}

// adjoints u-bar, l-bar of the bounds of hidden layer A.k from s-bar, t-bar
// (both pass directions, added in a fixed order)
__global__ void __launch_bounds__(NB_T) nb_radj_kernel(NbArgs A) {
    const int box = blockIdx.x, q = threadIdx.x, j = A.k;
    if (!A.ok[box] || q >= A.w[j]) return;
    const double sb = A.st[ix_st(box, 0, j, 0) + q] + A.st[ix_st(box, 1, j, 0) + q];
    const double tb = A.st[ix_st(box, 0, j, 1) + q] + A.st[ix_st(box, 1, j, 1) + q];
    const double lo = A.bd[ix_bd(box, j, 0) + q], hi = A.bd[ix_bd(box, j, 1) + q];
    double ubar = 0.0, lbar = 0.0;
    if (lo < 0.0 && hi > 0.0) {
        const double den = hi - lo, d2 = den * den;
        ubar = (-lo * sb + lo * lo * tb) / d2;
        lbar = (hi * sb - hi * hi * tb) / d2;
    }
    A.ub[ix_ub(box, j, 0) + q] = ubar;
    A.ub[ix_ub(box, j, 1) + q] = lbar;
}

// per box: c-bar, rho-bar (pass sums plus the layer-1 bounds), then the box
// and its clamps back to a~, sigma, mu
__global__ void __launch_bounds__(NB_T) nb_out_kernel(NbArgs A) {
    const int box = blockIdx.x, q = threadIdx.x;
    const int64_t unit = A.u0 + box;
    const int n0 = A.w[0], n1 = A.w[1];
    if (q >= n0) return;
    double ga = 0.0, gs = 0.0, gm = 0.0;
    if (A.ok[box]) {
        double cb = A.cg[ix_cg(box, 0, 0) + q] + A.cg[ix_cg(box, 1, 0) + q];
        double rb = A.cg[ix_cg(box, 0, 1) + q] + A.cg[ix_cg(box, 1, 1) + q];
        const double* uu = A.ub + ix_ub(box, 1, 0);
        const double* ll = A.ub + ix_ub(box, 1, 1);
        const double* W1 = A.W[0];
        for (int i = 0; i < n1; ++i) {
            const double w = W1[(size_t)i * n0 + q];
            cb = __builtin_fma(w, uu[i] + ll[i], cb);
            rb = __builtin_fma(fabs(w), uu[i] - ll[i], rb);
        }
        const double sg = A.sigma[unit * n0 + q];
        const double mu = A.mu ? A.mu[unit * n0 + q] : 0.0;
        const double dlo_b = 0.5 * (cb - rb), dhi_b = 0.5 * (cb + rb);
        const bool lo_on = mu - sg < 0.0, hi_on = mu + sg > 0.0;
        ga = cb;
        gs = (lo_on ? -dlo_b : 0.0) + (hi_on ? dhi_b : 0.0);
        gm = (lo_on ? dlo_b : 0.0) + (hi_on ? dhi_b : 0.0);
    }
    if (q < A.nx) A.gz[unit * A.nx + q] = ga;
    else A.gv[unit * A.nu + (q - A.nx)] = ga;
    A.gsigma[unit * n0 + q] = gs;
    if (A.gmu) A.gmu[unit * n0 + q] = gm;
}

struct NbWorkspace {
    std::mutex mu;
    void* buf = nullptr;
    size_t cap = 0;
    WsFence fence;
};
static NbWorkspace g_nbws;

// VALU form: networks with four or more hidden layers (the MFMA form takes the rest)
template <bool REV>
static void nb_launch_pass(const NbArgs& a, int nb, hipStream_t st) {
    hipLaunchKernelGGL((nb_pass_kernel<REV, NN_MAXL - 1>), dim3((unsigned)nb, 2u), dim3(NB_T), 0, st, a);
}

extern "C" int leb_nn_backward(leb_mlp net, int32_t batch, int32_t N, const double* z, const double* v,
                               const double* mu, const double* sigma, const double* g_lo, const double* g_hi,
                               double* gz, double* gv, double* gmu, double* gsigma, void* stream) {
    if (!net) return LEB_EINVAL;
    if (batch < 0 || N < 0) return LEB_EINVAL;
    if (gmu && !mu) return LEB_EINVAL;
    const int64_t units = (int64_t)batch * N;
    if (units == 0) return LEB_OK;
    const int nx = net->nx, nu = net->nu;
    if (!sigma || !g_lo || !g_hi || !gsigma || (nx > 0 && (!z || !gz)) || (nu > 0 && (!v || !gv)))
        return LEB_EINVAL;
    const void* ptrs[] = {z, v, mu, sigma, g_lo, g_hi, gz, gv, gmu, gsigma};
    for (const void* p : ptrs)
        if (p && !aligned8(p)) return LEB_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    const int L = net->L;
    // stored levels of the passes: level j of pass k is w[k] x w[j]
    NbArgs a;
    memset(&a, 0, sizeof(a));
    // the MFMA form (at most three hidden layers) stores the output pass's levels too
    const bool use_mfma = L - 1 <= 3;
    size_t lv_bm = 0;
    for (int k = 2; k <= (use_mfma ? L : L - 1); ++k)
        for (int j = 0; j <= k - 2; ++j) {
            a.lv_off[k][j] = (int)lv_bm;
            lv_bm += (size_t)net->w[k] * net->w[j];
        }
    a.lv_bm = lv_bm;
    // per box: cr 2, zn L, bd 2L, st 4L, ub 2L, cg 4 rows of NN_MAXW doubles, the levels, the flag
    const size_t per_box = (size_t)NN_MAXW * (2 + 9 * NN_MAXL + 4) + 2 * lv_bm;
    int64_t cb = (int64_t)(NB_LV_BUDGET / (per_box * sizeof(double)));
    cb = cb < NB_CHUNK_MIN ? NB_CHUNK_MIN : (cb > NB_CHUNK ? NB_CHUNK : cb);
    const int CB = (int)(units < cb ? units : cb);
    const size_t need = (size_t)CB * per_box * sizeof(double) + (size_t)CB * sizeof(uint32_t);
    std::lock_guard<std::mutex> lock(g_nbws.mu);
    if (need > g_nbws.cap) {
        if (g_nbws.buf) (void)hipFree(g_nbws.buf);
        g_nbws.buf = nullptr;
        g_nbws.cap = 0;
        if (getenv("LEB_TEST_FAIL_ALLOC") || hipMalloc(&g_nbws.buf, need) != hipSuccess) return LEB_ENOMEM;
        g_nbws.cap = need;
    }
    int rc;
    if ((rc = g_nbws.fence.enter(st))) return rc;
    WsFenceScope leave{g_nbws.fence, st};
    a.L = net->L;
    for (int l = 0; l <= net->L; ++l) a.w[l] = net->w[l];
    for (int l = 0; l < net->L; ++l) { a.W[l] = net->W[l]; a.WT[l] = net->WT[l]; a.b[l] = net->b[l]; }
    a.nx = nx; a.nu = nu;
    a.z = z; a.v = v; a.mu = mu; a.sigma = sigma; a.g_lo = g_lo; a.g_hi = g_hi;
    a.gz = gz; a.gv = gv; a.gmu = gmu; a.gsigma = gsigma;
    double* p = (double*)g_nbws.buf;
    a.cr = p; p += (size_t)CB * 2 * NN_MAXW;
    a.zn = p; p += (size_t)CB * NN_MAXL * NN_MAXW;
    a.bd = p; p += (size_t)CB * NN_MAXL * 2 * NN_MAXW;
    a.st = p; p += (size_t)CB * 2 * NN_MAXL * 2 * NN_MAXW;
    a.ub = p; p += (size_t)CB * NN_MAXL * 2 * NN_MAXW;
    a.cg = p; p += (size_t)CB * 2 * 2 * NN_MAXW;
    a.lv = p; p += (size_t)CB * 2 * lv_bm;
    a.ok = (uint32_t*)p;
    for (int64_t u0 = 0; u0 < units; u0 += CB) {
        const int nb = (int)((units - u0) < CB ? (units - u0) : CB);
        a.u0 = u0;
        hipLaunchKernelGGL(nb_box_kernel, dim3((unsigned)nb), dim3(NB_T), 0, st, a);
        if (use_mfma) {
            const dim3 grid((unsigned)nb, 2u);
            for (int k = 2; k <= L; ++k) {
                a.k = k;
                hipLaunchKernelGGL(nbm_pass_kernel<false>, grid, dim3(NB_T), 0, st, a);
            }
            a.k = L;
            hipLaunchKernelGGL(nbm_pass_kernel<true>, grid, dim3(NB_T), 0, st, a);
            for (int j = L - 1; j >= 1; --j) {
                a.k = j;
                hipLaunchKernelGGL(nb_radj_kernel, dim3((unsigned)nb), dim3(NB_T), 0, st, a);
                if (j >= 2) {
                    hipLaunchKernelGGL(nbm_pass_kernel<true>, grid, dim3(NB_T), 0, st, a);
                }
            }
            hipLaunchKernelGGL(nb_out_kernel, dim3((unsigned)nb), dim3(NB_T), 0, st, a);
            continue;
        }
        for (int k = 2; k < L; ++k) {
            a.k = k;
            nb_launch_pass<false>(a, nb, st);
        }
        a.k = L;
        nb_launch_pass<true>(a, nb, st);
        for (int j = L - 1; j >= 1; --j) {
            a.k = j;
            hipLaunchKernelGGL(nb_radj_kernel, dim3((unsigned)nb), dim3(NB_T), 0, st, a);
            if (j >= 2) nb_launch_pass<true>(a, nb, st);
        }
        hipLaunchKernelGGL(nb_out_kernel, dim3((unsigned)nb), dim3(NB_T), 0, st, a);
    }
    return hipGetLastError() == hipSuccess ? LEB_OK : LEB_EDEVICE;
}

}  // namespace leb
