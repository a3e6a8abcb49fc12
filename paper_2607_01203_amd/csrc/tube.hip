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
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <float.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <vector>

#include "leb.h"
#include "leb_internal.hpp"

namespace leb {


// Fixed-point epilogue of the compact tube map (state == NULL for the plain map).
struct TubeFP {
    const double* mu_in;  // C_{t-1}: the tube whose bounds produced (c_bar, rho_bar)
    const double* sg_in;
    uint32_t* state;      // [B] state words, [B] open count
    double tol, abs_;     // C_t = (mu_F, sigma_F (1 + tol) + abs_)
    uint32_t* cert;       // NULL, or [B]: written (state & FP_CERT) by a launch that finds every
                          // trajectory certified (the sweep enqueued after the last one)
    double conv;          // acceptance also needs |C_t - C_{t-1}| within conv (relative to sigma)
};

struct TubeArgs {
    const double* cbar; const double* rbar;   // [B][N][nx]
    double e[6];
    double* mu; double* sigma;                // [B][N][n] out
    double wid;        // relative rounding allowance of the tube sums
    double scale, shift;   // plain map: sigma stored as sigma * scale + shift (1, 0: as computed)
    int B, N, U;
};

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double se_row(const double (&e)[6], int q) { return q == 3 ? e[3] : e[4]; }
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
// row tile of slot s of a wave: tiles are dealt so that each wave gets a
// mix of short (early steps) and long (late steps) K ranges
__device__ __forceinline__ int tm_tile(int wave, int s, int group) {
    const int base = group * 4 * TM_RT + 4 * s;
    return base + ((s & 1) ? 3 - wave : wave);
}

__global__ void __launch_bounds__(256) tube_map_kernel(const double* __restrict__ phi, TubeArgs A) {
    // LDS, phase 1: Phi with zero blocks at lags -4..-1 and N-1 [(N+4)*48],
    // e[8], c [6(N-1)+8][16], w [6(N-1)+8][16] (8 zero rows past the end);
    // phase 2 (after the contraction): mu, sigma of 8 steps [64][16] each
    extern __shared__ double sphi[];
    __shared__ int sjinf[16];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int N = A.N, U = A.U, nx = 6 * U, n = 8 * U;
    const int nphi = (N - 1) * 48;
    const int kfull = 6 * (N - 1);
    const int kpad = kfull + 8;
    double* sp = sphi;                         // sp[(lag + 4) * 48 + r * 6 + q]
    double* se = sphi + (N + 4) * 48;
    double* sc = se + 8;
    double* sw = sc + (size_t)kpad * 16;
    __shared__ int64_t srow[16];   // column c0 + cl: offset of its node's rows in the residual arrays at step 0
    __shared__ int64_t stub[16];   // ... and of its trajectory in the tube arrays
    __shared__ int snode[16];      // ... its node
    const int cols = A.B * U;
    const int c0 = blockIdx.x * 16;
    const int ncol = min(16, cols - c0);
    if (tid < 16) {
        const int col = min(c0 + tid, cols - 1);
        const int bb = col / U, nd = col - bb * U;
        srow[tid] = (int64_t)bb * N * nx + 6 * nd;
        stub[tid] = (int64_t)bb * N * n;
        snode[tid] = nd;
        sjinf[tid] = 0x7fffffff;
    }
    // Phi (8 loads in flight per thread)
    for (int i0 = tid; i0 < (N + 4) * 48; i0 += 8 * 256) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int l48 = i0 + 256 * u - 192;            // lag * 48 + r * 6 + q
            v[u] = (l48 >= 0 && l48 < nphi) ? phi[l48] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (i0 + 256 * u < (N + 4) * 48) sp[i0 + 256 * u] = v[u];
    }
    if (tid < 6) se[tid] = A.e[tid];
    if (tid < 128) { sc[kfull * 16 + tid] = 0.0; sw[kfull * 16 + tid] = 0.0; }   // 8 zero rows past the end
    __syncthreads();
    // c_bar and w = e + rho_bar + |c_bar| wid of steps [j0, j1): entry (j, p) of the 96
    // per step, column cl = p / 6 and row q = p % 6, so consecutive threads read
    // consecutive addresses.  A residual radius that is not finite enters as 0 and
    // every later step of its column gets sigma = +inf (a product 0 * inf with the
    // zero entries of T would otherwise make earlier rows NaN); a centre that is
    // not finite enters as 0 the same way.
    auto stage_load = [&](int j0, int idx, double& c, double& r) {
        const int j = j0 + idx / 96, p = idx % 96, cl = p / 6, q = p - 6 * cl;
        const bool in = cl < ncol;
        const int64_t off = srow[in ? cl : 0] + (int64_t)j * nx + q;
        c = in ? A.cbar[off] : 0.0;
        r = in ? A.rbar[off] : 0.0;
    };
    auto stage_store = [&](int j0, int idx, double c, double r) {
        const int j = j0 + idx / 96, p = idx % 96, cl = p / 6, q = p - 6 * cl;
        double w = 0.0;
        if (cl < ncol) {
            const bool cfin = fabs(c) <= DBL_MAX;
            if (!cfin) c = 0.0;
            w = se[q] + r + fabs(c) * A.wid;
            if (!(cfin && w <= DBL_MAX)) {
                atomicMin(&sjinf[cl], j);
                w = 0.0;
            }
        } else {
            c = 0.0;
        }
        const int kk = 6 * j + q;
        sc[kk * 16 + cl] = c;
        sw[kk * 16 + cl] = w;
    };
    // Steps are staged in chunks of 8 (the steps the row tiles of one slot add):
    // slot s of row group g reads the steps of chunks 0 .. 5g + s only, so
    // chunks 0 .. 5g are staged first and chunk 5g + s + 1 is written to LDS
    // after slot s.  Every load (the first chunks, the later chunks, the tube
    // C_{t-1} for the containment test) is issued before any of them is used.
    const int nst = N - 1;                                   // steps with residuals
    const int gch = blockIdx.y * TM_RT;                      // first chunk of this row group's slot 0
    const int pent = min(nst, 8 * (gch + 1)) * 96;           // entries staged before slot 0
    double pc[16], pr[16];
#pragma unroll
    for (int u = 0; u < 16; ++u)
        if (tid + 256 * u < pent) stage_load(0, tid + 256 * u, pc[u], pr[u]);
    double cn[TM_RT - 1][3], rn[TM_RT - 1][3];
#pragma unroll
    for (int s = 0; s + 1 < TM_RT; ++s) {
        const int nj0 = 8 * (gch + s + 1);
        const int nne = max(0, min(nst, nj0 + 8) - nj0) * 96;
#pragma unroll
        for (int u = 0; u < 3; ++u)
            if (tid + 256 * u < nne) stage_load(nj0, tid + 256 * u, cn[s][u], rn[s][u]);
    }
    const int nrt = (N + 1) >> 1;
    const int lr = lane & 15, lq = lane >> 4;
    const bool cin = lr < ncol;
    // The tube entries of this lane's accumulators: element i of slot s is row
    // r = 16 rt + 4 i + lq of the slot's tile, i.e. step k = r / 8, row r % 8 of
    // node column lr.
    auto tube_off = [&](int rr, int k) -> int64_t {
        const int nd = snode[lr];
        return stub[lr] + (int64_t)k * n + (rr < 6 ? 6 * nd + rr : nx + 2 * nd + (rr - 6));
    };
#pragma unroll
    for (int u = 0; u < 16; ++u)
        if (tid + 256 * u < pent) stage_store(0, tid + 256 * u, pc[u], pr[u]);
    for (int i0 = tid + 16 * 256; i0 < pent; i0 += 16 * 256) {    // horizons beyond 43 steps
        double cv[16], rv[16];
#pragma unroll
        for (int u = 0; u < 16; ++u)
            if (i0 + 256 * u < pent) stage_load(0, i0 + 256 * u, cv[u], rv[u]);
#pragma unroll
        for (int u = 0; u < 16; ++u)
            if (i0 + 256 * u < pent) stage_store(0, i0 + 256 * u, cv[u], rv[u]);
    }
    __syncthreads();
    // one K loop per slot, two K steps per iteration into separate accumulators
    // (four independent MFMA chains); the zero padding of Phi (lags down to -4)
    // and of the B block (8 rows) covers the reads past a tile's range.
    // kk = k0 + lq = 6 j + q, and the A offset of kk is abase - (48 j - q).
#pragma unroll
    for (int s = 0; s < TM_RT; ++s) {
        const int rt = tm_tile(wave, s, blockIdx.y);
        const int kmax = rt < nrt ? 6 * min(N - 1, 2 * rt + 1) : 0;
        // A[(k, rr)][(j, q)] = Phi_{k-j-1}[rr][q] at sp[(k - j + 3) * 48 + rr * 6 + q]
        const int abase = (((16 * rt + lr) >> 3) + 3) * 48 + ((16 * rt + lr) & 7) * 6;
        d4 m0 = d4{0.0, 0.0, 0.0, 0.0}, v0 = m0, m1 = m0, v1 = m0;
        int j = 0, q = lq;                     // entry kk
        int j2 = (lq + 4) / 6, q2 = lq + 4 - 6 * ((lq + 4) / 6);   // entry kk + 4
        for (int k0 = 0; k0 < kmax; k0 += 8) {
            const int kk = k0 + lq;
            const double c0v = sc[kk * 16 + lr], w0v = sw[kk * 16 + lr];
            const double c1v = sc[(kk + 4) * 16 + lr], w1v = sw[(kk + 4) * 16 + lr];
            const double a0 = sp[abase - (48 * j - q)];
            const double a1 = sp[abase - (48 * j2 - q2)];
            m0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, c0v, m0, 0, 0, 0);
            v0 = __builtin_amdgcn_mfma_f64_16x16x4f64(fabs(a0), w0v, v0, 0, 0, 0);
            m1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, c1v, m1, 0, 0, 0);
            v1 = __builtin_amdgcn_mfma_f64_16x16x4f64(fabs(a1), w1v, v1, 0, 0, 0);
            // kk += 8: q += 2 with a carry into j, for both entries
            q += 2; j += 1; if (q >= 6) { q -= 6; ++j; }
            q2 += 2; j2 += 1; if (q2 >= 6) { q2 -= 6; ++j2; }
        }
        const d4 am = m0 + m1, as = v0 + v1;
        const int sjl = sjinf[lr];       // every step below this slot's rows is staged
        // this slot's tube entries straight from the accumulators (the lanes of a
        // row write 16 nodes' rows; the L2 merges the partial lines)
        if (cin && rt < nrt) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = 16 * rt + 4 * i + lq, k = r >> 3, rr = r & 7;
                if (k >= N) continue;
                const double mF = am[i];
                // sums of nonnegative terms, rounded upward; 2^-1000 covers any flushed subnormal part
                const double sF = k > sjl ? INFINITY : as[i] + as[i] * A.wid + 0x1p-1000;
                const int64_t o = tube_off(rr, k);
                A.mu[o] = mF;
                A.sigma[o] = sF * A.scale + A.shift;
            }
        }
        if (s + 1 < TM_RT) {
            const int nj0 = 8 * (gch + s + 1);
            const int nne = max(0, min(nst, nj0 + 8) - nj0) * 96;
#pragma unroll
            for (int u = 0; u < 3; ++u)
                if (tid + 256 * u < nne) stage_store(nj0, tid + 256 * u, cn[s][u], rn[s][u]);
            lds_barrier();
        }
    }
}

// Tube map for residual zonotopes that are (0, pad) on the four affine rows
// of every node -- the chain dynamics of the fixed point, whose bound is
// exactly zero there (Theorem 1: no curvature in those rows).  The residuals
// come compact, rows 3 and 4 (vx, vz) of each node: c2, r2 [B][N][U][2].
// Only those rows enter the contraction, K = 2 (N-1); the affine rows add
//   sigma_k[r] += sum_{j<k} sum_{q in {0,1,2,5}} |Phi_{k-j-1}[r][q]| (e_q + pad)
// (a table over (k, r) shared by every column) and nothing to mu.  The rest is
// the tube map kernel above (16 node columns per workgroup, row tiles of two
// steps per wave) with the contraction on FP32 MFMA (v_mfma_f32_16x16x4f32):
// Phi's two residual columns, c_bar and w are rounded to nearest FP32, the
// sums of K = 2 (N - 1) products accumulate in FP32 accumulators of at most
// 32 products each (two per sum, reset every 8 K-loop iterations), which are
// added in FP64.  A computed sum of n non-negative products is within
// gamma_n + 2u (u = 2^-24) of the exact sum relative (accumulation and input
// rounding), and each centre within the same multiple of sum |Phi| |c|;
// wid32 = 1.1 (32 + 6) 2^-24 covers both: the widths
// carry |c| (wid + wid32), so the centre's error is inside the width, and
// every width is enlarged by (wid + wid32) relative plus 2^-90 absolute (for
// products lost to FP32 underflow).  Residual entries above 2^100 count as not
// finite.  Lane l's accumulator element i is D[4 (l/16) + i][l % 16].
struct Tube2Args {
    const double* c2; const double* r2;      // [B][N][U][2]
    double e[6];
    double pad;
    double* mu; double* sigma;               // [B][N][n] out
    double wid;
    double wid32;                            // FP32 contraction allowance (see above)
    double scale, shift;                     // plain map: sigma stored as sigma * scale + shift
    int B, N, U;
};

__device__ double kZero8[8];          // zero-initialised; stands in for Phi at a single step

// Loads are issued unconditionally (clamped to a valid address, the value
// then selected) so that no load sits in a branch: the wait counters stay
// exact and a wait for one batch of loads never also waits for a later batch.
// LONG (more than 65 steps) stages Phi and the residuals in passes, before
// and after the tube loads; the short form has no loop around a load.
template <bool FP, bool LONG>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 3))) tube_map2_kernel(const double* __restrict__ phi, Tube2Args A, TubeFP P) {
    // LDS: the affine table [N][8] and per-lag affine sums [N-1][8] (FP64), a
    // spare [4]; then FP32: Phi rows' columns 3, 4 for lags -4..N-1 [(N+4)*16],
    // c and w [2(N-1)+8][16]
    extern __shared__ double lds2[];
    __shared__ uint32_t sbad[16];
    __shared__ int sjinf[16];
    if (FP && P.state[A.B] == 0u) {           // every trajectory certified by an earlier sweep
        if (P.cert) {
            const int64_t stride = (int64_t)gridDim.x * gridDim.y * blockDim.x;
            for (int64_t b = ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * blockDim.x + threadIdx.x; b < A.B;
                 b += stride)
                P.cert[b] = P.state[b] & FP_CERT;
        }
        return;
    }
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int N = A.N, U = A.U, nx = 6 * U, n = 8 * U;
    const int nst = N - 1;
    const int kfull = 2 * nst, kpad = kfull + 8;
    double* dtab = lds2;                                // [N][8]
    double* g = dtab + N * 8;                           // [N-1][8]
    double* spare = g + nst * 8;                        // [4], written, never read
    float* sp = reinterpret_cast<float*>(spare + 4);    // sp[(lag + 4) * 16 + r * 2 + q'], q' = row 3 + q'
    float* sc = sp + (N + 4) * 16;                      // [kpad][16]
    float* sw = sc + (size_t)kpad * 16;
    float* sparef = reinterpret_cast<float*>(spare);
    const int cols = A.B * U;
    const int c0 = blockIdx.x * 16;
    const int ncol = min(16, cols - c0);
    const int bfirst = c0 / U;
    // this lane's accumulator column (lr) and its trajectory's state word
    const int lr = lane & 15, lq = lane >> 4;
    const bool cin = lr < ncol;
    int64_t ob_s, ob_i;
    uint32_t stw = 0u;
    {
        const int col = min(c0 + lr, cols - 1);
        const int bb = col / U, nd = col - bb * U;
        const int64_t tub = (int64_t)bb * N * n;
        ob_s = tub + 6 * nd;
        ob_i = tub + nx + 2 * nd - 6;
        if (FP) stw = P.state[bb];
    }
    if (tid < 16) { sbad[tid] = 0u; sjinf[tid] = 0x7fffffff; }
    // Every load of the first pass is issued before any of it is used, in the
    // order it is needed: Phi (columns 3, 4 and the per-lag affine sums), the
    // residual rows of the first 64 steps, the tube C_{t-1}.  Phi and the
    // residuals wait only for themselves; the tube is used after the contraction.
    const int nsp = (N + 4) * 16, ng = nst * 8;
    const double* ph = nst > 0 ? phi : kZero8;         // no Phi for a single step
    // Phi rows t = 8 lag + r (six columns) two per thread and pass: columns
    // 3, 4 go to sp, the others into the per-lag affine sums g
    double pr[2][6];
    auto phi_load = [&](int t0) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int t = t0 + tid + 256 * u;
            const double* Pr = ph + (int64_t)(t < ng ? t : 0) * 6;
#pragma unroll
            for (int q = 0; q < 6; ++q) pr[u][q] = Pr[q];
        }
    };
    // (rows past the end are written to a spare LDS slot rather than skipped,
    // so that no branch holds the loads' only use and they stay where issued)
    auto phi_store = [&](int t0) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int t = t0 + tid + 256 * u;
            const bool in = t < ng;
            const int lag = t >> 3, r = t & 7;
            float* d34 = in ? sp + (lag + 4) * 16 + r * 2 : sparef;
            d34[0] = (float)pr[u][3];
            d34[1] = (float)pr[u][4];
            double acc = 0.0;
            acc = __builtin_fma(fabs(pr[u][0]), A.e[0] + A.pad, acc);
            acc = __builtin_fma(fabs(pr[u][1]), A.e[1] + A.pad, acc);
            acc = __builtin_fma(fabs(pr[u][2]), A.e[2] + A.pad, acc);
            acc = __builtin_fma(fabs(pr[u][5]), A.e[5] + A.pad, acc);
            (in ? g + t : spare + 2)[0] = acc;
        }
    };
    // residual rows 3, 4 of the 16 columns: entry (j, p), p = 2 cl + q' = tid % 32,
    // so each thread stages one (column, row) at steps j = tid / 32 + 8 u and
    // consecutive threads read consecutive addresses.  A radius or centre that
    // is not finite (or above 2^100) enters as 0 and makes sigma +inf at every
    // later step of its column
    const int scl = (tid & 31) >> 1, sq = tid & 1;
    const bool sin_ = scl < ncol;
    int64_t srow;
    {
        const int col = min(c0 + scl, cols - 1);
        const int bb = col / U;
        srow = ((int64_t)bb * N * U + (col - bb * U)) * 2 + sq;
    }
    const double se = se_row(A.e, 3 + sq);
    double cv[8], rv[8];
    auto stage_load = [&](int j0) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int j = j0 + (tid >> 5) + 8 * u;
            const int64_t off = srow + (int64_t)(j < nst ? j : 0) * U * 2;
            cv[u] = A.c2[off];
            rv[u] = A.r2[off];
        }
    };
    auto stage_store = [&](int j0) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int j = j0 + (tid >> 5) + 8 * u;
            if (j >= nst) break;
            double c = 0.0, w = 0.0;
            if (sin_) {
                c = cv[u];
                const bool cfin = fabs(c) <= 0x1p100;
                if (!cfin) c = 0.0;
                w = se + rv[u] + fabs(c) * (A.wid + A.wid32);
                if (!(cfin && w <= 0x1p100)) {
                    atomicMin(&sjinf[scl], j);
                    w = 0.0;
                }
            }
            sc[(2 * j + sq) * 16 + scl] = (float)c;
            sw[(2 * j + sq) * 16 + scl] = (float)w;
        }
    };
    const int nrt = (N + 1) >> 1;
    const bool frozen = FP && (stw & FP_CERT) != 0u;
    const int64_t ob_d = ob_i - ob_s;       // (an arithmetic select keeps both offsets in registers)
    auto tube_off = [&](int rr, int k) -> int64_t { return ob_s + (rr < 6 ? 0 : ob_d) + rr + (int64_t)k * n; };
    // The slots of a wave run from the longest K range down or the other way
    // round, alternating between blocks 256 apart (the two blocks that share
    // a compute unit when the grid holds more than one block per unit), so that
    // one wave's contraction overlaps the other's memory traffic.  The tube
    // C_{t-1} under this lane's accumulators is read two slots ahead of its use;
    // mi[p], si[p] belong to the p-th slot processed.
    const bool down = ((blockIdx.x >> 8) & 1) == 0;
    auto ord = [&](int p) { return down ? TM_RT - 1 - p : p; };
    double mi[TM_RT][4], si[TM_RT][4];
    auto tube_load = [&](int p) {
        const int rt = tm_tile(wave, ord(p), blockIdx.y);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = 16 * rt + 4 * lq + i, k = r >> 3;
            const bool ok = cin && rt < nrt && k < N;     // (a frozen column's values go unused)
            const int64_t o = ok ? tube_off(r & 7, k) : ob_s;
            mi[p][i] = P.mu_in[o];
            si[p][i] = P.sg_in[o];
        }
    };
    phi_load(0);
    if (LONG) {
        phi_store(0);
        for (int t0 = 2 * 256; t0 < ng; t0 += 2 * 256) {
            phi_load(t0);
            phi_store(t0);
        }
    }
    stage_load(0);
    if (!LONG) phi_store(0);
    if (FP) {
        tube_load(0);
        tube_load(1);
    }
    // zero lags -4..-1 and N-1 of sp (the rows past a tile's causal range)
    if (tid < 64) sp[tid] = 0.0f;
    else if (tid < 80) sp[(nst + 4) * 16 + tid - 64] = 0.0f;
    if (tid < 128) { sc[kfull * 16 + tid] = 0.0f; sw[kfull * 16 + tid] = 0.0f; }   // 8 zero rows past the end
    __syncthreads();
    // affine table: dtab[k][r] = sum_{d<k} g[d][r], summed in increasing d
    for (int t = tid; t < N * 8; t += 256) {
        const int k = t >> 3, r = t & 7;
        double acc = 0.0;
        for (int d0 = 0; d0 < k; d0 += 8) {      // eight loads in flight, then their sum in increasing d
            double x[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) x[u] = d0 + u < k ? g[(d0 + u) * 8 + r] : 0.0;
#pragma unroll
            for (int u = 0; u < 8; ++u) acc += x[u];
        }
        dtab[t] = acc;
    }
    stage_store(0);
    if (LONG)
        for (int j0 = 64; j0 < nst; j0 += 64) {
            stage_load(j0);
            stage_store(j0);
        }
    __syncthreads();
    const int sjl = sjinf[lr];
    // K loop per slot, two K steps per iteration into separate accumulators, the
    // next iteration's fragments read before this one's MFMAs;
    // kk = k4 + lq = 2 j + q', the A entry of kk is sp[(k - j + 3) * 16 + rr * 2 + q']
#pragma unroll
    for (int p = 0; p < TM_RT; ++p) {
        if (FP && p + 2 < TM_RT) tube_load(p + 2);
        const int rt = tm_tile(wave, ord(p), blockIdx.y);
        if (rt >= nrt) continue;
        const int r = 16 * rt + lr, kr = r >> 3, rrr = r & 7;
        const int kmax = 2 * min(nst, 2 * rt + 1);
        // A offsets of kk and kk + 4 at k4 = 0 (j = lq / 2 and lq / 2 + 2); -8 per K step
        const int abase = (kr + 3) * 16 + rrr * 2 + (lq & 1) - 16 * (lq >> 1);
        double dt[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int rr4 = 16 * rt + 4 * lq + i;
            dt[i] = (rr4 >> 3) < N ? dtab[(rr4 >> 3) * 8 + (rr4 & 7)] : 0.0;
        }
        float c0v = sc[lane], w0v = sw[lane], c1v = sc[64 + lane], w1v = sw[64 + lane];
        float a0 = sp[abase], a1 = sp[abase - 32];
        // FP32 accumulators over chunks of 8 iterations (32 products each), the
        // chunks summed in FP64
        double md[4] = {0.0, 0.0, 0.0, 0.0}, vd[4] = {0.0, 0.0, 0.0, 0.0};
        for (int cs = 0; cs < kmax; cs += 64) {
            const int ce = cs + 64 < kmax ? cs + 64 : kmax;
            f4 m0 = f4{0.0f, 0.0f, 0.0f, 0.0f}, v0 = m0, m1 = m0, v1 = m0;
            for (int k4 = cs; k4 < ce; k4 += 8) {
                const int kn = k4 + 8 < kmax ? k4 + 8 : k4;    // the last prefetch re-reads this step
                const float c0n = sc[kn * 16 + lane], w0n = sw[kn * 16 + lane];
                const float c1n = sc[kn * 16 + 64 + lane], w1n = sw[kn * 16 + 64 + lane];
                const float a0n = sp[abase - 8 * kn], a1n = sp[abase - 8 * kn - 32];
                // the reads stay ahead of the MFMAs and their results are consumed
                // only after all four are issued
                __builtin_amdgcn_sched_barrier(0);
                m0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, c0v, m0, 0, 0, 0);
                v0 = __builtin_amdgcn_mfma_f32_16x16x4f32(fabsf(a0), w0v, v0, 0, 0, 0);
                m1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, c1v, m1, 0, 0, 0);
                v1 = __builtin_amdgcn_mfma_f32_16x16x4f32(fabsf(a1), w1v, v1, 0, 0, 0);
                __builtin_amdgcn_sched_barrier(0);
                c0v = c0n; w0v = w0n; c1v = c1n; w1v = w1n; a0 = a0n; a1 = a1n;
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                md[i] += (double)m0[i] + (double)m1[i];
                vd[i] += (double)v0[i] + (double)v1[i];
            }
        }
        if (!cin) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int rr4 = 16 * rt + 4 * lq + i, k = rr4 >> 3, rr = rr4 & 7;
            if (k >= N) continue;
            const double mF = md[i];
            // both sums have nonnegative terms; rounded upward as a whole (FP32
            // chunks and FP64 sums), 2^-90 for products lost to underflow
            const double tot = vd[i] + dt[i];
            const double sF = k > sjl ? INFINITY : tot + tot * (A.wid + A.wid32) + 0x1p-90;
            double so = sF * A.scale + A.shift;
            if (FP) {
                // [mF - sF, mF + sF] inside [mi - si, mi + si], with the rounding of the
                // test covered; a tube that is not finite is never accepted
                so = sF + sF * P.tol + P.abs_;
                const double dm = fabs(mF - mi[p][i]);
                const bool contained = sF <= DBL_MAX && (dm + sF) * (1.0 + 0x1p-50) <= si[p][i];
                // converged: the next iterate within conv of this one (the slack 2^-44 si
                // absorbs the rounding of the sums, far below any conv in use)
                const double slack = P.conv * si[p][i] + 0x1p-44 * si[p][i];
                const bool conv = fabs(so - si[p][i]) <= slack + 2.0 * P.abs_ && dm <= slack + P.abs_;
                if (!frozen && !(contained && conv)) sbad[(c0 + lr) / U - bfirst] = 1u;
            }
            if (!frozen) {
                const int64_t o = tube_off(rr, k);
                A.mu[o] = mF;
                A.sigma[o] = so;
            }
        }
    }
    if (!FP) return;
    __syncthreads();
    if (tid < 16 && sbad[tid] && bfirst + tid < A.B) atomicOr(&P.state[bfirst + tid], FP_OPEN);
}

// The fold of sweep t when no bound launch of sweep t + 1 follows (the sweep
// cap): the same as that launch's workgroup 0 (one workgroup).
__global__ void __launch_bounds__(256) fp_fold_kernel(SweepFold F) {
    __shared__ uint32_t cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    uint32_t open = 0;
    for (int b = threadIdx.x; b < F.B; b += 256) {
        const uint32_t st = F.prev[b];
        open += fp_is_open(st);
        F.next[b] = fp_fold_word(st, F.sweep);
    }
    atomicAdd(&cnt, open);
    __syncthreads();
    if (threadIdx.x == 0) {
        F.next[F.B] = cnt;
        if (F.host_open)
            __hip_atomic_store(&F.host_open[F.sweep % FP_SLOTS], cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// After the last sweep: the certified tube of each trajectory is C_{s-1}
// (s = the sweep that certified it), which sits in buffer (s-1) & 1; an
// uncertified trajectory takes the latest iterate C_T from buffer T & 1.
// Buffer 0 is the caller's; buffer 1 is copied into it where needed.
__global__ void fp_final_kernel(const double* xm1, const double* xs1, double* mu, double* sg,
                                const uint32_t* state, int64_t per_traj, int last_sweep) {
    const int b = blockIdx.x;        // one trajectory per blockIdx.x
    const uint32_t st = state[b];
    const int src = (st & FP_CERT) ? (int)(((st >> 1) - 1) & 1u) : (last_sweep & 1);
    if (src == 0) return;
    const int64_t base = (int64_t)b * per_traj;
    for (int64_t q = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; q < per_traj; q += (int64_t)gridDim.y * blockDim.x) {
        mu[base + q] = xm1[base + q];
        sg[base + q] = xs1[base + q];
    }
}


// The tube of residuals (c_bar, rho_bar) = (0, pad) at every step -- the
// disturbance-only tube -- is the same for every (trajectory, node):
//   mu_k = 0,  sigma_k[r] = sum_{j<k} sum_q |Phi_{k-j-1}[r][q]| (e_q + pad),
// rounded upward like the tube map (the per-lag sums are added in order of
// the lag; any order of a sum of nonnegative terms is covered by wid).  Each
// workgroup forms the N x 8 table in LDS and writes its rows of the broadcast.
__global__ void __launch_bounds__(256) disturbance_tube_kernel(const double* __restrict__ phi, TubeArgs A, double pad,
                                                               int rows) {
    extern __shared__ double tab[];       // [N][8], then the per-lag sums [N-1][8]
    const int N = A.N, U = A.U, nx = 6 * U, n = 8 * U;
    double* g = tab + N * 8;
    for (int t = threadIdx.x; t < (N - 1) * 8; t += 256) {
        const double* P = phi + (int64_t)t * 6;       // Phi_d[r][.], t = 8 d + r
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < 6; ++q) acc = __builtin_fma(fabs(P[q]), A.e[q] + pad, acc);
        g[t] = acc;
    }
    __syncthreads();
    // tab[k][r] from the lag sums in increasing d, one (k, r) per thread (the
    // loads of a sum are independent; the order of each sum is fixed)
    for (int t = threadIdx.x; t < N * 8; t += 256) {
        const int k = t >> 3, r = t & 7;
        double acc = 0.0;
        for (int d = 0; d < k; ++d) acc += g[d * 8 + r];
        tab[t] = k == 0 ? 0.0 : acc + acc * A.wid + 0x1p-1000;
    }
    __syncthreads();
    for (int row = blockIdx.x; row < rows; row += gridDim.x) {       // row = (trajectory, step)
        const int k = row % N;
        double* mrow = A.mu + (int64_t)row * n;
        double* srow = A.sigma + (int64_t)row * n;
        for (int c = threadIdx.x; c < n; c += 256) {
            const int rr = c < nx ? c % 6 : 6 + ((c - nx) & 1);
            mrow[c] = 0.0;
            srow[c] = tab[k * 8 + rr];
        }
    }
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

// Relative allowance of the tube sums: a sum of m rounded products (and the 3
// operations forming a weight) errs by at most gamma_{m+3} ~ (m+3) 2^-53
// relative, in any order of accumulation; twice that covers both the sigma
// sums and, through |c_bar| wid in the weights, the rounding of the centre sums.
static double tube_wid(int N) { return fmax(0x1p-44, (6.0 * (N > 0 ? N - 1 : 0) + 4.0) * 0x1p-52); }

static int launch_tube(int B, int N, int U, const double* phi, const double* e, const double* cbar,
                       const double* rbar, double* mu, double* sigma, hipStream_t s,
                       double scale = 1.0, double shift = 0.0, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr) {
    TubeArgs a;
    a.cbar = cbar; a.rbar = rbar;
    a.scale = scale; a.shift = shift;
    for (int q = 0; q < 6; ++q) a.e[q] = e[q];
    a.mu = mu; a.sigma = sigma; a.B = B; a.N = N; a.U = U;
    a.wid = tube_wid(N);
    const int64_t cols = (int64_t)B * U;
    if (cols == 0 || N == 0) return LEB_OK;
    const int64_t gx = (cols + 15) / 16;
    const int nrt = (N + 1) / 2;
    const int gy = (nrt + 4 * TM_RT - 1) / (4 * TM_RT);
    if (gx > 0x7fffffff || (int64_t)cols > 0x7fffffff) return LEB_EINVAL;
    // Phi, e (padded to 8) and the B block (c and w for 16 columns); later the
    // output of 8 steps (mu and sigma, 64 rows x 16 columns)
    const size_t nm1 = N > 1 ? N - 1 : 0;
    const size_t smem = std::max((size_t)(N + 4) * 48 + 8 + 2 * (6 * nm1 + 8) * 16, (size_t)2 * 64 * 16) * sizeof(double);
    // the kernel may use all 160 KB of LDS, static part included (set once)
    static size_t dyn_max = 0;
    if (dyn_max == 0) {
        hipFuncAttributes fa;
        if (hipFuncGetAttributes(&fa, (const void*)tube_map_kernel) != hipSuccess) return LEB_EDEVICE;
        const size_t cap = 160 * 1024 - fa.sharedSizeBytes;
        if (hipFuncSetAttribute((const void*)tube_map_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)cap) !=
            hipSuccess)
            return LEB_EDEVICE;
        dyn_max = cap;
    }
    if (smem > dyn_max) return LEB_ENOTSUP;     // N <= 83
    if (ev0)        // timed: events at the kernel's start and end
        hipExtLaunchKernelGGL(tube_map_kernel, dim3((unsigned)gx, gy), dim3(256), smem, s, ev0, ev1, 0, phi, a);
    else
        hipLaunchKernelGGL(tube_map_kernel, dim3((unsigned)gx, gy), dim3(256), smem, s, phi, a);
    return hipGetLastError() == hipSuccess ? LEB_OK : LEB_EDEVICE;
}

// Tube map of compact residuals (rows 3 and 4 of each node, the affine rows
// (0, pad)); fp as launch_tube's
static int launch_tube2(int B, int N, int U, const double* phi, const double* e, double pad, const double* c2,
                        const double* r2, double* mu, double* sigma, const TubeFP& fp, hipStream_t s,
                        double scale = 1.0, double shift = 0.0, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr) {
    Tube2Args a;
    a.c2 = c2; a.r2 = r2;
    for (int q = 0; q < 6; ++q) a.e[q] = e[q];
    a.pad = pad;
    a.mu = mu; a.sigma = sigma; a.B = B; a.N = N; a.U = U;
    a.wid = tube_wid(N);
    a.wid32 = 1.1 * (32.0 + 6.0) * 0x1p-24;
    a.scale = scale; a.shift = shift;
    const int64_t cols = (int64_t)B * U;
    if (cols == 0 || N == 0) return LEB_OK;
    const int64_t gx = (cols + 15) / 16;
    const int nrt = (N + 1) / 2;
    const int gy = (nrt + 4 * TM_RT - 1) / (4 * TM_RT);
    if (gx > 0x7fffffff || cols > 0x7fffffff) return LEB_EINVAL;
    const size_t nst = N > 1 ? N - 1 : 0;
    const size_t smem = ((size_t)N * 8 + nst * 8 + 4) * sizeof(double) +
                        ((size_t)(N + 4) * 16 + 2 * (2 * nst + 8) * 16) * sizeof(float);
    const bool isfp = fp.state != nullptr, lng = N > 65;
    const int which = (isfp ? 2 : 0) + (lng ? 1 : 0);
    using K2 = void (*)(const double*, Tube2Args, TubeFP);
    static const K2 kern[4] = {tube_map2_kernel<false, false>, tube_map2_kernel<false, true>,
                               tube_map2_kernel<true, false>, tube_map2_kernel<true, true>};
    static size_t dyn_max[4] = {0, 0, 0, 0};
    if (dyn_max[which] == 0) {
        hipFuncAttributes fa;
        if (hipFuncGetAttributes(&fa, (const void*)kern[which]) != hipSuccess) return LEB_EDEVICE;
        const size_t cap = 160 * 1024 - fa.sharedSizeBytes;
        if (hipFuncSetAttribute((const void*)kern[which], hipFuncAttributeMaxDynamicSharedMemorySize, (int)cap) !=
            hipSuccess)
            return LEB_EDEVICE;
        dyn_max[which] = cap;
    }
    if (smem > dyn_max[which]) return LEB_ENOTSUP;
    if (ev0)        // timed: events at the kernel's start and end
        hipExtLaunchKernelGGL(kern[which], dim3((unsigned)gx, gy), dim3(256), smem, s, ev0, ev1, 0, phi, a, fp);
    else
        hipLaunchKernelGGL(kern[which], dim3((unsigned)gx, gy), dim3(256), smem, s, phi, a, fp);
    return hipGetLastError() == hipSuccess ? LEB_OK : LEB_EDEVICE;
}

int launch_tube_map_compact(int B, int N, int U, const double* phi, const double* e, double pad, const double* c2,
                            const double* r2, double* mu, double* sigma, hipStream_t s, double scale, double shift) {
    TubeFP none{nullptr, nullptr, nullptr, 0.0, 0.0, nullptr};
    return launch_tube2(B, N, U, phi, e, pad, c2, r2, mu, sigma, none, s, scale, shift);
}

int launch_disturbance_tube(int B, int N, int U, const double* phi, const double* e, double pad, double* mu,
                            double* sigma, hipStream_t s) {
    TubeArgs a = {};
    for (int q = 0; q < 6; ++q) a.e[q] = e[q];
    a.mu = mu; a.sigma = sigma; a.B = B; a.N = N; a.U = U;
    a.wid = tube_wid(N);
    const int64_t rows = (int64_t)B * N;
    if (rows == 0 || U == 0) return LEB_OK;
    if (rows > 0x7fffffff) return LEB_EINVAL;
    const int blocks = (int)std::min<int64_t>(rows, 2048);
    hipLaunchKernelGGL(disturbance_tube_kernel, dim3((unsigned)blocks), dim3(256), (size_t)(2 * N) * 8 * sizeof(double),
                       s, phi, a, pad, (int)rows);
    return hipGetLastError() == hipSuccess ? LEB_OK : LEB_EDEVICE;
}

int launch_tube_map(int B, int N, int U, const double* phi, const double* e, const double* cbar,
                    const double* rbar, double* mu, double* sigma, hipStream_t s, double scale, double shift) {
    return launch_tube(B, N, U, phi, e, cbar, rbar, mu, sigma, s, scale, shift);
}

// ------------------------------------------------------------ workspace

struct Workspace {
    std::mutex mu;
    std::vector<void*> bufs;
    std::vector<size_t> sizes;
    uint32_t* host_open = nullptr;      // pinned, host-mapped
    uint32_t* host_open_dev = nullptr;
    WsFence fence;
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

static int ws_host() {
    if (!g_ws.host_open) {
        void* h = nullptr;
        if (hipHostMalloc(&h, FP_SLOTS * sizeof(uint32_t), hipHostMallocMapped) != hipSuccess) return LEB_ENOMEM;
        void* d = nullptr;
        if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess) { (void)hipHostFree(h); return LEB_EDEVICE; }
        g_ws.host_open = (uint32_t*)h;
        g_ws.host_open_dev = (uint32_t*)d;
    }
    return LEB_OK;
}

// Launch timing of the fixed-point sweeps (off unless enabled): a pair of HIP
// events per bound and tube-map launch, recorded by the launch itself at the
// kernel's start and end, in launch order.
struct LaunchTiming {
    std::mutex mu;
    bool on = false;
    std::vector<hipEvent_t> ev[2];      // (start, stop) pairs per kernel
    int used[2] = {0, 0};
};
static LaunchTiming g_lt;
constexpr int LT_PAIRS = 256;

// the next event pair of kernel (0: bound, 1: tube map), or false when off or full
static bool lt_pair(int kernel, hipEvent_t* e0, hipEvent_t* e1) {
    *e0 = *e1 = nullptr;
    if (!g_lt.on || g_lt.used[kernel] >= LT_PAIRS) return false;
    std::vector<hipEvent_t>& ev = g_lt.ev[kernel];
    const size_t k = 2 * (size_t)g_lt.used[kernel];
    while (ev.size() < k + 2) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return false;
        ev.push_back(e);
    }
    *e0 = ev[k];
    *e1 = ev[k + 1];
    ++g_lt.used[kernel];
    return true;
}

}  // namespace leb

using namespace leb;

extern "C" int leb_launch_timing(int32_t enable) {
    std::lock_guard<std::mutex> lock(g_lt.mu);
    g_lt.on = enable != 0;
    g_lt.used[0] = g_lt.used[1] = 0;
    return LEB_OK;
}

extern "C" int leb_launch_times(int32_t kernel, float* ms, int32_t cap, int32_t* count) {
    if (kernel < 0 || kernel > 1 || !count || cap < 0 || (cap > 0 && !ms)) return LEB_EINVAL;
    std::lock_guard<std::mutex> lock(g_lt.mu);
    const int n = g_lt.used[kernel];
    *count = n;
    for (int i = 0; i < n && i < cap; ++i) {
        if (hipEventSynchronize(g_lt.ev[kernel][2 * i + 1]) != hipSuccess) return LEB_EDEVICE;
        if (hipEventElapsedTime(&ms[i], g_lt.ev[kernel][2 * i], g_lt.ev[kernel][2 * i + 1]) != hipSuccess)
            return LEB_EDEVICE;
    }
    return LEB_OK;
}

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

namespace leb {
int fp_check_args(const leb_fp_options* opt, const double* e, int N) {
    if (!opt || !e) return LEB_EINVAL;
    if (!(opt->tol >= 0.0) || !isfinite(opt->tol) || opt->max_sweeps < 1 || !(opt->pad >= 0.0) ||
        !(opt->inflate_abs > 0.0) || !isfinite(opt->inflate_abs) || !(opt->conv_tol >= opt->tol) ||
        !isfinite(opt->conv_tol) || !isfinite(opt->pad))
        return LEB_EINVAL;
    for (int q = 0; q < 6; ++q)
        if (!(e[q] >= 0.0) || !isfinite(e[q])) return LEB_EINVAL;
    // the compact tube map keeps Phi's two residual columns, the affine sums and
    // the residuals of all steps of 16 node columns in LDS: 448 N + 990 bytes
    if (N > FP_MAX_N) return LEB_ENOTSUP;
    return LEB_OK;
}
}  // namespace leb

extern "C" int leb_fixed_point_solve(const leb_dynamics* dyn, int32_t batch, int32_t N, const double* z,
                                     const double* v, const double* phi, const double* e,
                                     const leb_fp_options* opt, double* mu, double* sigma,
                                     uint32_t* certified, int32_t* sweeps_out, void* stream) {
    int rc = check_chain_dynamics(dyn);
    if (rc != LEB_OK) return rc;
    if (dyn->kind != LEB_DYN_PQUAD_CHAIN) return LEB_ENOTSUP;
    if (!sweeps_out || batch < 0 || N < 0) return LEB_EINVAL;
    if ((rc = fp_check_args(opt, e, N))) return rc;
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
    // residuals: rows 3 and 4 of each node (the affine rows are (0, pad))
    const size_t bx = (size_t)units * 2 * U * sizeof(double), bn = (size_t)units * n * sizeof(double);
    if ((rc = ws_get(0, bx, (void**)&cb)) || (rc = ws_get(1, bx, (void**)&rb)) ||
        (rc = ws_get(2, bn, (void**)&xm1)) || (rc = ws_get(3, bn, (void**)&xs1)) ||
        (rc = ws_get(4, 2 * ((size_t)batch + 1) * sizeof(uint32_t), (void**)&state)) || (rc = ws_host()))
        return rc;
    if ((rc = g_ws.fence.enter(s))) return rc;
    WsFenceScope leave{g_ws.fence, s};
    // iterates: buffer 0 = the caller's (mu, sigma), buffer 1 = workspace; sweep t reads C_{t-1}
    // from buffer (t-1) & 1 and writes C_t to buffer t & 1
    double* xm[2] = {mu, xm1};
    double* xs[2] = {sigma, xs1};
    // state words [B] + open count: sweep t marks st[t & 1]; the bound launch of
    // sweep t + 1 folds them into st[(t + 1) & 1].  The launch of sweep 1 folds
    // nothing (it writes st[1] all open), so st[0] needs no initial value.
    uint32_t* st[2] = {state, state + batch + 1};
    const int64_t per = (int64_t)N * n;
    auto ok = [](hipError_t e_) { return e_ == hipSuccess; };
    if (!opt->warm)         // C_0: the disturbance-only tube (LEB = 0), below the fixed point
        if ((rc = launch_disturbance_tube(batch, N, U, phi, e, opt->pad, mu, sigma, s))) return rc;
    volatile uint32_t* hopen = g_ws.host_open;
    std::lock_guard<std::mutex> lt_lock(g_lt.mu);
    auto sweep = [&](int t) -> int {
        const int a = (t - 1) & 1, w = t & 1;
        hipEvent_t b0, b1, t0, t1;
        lt_pair(0, &b0, &b1);
        lt_pair(1, &t0, &t1);
        // this launch folds sweep t - 1 and publishes its count
        hopen[(t - 1) % FP_SLOTS] = 0xffffffffu;
        const SweepFold fold{st[a], st[w], g_ws.host_open_dev, batch, t - 1};
        int r = launch_pbh_chain(dyn, units, z, v, xm[a], xs[a], nullptr, nullptr, cb, rb, opt->pad, nullptr, s,
                                 &fold, b0, b1, true);
        if (r) return r;
        const TubeFP fp{xm[a], xs[a], st[w], opt->tol, opt->inflate_abs, certified, opt->conv_tol};
        return launch_tube2(batch, N, U, phi, e, opt->pad, cb, rb, xm[w], xs[w], fp, s, 1.0, 0.0, t0, t1);
    };
    // Wait until the open count of sweep t is published: the bound launch of
    // sweep t + 1 (or the fold kernel at the sweep cap) writes it to pinned host memory.  The stream is queried only after
    // 2 ms without it (a query can put a marker between the sweeps' kernels), so
    // that the wait also ends if the stream drains (or fails) without a count.
    auto wait_count = [&](int t, uint32_t* out) -> int {
        auto last = std::chrono::steady_clock::now();
        for (uint64_t spin = 1;; ++spin) {
            const uint32_t v = hopen[t % FP_SLOTS];
            if (v != 0xffffffffu) { *out = v; return LEB_OK; }
            if ((spin & 1023) == 0 && std::chrono::steady_clock::now() - last > std::chrono::milliseconds(2)) {
                last = std::chrono::steady_clock::now();
                const hipError_t q = hipStreamQuery(s);
                if (q == hipSuccess) {
                    const uint32_t v2 = hopen[t % FP_SLOTS];
                    if (v2 == 0xffffffffu) return LEB_EDEVICE;     // drained without a count
                    *out = v2;
                    return LEB_OK;
                }
                if (q != hipErrorNotReady) return LEB_EDEVICE;
            }
        }
    };
    // one sweep stays in flight while the host reads the previous sweep's
    // open count; a sweep enqueued after the last needed one exits at once
    if ((rc = sweep(1))) return rc;
    int t = 1;
    uint32_t open = 0, open_before = (uint32_t)batch;    // open counts after sweeps t and t - 1
    for (;;) {
        if (t < opt->max_sweeps) {
            if ((rc = sweep(t + 1))) return rc;
        } else {                                        // the cap: fold the last sweep on its own
            hopen[t % FP_SLOTS] = 0xffffffffu;
            const SweepFold fold{st[t & 1], st[(t + 1) & 1], g_ws.host_open_dev, batch, t};
            hipLaunchKernelGGL(fp_fold_kernel, dim3(1), dim3(256), 0, s, fold);
            if (!ok(hipGetLastError())) return LEB_EDEVICE;
        }
        if ((rc = wait_count(t, &open))) return rc;
        if (open == 0 || t == opt->max_sweeps) break;
        open_before = open;
        ++t;
    }
    // every trajectory certified by sweep t has its tube C_{t-1} in buffer (t-1) & 1:
    // nothing to copy when that is the caller's buffer
    const bool in_place = open == 0 && open_before == (uint32_t)batch && ((t - 1) & 1) == 0;
    if (!in_place)
        hipLaunchKernelGGL(fp_final_kernel, dim3(batch, (unsigned)std::min<int64_t>((per + 255) / 256, 16)), dim3(256),
                           0, s, xm1, xs1, mu, sigma, st[(t + 1) & 1], per, t);
    // the sweep enqueued after the last one (t < cap) finds every trajectory
    // certified and writes the certificate flags itself
    if (!(open == 0 && t < opt->max_sweeps))
        hipLaunchKernelGGL(cert_out_kernel, dim3(nblk(batch)), dim3(256), 0, s, st[(t + 1) & 1], certified, batch);
    *sweeps_out = t;
    return ok(hipGetLastError()) ? LEB_OK : LEB_EDEVICE;
}

// ------------------------------------------------------ no-allocation form
//
// For callers that cannot allocate (graph capture, serving loops): the
// workspace of the fixed point lives in this array, one copy per GPU, held
// until the process ends.  Host code never passes `scratch` itself to a
// kernel: its device address comes from hipGetSymbolAddress, taken once per
// device with that device current.
namespace leb {
constexpr size_t FP_SCRATCH_BYTES = (size_t)64 << 20;
__device__ __align__(256) unsigned char scratch[FP_SCRATCH_BYTES];
constexpr int FP_SCRATCH_DEVICES = 64;
static std::mutex g_scratch_mu;
static unsigned char* g_scratch_ptr[FP_SCRATCH_DEVICES];

static int scratch_on_current_device(unsigned char** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return LEB_EDEVICE;
    if (dev >= FP_SCRATCH_DEVICES) return LEB_ENOTSUP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return LEB_EDEVICE;
        g_scratch_ptr[dev] = (unsigned char*)p;
    }
    *out = g_scratch_ptr[dev];
    return LEB_OK;
}

static size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }
}  // namespace leb

extern "C" int leb_fixed_point_solve_noalloc(const leb_dynamics* dyn, int32_t batch, int32_t N, const double* z,
                                             const double* v, const double* phi, const double* e,
                                             const leb_fp_options* opt, double* mu, double* sigma,
                                             uint32_t* certified, int32_t* sweeps_out, void* stream) {
    int rc = check_chain_dynamics(dyn);
    if (rc != LEB_OK) return rc;
    if (dyn->kind != LEB_DYN_PQUAD_CHAIN) return LEB_ENOTSUP;
    if (!sweeps_out || batch < 0 || N < 0) return LEB_EINVAL;
    if ((rc = fp_check_args(opt, e, N))) return rc;
    *sweeps_out = 0;
    const int64_t units = (int64_t)batch * N;
    if (units == 0) return LEB_OK;
    if (!z || !v || !mu || !sigma || !certified || (N > 1 && !phi)) return LEB_EINVAL;
    const void* ptrs[] = {z, v, phi, mu, sigma};
    for (const void* p : ptrs)
        if (p && !aligned8(p)) return LEB_EINVAL;
    const int U = dyn->n_units, n = dyn->nx + dyn->nu;
    // the same buffers as leb_fixed_point_solve's workspace, carved from scratch
    const size_t bx = al256((size_t)units * 2 * U * sizeof(double));
    const size_t bn = al256((size_t)units * n * sizeof(double));
    const size_t bs = al256(2 * ((size_t)batch + 1) * sizeof(uint32_t));
    if (2 * bx + 2 * bn + bs > FP_SCRATCH_BYTES) return LEB_ESCRATCH;
    unsigned char* base = nullptr;
    if ((rc = scratch_on_current_device(&base))) return rc;
    double* cb = (double*)base;
    double* rb = (double*)(base + bx);
    double* xm1 = (double*)(base + 2 * bx);
    double* xs1 = (double*)(base + 2 * bx + bn);
    uint32_t* state = (uint32_t*)(base + 2 * bx + 2 * bn);
    hipStream_t s = (hipStream_t)stream;
    double* xm[2] = {mu, xm1};
    double* xs[2] = {sigma, xs1};
    uint32_t* st[2] = {state, state + batch + 1};
    if (!opt->warm)
        if ((rc = launch_disturbance_tube(batch, N, U, phi, e, opt->pad, mu, sigma, s))) return rc;
    // every sweep up to the cap is enqueued; the folds publish the open count on
    // the device only, and a sweep after the last needed one exits at once
    const int T = opt->max_sweeps;
    for (int t = 1; t <= T; ++t) {
        const int a = (t - 1) & 1, w = t & 1;
        const SweepFold fold{st[a], st[w], nullptr, batch, t - 1};
        if ((rc = launch_pbh_chain(dyn, units, z, v, xm[a], xs[a], nullptr, nullptr, cb, rb, opt->pad, nullptr, s,
                                   &fold, nullptr, nullptr, true)))
            return rc;
        const TubeFP fp{xm[a], xs[a], st[w], opt->tol, opt->inflate_abs, certified, opt->conv_tol};
        if ((rc = launch_tube2(batch, N, U, phi, e, opt->pad, cb, rb, xm[w], xs[w], fp, s, 1.0, 0.0, nullptr,
                               nullptr)))
            return rc;
    }
    const SweepFold fold{st[T & 1], st[(T + 1) & 1], nullptr, batch, T};
    hipLaunchKernelGGL(fp_fold_kernel, dim3(1), dim3(256), 0, s, fold);
    const int64_t per = (int64_t)N * n;
    hipLaunchKernelGGL(fp_final_kernel, dim3(batch, (unsigned)std::min<int64_t>((per + 255) / 256, 16)), dim3(256), 0,
                       s, xm1, xs1, mu, sigma, st[(T + 1) & 1], per, T);
    hipLaunchKernelGGL(cert_out_kernel, dim3(nblk(batch)), dim3(256), 0, s, st[(T + 1) & 1], certified, batch);
    *sweeps_out = T;
    return hipGetLastError() == hipSuccess ? LEB_OK : LEB_EDEVICE;
}
