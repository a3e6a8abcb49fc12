// sls.hip -- the system-level-synthesis layer around the bound: closed-loop
// responses from the parallel Riccati recursions, the time-varying tube map
// over them, the state-dependent disturbance error, and the exact tube/LEB
// fixed point of one controller update.
//
// Responses (appendix on solving for Phi, eqs. backward_prop and
// forward_prop; reformulated problem eq. fastsls_qp_reform): the problem
// splits over the disturbance time j, so one workgroup owns one (trajectory,
// j) pair and runs, with every matrix in LDS,
//   backward  P_{N,j} = diag(qx_{N,j}); for k = N-1 .. j+1:
//             S = diag(qu_{k,j}) + B_k^T P B_k,  Bc = B_k^T P A_k,
//             K_{k,j} = -S^-1 Bc (Cholesky),  P <- diag(qx_{k,j}) + A_k^T P A_k + K^T Bc
//   forward   X = I; for k = j+1 .. N-1: Phi^x_{k,j} = X, Phi^u_{k,j} = K_{k,j} X,
//             X <- (A_k + B_k K_{k,j}) X.
// All FP64: the gains define the controller, they are not enclosures.
//
// Tube (eqs. tight_tube_center, tight_tube_width) with per-step disturbance
// matrices E_j [nx][nw]:
//   mu_k = sum_{j<k} Phi_{k,j} c_bar_j,
//   sigma_k = sum_{j<k} |Phi_{k,j} E_j| 1 + |Phi_{k,j}| rho_bar_j,
// plus an allowance that covers the FP64 rounding of both sums.  The blocks
// Phi_{k,0..k-1} of one row k are contiguous, so a workgroup streams its row
// once, coalesced, through LDS.
//
// Fixed point (section V loop, Theorem 3): the map from the bounds to the
// tube is causal (the tube at k needs the bounds at j < k only), so one pass
// over k in order gives the exact fixed point C = F(C): step k runs one row
// launch (finish step k-1's residual zonotope, then the tube row k) and one
// bound launch over all trajectories at step k.  The tube rows round upward
// and the bounds are outward, so C is a post-fixed point of the exact map and
// the Theorem 3 induction holds.
//
// Disturbance error (eqs. linearization_error_dist, interval_r_dist): with a
// thrust-magnitude disturbance of every planar quadrotor of a chain (total
// thrust (u1 + u2) + thrust w_i), node i's column of E(x) is
// thrust dt/m (-sin theta_i, cos theta_i) on its (vx, vz) rows; over the tube
// set, r_dist lies in +-s with s = mag([E](Omega^x_k) - E_k) row-summed.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <mutex>

#include "leb.h"
#include "leb_internal.hpp"
#include "pbh_node.hpp"

namespace leb {

constexpr int SLS_MAX_NX = 32;
constexpr int SLS_MAX_NU = 16;
constexpr int SLS_MAX_NW = 64;
constexpr int SLS_THREADS = 256;
constexpr int SLS_PF = 8;                      // prefetch registers per thread (nx^2 + 2 nx nu <= 8 threads)
constexpr size_t SLS_ROW_LDS = 48 * 1024;      // LDS budget of a tube-row workgroup
constexpr size_t SLS_LDS_MAX = 64 * 1024;      // LDS of the one-launch fixed point (resident data + row region)

// ------------------------------------------------------------ responses

struct RiccatiArgs {
    const double* A; const double* B; const double* qx; const double* qu;
    double* K; double* phi;
    int nx, nu, N;
};

// NXC, NUC > 0: nx and nu fixed at compile time (the short dot products are
// then unrolled and their LDS loads issued together); 0: taken from a.
template <int NUB, int PF, int NXC = 0, int NUC = 0>
__global__ void __launch_bounds__(SLS_THREADS) sls_riccati_kernel(RiccatiArgs a) {
    const int j = blockIdx.x, b = blockIdx.y;
    const int nx = NXC ? NXC : a.nx, nu = NUC ? NUC : a.nu, N = a.N, n = nx + nu;
    if (j >= N - 1) return;                      // no k with j < k < N
    extern __shared__ double sm[];
    double* P = sm;                              // nx*nx   cost-to-go, then X of the forward pass
    double* Ak = P + nx * nx;                    // nx*nx
    double* PA = Ak + nx * nx;                   // nx*nx   P A_k, then X' of the forward pass
    double* Acl = PA + nx * nx;                  // nx*nx   A_k + B_k K
    double* Bk = Acl + nx * nx;                  // nx*nu
    double* PB = Bk + nx * nu;                   // nx*nu
    double* Bc = PB + nx * nu;                   // nu*nx
    double* Kk = Bc + nu * nx;                   // nu*nx
    double* L = Kk + nu * nx;                    // nu*nu   S, then its Cholesky factor
    double* sqx = L + nu * nu;                   // nx      diag(Q^x_{k,j})
    double* squ = sqx + nx;                      // nu      diag(Q^u_{k,j})
    __shared__ int bad;
    const int tid = threadIdx.x, nt = blockDim.x;
    const double* Ab = a.A + (size_t)b * N * nx * nx;
    const double* Bb = a.B + (size_t)b * N * nx * nu;
    const double* qxb = a.qx + (size_t)b * (N + 1) * N * nx;
    const double* qub = a.qu + (size_t)b * N * N * nu;
    double* Kb = a.K + (size_t)b * N * N * nu * nx;
    double* phib = a.phi + (size_t)b * N * N * n * nx;
    if (tid == 0) bad = 0;
    for (int q = tid; q < nx * nx; q += nt) {
        const int r = q / nx, c = q - r * nx;
        P[q] = r == c ? qxb[((size_t)N * N + j) * nx + r] : 0.0;
    }
    // a step's (A_k, B_k, weights) -- or (A_k, B_k, K_k) in the forward pass --
    // are loaded into registers two steps ahead (two buffers, the step loop
    // taken two at a time so each buffer has a fixed role) and stored to LDS
    // after the last barrier of the step before theirs
    double pfa[PF], pfb[PF];
    const int nab = nx * n;
    auto fetch = [&](int k, bool fwd, double* pf) {
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int q = tid + u * nt;
            double x = 0.0;
            if (q < nx * nx) x = Ab[(size_t)k * nx * nx + q];
            else if (q < nab) x = Bb[(size_t)k * nx * nu + (q - nx * nx)];
            else if (fwd) { if (q < nab + nu * nx) x = Kb[((size_t)k * N + j) * nu * nx + (q - nab)]; }
            else if (q < nab + nx) x = qxb[((size_t)k * N + j) * nx + (q - nab)];
            else if (q < nab + n) x = qub[((size_t)k * N + j) * nu + (q - nab - nx)];
            pf[u] = x;
        }
    };
    auto stash = [&](bool fwd, const double* pf) {
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int q = tid + u * nt;
            if (q < nx * nx) Ak[q] = pf[u];
            else if (q < nab) Bk[q - nx * nx] = pf[u];
            else if (fwd) { if (q < nab + nu * nx) Kk[q - nab] = pf[u]; }
            else if (q < nab + nx) sqx[q - nab] = pf[u];
            else if (q < nab + n) squ[q - nab - nx] = pf[u];
        }
    };
    fetch(N - 1, false, pfa);
    stash(false, pfa);
    if (N - 2 > j) fetch(N - 2, false, pfb);
    auto bstep = [&](int k, double* fb, const double* sb) {
        lds_barrier();
        if (k - 2 > j) fetch(k - 2, false, fb);
        // P A_k and P B_k
        for (int q = tid; q < nx * n; q += nt) {
            double s = 0.0;
            if (q < nx * nx) {
                const int r = q / nx, c = q - r * nx;
                for (int l = 0; l < nx; ++l) s = fma(P[r * nx + l], Ak[l * nx + c], s);
                PA[q] = s;
            } else {
                const int q2 = q - nx * nx, r = q2 / nu, c = q2 - r * nu;
                for (int l = 0; l < nx; ++l) s = fma(P[r * nx + l], Bk[l * nu + c], s);
                PB[q2] = s;
            }
        }
        lds_barrier();
        // S = diag(qu) + B^T (P B),  Bc = B^T (P A)
        for (int q = tid; q < nu * n; q += nt) {
            if (q < nu * nu) {
                const int r = q / nu, c = q - r * nu;
                double s = 0.0;
                for (int l = 0; l < nx; ++l) s = fma(Bk[l * nu + r], PB[l * nu + c], s);
                L[q] = (r == c ? squ[r] : 0.0) + s;
            } else {
                const int q2 = q - nu * nu, r = q2 / nx, c = q2 - r * nx;
                double s = 0.0;
                for (int l = 0; l < nx; ++l) s = fma(Bk[l * nu + r], PA[l * nx + c], s);
                Bc[q2] = s;
            }
        }
        lds_barrier();
        // Cholesky S = L L^T (lower triangle in place; diagonal holds 1/L_ii)
        if (tid == 0) {
            for (int c = 0; c < nu; ++c) {
                double d = L[c * nu + c];
                for (int m = 0; m < c; ++m) d -= L[c * nu + m] * L[c * nu + m];
                if (!(d > 0.0) || !isfinite(d)) { bad = 1; d = 1.0; }
                const double inv = 1.0 / sqrt(d);
                L[c * nu + c] = inv;
                for (int r = c + 1; r < nu; ++r) {
                    double s = L[r * nu + c];
                    for (int m = 0; m < c; ++m) s -= L[r * nu + m] * L[c * nu + m];
                    L[r * nu + c] = s * inv;
                }
            }
        }
        lds_barrier();
        // K = -S^-1 Bc, one column per thread: L y = Bc[:, c], then L^T x = y, in registers
        for (int c = tid; c < nx; c += nt) {
            double y[NUB];
#pragma unroll
            for (int r = 0; r < NUB; ++r) {
                if (r < nu) {
                    double s = Bc[r * nx + c];
#pragma unroll
                    for (int m = 0; m < r; ++m) s -= L[r * nu + m] * y[m];
                    y[r] = s * L[r * nu + r];
                }
            }
#pragma unroll
            for (int r = NUB - 1; r >= 0; --r) {
                if (r < nu) {
                    double s = y[r];
#pragma unroll
                    for (int m = r + 1; m < NUB; ++m)
                        if (m < nu) s -= L[m * nu + r] * y[m];
                    y[r] = s * L[r * nu + r];
                }
            }
#pragma unroll
            for (int r = 0; r < NUB; ++r)
                if (r < nu) Kk[r * nx + c] = bad ? NAN : -y[r];
        }
        lds_barrier();
        // P <- diag(qx) + A^T (P A) + K^T Bc; the gain goes out
        for (int q = tid; q < nx * nx; q += nt) {
            const int r = q / nx, c = q - r * nx;
            double s = 0.0;
            for (int l = 0; l < nx; ++l) s = fma(Ak[l * nx + r], PA[l * nx + c], s);
            double t = 0.0;
            for (int m = 0; m < nu; ++m) t = fma(Kk[m * nx + r], Bc[m * nx + c], t);
            P[q] = (r == c ? sqx[r] : 0.0) + s + t;
        }
        for (int q = tid; q < nu * nx; q += nt) Kb[((size_t)k * N + j) * nu * nx + q] = Kk[q];
        lds_barrier();
        if (k - 1 > j) stash(false, sb);
    };
    for (int k = N - 1; k > j; k -= 2) {
        bstep(k, pfa, pfb);
        if (k - 1 > j) bstep(k - 1, pfb, pfa);
    }
    // forward propagation from Phi^x_{j+1,j} = I; the gains were stored by this
    // workgroup above, and this full barrier orders those stores before the loads
    __syncthreads();
    double* X = P;
    double* Xn = PA;
    for (int q = tid; q < nx * nx; q += nt) X[q] = (q / nx == q % nx) ? 1.0 : 0.0;
    fetch(j + 1, true, pfa);
    stash(true, pfa);
    if (j + 2 < N) fetch(j + 2, true, pfb);
    auto fstep = [&](int k, double* fb, const double* sb) {
        lds_barrier();
        if (k + 2 < N) fetch(k + 2, true, fb);
        double* out = phib + ((size_t)k * N + j) * n * nx;
        for (int q = tid; q < n * nx; q += nt) {
            const int r = q / nx, c = q - r * nx;
            double s;
            if (r < nx) {
                s = X[q];
            } else {
                s = 0.0;
                for (int m = 0; m < nx; ++m) s = fma(Kk[(r - nx) * nx + m], X[m * nx + c], s);
            }
            out[q] = s;
        }
        for (int q = tid; q < nx * nx; q += nt) {
            const int r = q / nx, c = q - r * nx;
            double s = 0.0;
            for (int m = 0; m < nu; ++m) s = fma(Bk[r * nu + m], Kk[m * nx + c], s);
            Acl[q] = Ak[q] + s;
        }
        lds_barrier();
        if (k + 1 < N) {
            for (int q = tid; q < nx * nx; q += nt) {
                const int r = q / nx, c = q - r * nx;
                double s = 0.0;
                for (int l = 0; l < nx; ++l) s = fma(Acl[r * nx + l], X[l * nx + c], s);
                Xn[q] = s;
            }
            lds_barrier();
            double* t = X; X = Xn; Xn = t;
            stash(true, sb);
        }
    };
    for (int k = j + 1; k < N; k += 2) {
        fstep(k, pfa, pfb);
        if (k + 1 < N) fstep(k + 1, pfb, pfa);
    }
}

// The same recursions on FP64 MFMA (v_mfma_f64_16x16x4f64) for nx <= 16,
// nu <= 4: one wave per (trajectory, j), every matrix a zero-padded 16 x 16
// tile held in registers in the accumulator layout (lane l holds element
// [4i + l/16][l%16] of its tile, i = 0..3).  That layout is also the B operand
// of a product and, read as the A operand, the transpose, so every product
// takes the form X^T Y and stays in registers:
//   P A = P^T A and P B = P^T B (P is symmetric), S = B^T (P B),
//   Bc = B^T (P A), P' = diag(qx) + A^T (P A) + K^T Bc;
//   forward: K X = (K^T)^T X, (A + B K)^T = A^T + K^T B^T, X' = ((A + B K)^T)^T X,
// with A^T, B^T, K^T loaded straight into the accumulator layout.  Only S
// and Bc pass through LDS, for the nu x nu Cholesky factor and the column
// solves (lanes c < nx, each factoring S itself).
typedef double sls_d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ sls_d4 mm_tn(const sls_d4& X, const sls_d4& Y, sls_d4 acc) {   // acc + X^T Y
#pragma unroll
    for (int t = 0; t < 4; ++t) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(X[t], Y[t], acc, 0, 0, 0);
    return acc;
}

// M (R x C, leading dimension ld) in the accumulator layout; tr: M^T instead
__device__ __forceinline__ sls_d4 tile_load(const double* M, int R, int C, int ld, int lr, int lq, bool tr) {
    sls_d4 v;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int row = tr ? lr : 4 * i + lq, col = tr ? 4 * i + lq : lr;
        v[i] = (row < R && col < C) ? M[row * ld + col] : 0.0;
    }
    return v;
}

template <int NUB>
__global__ void __launch_bounds__(64) sls_riccati_mfma_kernel(RiccatiArgs a) {
    const int j = blockIdx.x, b = blockIdx.y;
    const int nx = a.nx, nu = a.nu, N = a.N, n = nx + nu;
    if (j >= N - 1) return;
    __shared__ double sS[NUB * NUB];
    __shared__ double sBc[NUB * 16];
    __shared__ double sK[16 * 16];
    const int lane = threadIdx.x, lr = lane & 15, lq = lane >> 4;
    const double* Ab = a.A + (size_t)b * N * nx * nx;
    const double* Bb = a.B + (size_t)b * N * nx * nu;
    const double* qxb = a.qx + (size_t)b * (N + 1) * N * nx;
    const double* qub = a.qu + (size_t)b * N * N * nu;
    double* Kb = a.K + (size_t)b * N * N * nu * nx;
    double* phib = a.phi + (size_t)b * N * N * n * nx;
    for (int q = lane; q < 256; q += 64) sK[q] = 0.0;          // rows >= nu stay 0
    // element of this lane on the diagonal (row 4i + lq == lr), if any
    const int di = (lr >= lq && ((lr - lq) & 3) == 0) ? (lr - lq) >> 2 : -1;
    sls_d4 P;
#pragma unroll
    for (int i = 0; i < 4; ++i) P[i] = (i == di && lr < nx) ? qxb[((size_t)N * N + j) * nx + lr] : 0.0;
    auto wts = [&](int k, double* qx_d, double* qu_d) {
        *qx_d = (di >= 0 && lr < nx) ? qxb[((size_t)k * N + j) * nx + lr] : 0.0;
        *qu_d = (di >= 0 && lr < nu) ? qub[((size_t)k * N + j) * nu + lr] : 0.0;
    };
    sls_d4 An = tile_load(Ab + (size_t)(N - 1) * nx * nx, nx, nx, nx, lr, lq, false);
    sls_d4 Bn = tile_load(Bb + (size_t)(N - 1) * nx * nu, nx, nu, nu, lr, lq, false);
    double qxn, qun;
    wts(N - 1, &qxn, &qun);
    const sls_d4 z4 = {0.0, 0.0, 0.0, 0.0};
    for (int k = N - 1; k > j; --k) {
        const sls_d4 A = An, B = Bn;
        const double qxd = qxn, qud = qun;
        if (k - 1 > j) {
            An = tile_load(Ab + (size_t)(k - 1) * nx * nx, nx, nx, nx, lr, lq, false);
            Bn = tile_load(Bb + (size_t)(k - 1) * nx * nu, nx, nu, nu, lr, lq, false);
            wts(k - 1, &qxn, &qun);
        }
        const sls_d4 PA = mm_tn(P, A, z4);
        const sls_d4 PB = mm_tn(P, B, z4);
        sls_d4 S = mm_tn(B, PB, z4);
        const sls_d4 Bc = mm_tn(B, PA, z4);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = 4 * i + lq;
            if (row < nu) {
                if (lr < nu) sS[row * NUB + lr] = S[i] + (i == di ? qud : 0.0);
                sBc[row * 16 + lr] = Bc[i];
            }
        }
        lds_barrier();
        if (lane < nx) {
            // S = L L^T (nu <= NUB) in registers, then L y = Bc[:, c], L^T x = y
            double L[NUB][NUB], inv[NUB];         // inv: 1 / L_cc, one division per pivot
            bool bad = false;
#pragma unroll
            for (int c = 0; c < NUB; ++c) {
                if (c < nu) {
                    double d = sS[c * NUB + c];
#pragma unroll
                    for (int m = 0; m < c; ++m) d -= L[c][m] * L[c][m];
                    if (!(d > 0.0) || !isfinite(d)) { bad = true; d = 1.0; }
                    inv[c] = 1.0 / sqrt(d);
#pragma unroll
                    for (int r = c + 1; r < NUB; ++r) {
                        if (r < nu) {
                            double t = sS[r * NUB + c];
#pragma unroll
                            for (int m = 0; m < c; ++m) t -= L[r][m] * L[c][m];
                            L[r][c] = t * inv[c];
                        }
                    }
                }
            }
            double y[NUB];
#pragma unroll
            for (int r = 0; r < NUB; ++r) {
                if (r < nu) {
                    double t = sBc[r * 16 + lane];
#pragma unroll
                    for (int m = 0; m < r; ++m) t -= L[r][m] * y[m];
                    y[r] = t * inv[r];
                }
            }
#pragma unroll
            for (int r = NUB - 1; r >= 0; --r) {
                if (r < nu) {
                    double t = y[r];
#pragma unroll
                    for (int m = r + 1; m < NUB; ++m)
                        if (m < nu) t -= L[m][r] * y[m];
                    y[r] = t * inv[r];
                }
            }
#pragma unroll
            for (int r = 0; r < NUB; ++r) {
                if (r < nu) {
                    const double kv = bad ? NAN : -y[r];
                    sK[r * 16 + lane] = kv;
                    Kb[((size_t)k * N + j) * nu * nx + r * nx + lane] = kv;
                }
            }
        }
        lds_barrier();
        sls_d4 K;
#pragma unroll
        for (int i = 0; i < 4; ++i) K[i] = sK[(4 * i + lq) * 16 + lr];
        sls_d4 Pn;
#pragma unroll
        for (int i = 0; i < 4; ++i) Pn[i] = i == di ? qxd : 0.0;
        Pn = mm_tn(A, PA, Pn);
        P = mm_tn(K, Bc, Pn);
        lds_barrier();                         // sS, sBc, sK are rewritten by the next step
    }
    // forward propagation from Phi^x_{j+1,j} = I; the gains were stored above
    // by this wave, and the full barrier orders those stores before the loads
    __syncthreads();
    sls_d4 X;
#pragma unroll
    for (int i = 0; i < 4; ++i) X[i] = (i == di && lr < nx) ? 1.0 : 0.0;
    auto fwd_load = [&](int k, sls_d4* AT, sls_d4* BT, sls_d4* Kt, sls_d4* KT) {
        const double* Kp = Kb + ((size_t)k * N + j) * nu * nx;
        *AT = tile_load(Ab + (size_t)k * nx * nx, nx, nx, nx, lr, lq, true);
        *BT = tile_load(Bb + (size_t)k * nx * nu, nx, nu, nu, lr, lq, true);
        *Kt = tile_load(Kp, nu, nx, nx, lr, lq, false);
        *KT = tile_load(Kp, nu, nx, nx, lr, lq, true);
    };
    sls_d4 ATn, BTn, Kn, KTn;
    fwd_load(j + 1, &ATn, &BTn, &Kn, &KTn);
    for (int k = j + 1; k < N; ++k) {
        const sls_d4 AT = ATn, BT = BTn, Kt = Kn, KT = KTn;
        if (k + 1 < N) fwd_load(k + 1, &ATn, &BTn, &Kn, &KTn);
        double* out = phib + ((size_t)k * N + j) * n * nx;
        const sls_d4 U = mm_tn(KT, X, z4);          // K X
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = 4 * i + lq;
            if (lr < nx) {
                if (row < nx) out[row * nx + lr] = X[i];
                if (row < nu) out[(nx + row) * nx + lr] = U[i];
            }
        }
        if (k + 1 < N) {
            const sls_d4 AclT = mm_tn(Kt, BT, AT);  // (A + B K)^T
            X = mm_tn(AclT, X, z4);                 // (A + B K) X
        }
    }
}

static size_t riccati_smem(int nx, int nu) {
    return sizeof(double) * (size_t)(4 * nx * nx + 4 * nx * nu + nu * nu + nx + nu);
}

// ------------------------------------------------------------ tube rows

struct TubeRowArgs {
    const double* phi;       // [b][N][N][n][nx]
    const double* E;         // [b][N][nx][nw]
    const double* cbar;      // [b][N][nx]
    const double* rbar;      // [b][N][nx]
    double* mu;              // [b][N][n]
    double* sigma;           // [b][N][n]
    const double* sigE;      // [b][N][n] the disturbance part of sigma (ROW_NOE reads it)
    int nx, nu, nw, N, jc;
};

// What a tube row sums: both parts of eq. tight_tube_width (ROW_FULL), only
// the disturbance part sum_j |Phi_{k,j} E_j| 1, which does not depend on the
// bounds (ROW_E), or the centre and the residual part, adding the disturbance
// part from sigE (ROW_NOE).
constexpr int ROW_FULL = 0, ROW_E = 1, ROW_NOE = 2;

// One trajectory's operands of tube row k (generic pointers: global or LDS).
struct RowRef {
    const double* phi;       // Phi_{k,0} (the row block of k)
    const double* E;         // E_0 (ROW_FULL, ROW_E)
    const double* cb;        // c_bar_0 (ROW_FULL, ROW_NOE)
    const double* rb;        // rho_bar_0
    const double* sigE;      // the disturbance part of row k, n values (ROW_NOE)
};

__device__ __forceinline__ RowRef row_ref(const TubeRowArgs& a, int b, int k) {
    const int nx = a.nx, n = nx + a.nu, N = a.N;
    RowRef r;
    r.phi = a.phi + (((size_t)b * N + k) * N) * n * nx;
    r.E = a.E ? a.E + (size_t)b * N * nx * a.nw : nullptr;
    r.cb = a.cbar ? a.cbar + (size_t)b * N * nx : nullptr;
    r.rb = a.rbar ? a.rbar + (size_t)b * N * nx : nullptr;
    r.sigE = a.sigE ? a.sigE + ((size_t)b * N + k) * n : nullptr;
    return r;
}

// Tube row k of trajectory b.  Thread t = jj * n + i works on row i of
// Phi_{k, j0 + jj}, which it loads straight into registers (every entry of
// Phi is used by one thread only); E_j, |E_j| 1, c_bar_j and rho_bar_j are
// shared through LDS, jc disturbance times per chunk.  NXB >= nx is the
// register length of a row.  Leaves the row's (mu, sigma) in mo[], so[] (LDS,
// n entries) after the final barrier.
template <int MODE, int NXB>
__device__ void tube_row(const TubeRowArgs& a, const RowRef& rr, int k, double* sm, double* mo, double* so) {
    const int nx = a.nx, nw = a.nw, n = nx + a.nu, jc = a.jc;
    const int tid = threadIdx.x, nt = blockDim.x;
    const bool useE = MODE != ROW_NOE, useR = MODE != ROW_E;
    double* sE = sm;                                          // jc*nx*nw   (useE)
    double* se1 = sE + (useE ? (size_t)jc * nx * nw : 0);     // jc*nx      (useE)
    double* scb = se1 + (useE ? jc * nx : 0);                 // jc*nx      (useR)
    double* srb = scb + (useR ? jc * nx : 0);                 // jc*nx      (useR)
    double* red = srb + (useR ? jc * nx : 0);                 // 3*jc*n
    const int jj = tid / n, i = tid - jj * n;
    const bool act = jj < jc;
    double am = 0.0, as = 0.0, ag = 0.0;
    const double* prow = rr.phi;
    for (int j0 = 0; j0 < k; j0 += jc) {
        const int cnt = min(jc, k - j0);
        const bool mine = act && jj < cnt;
        double r[NXB];
        if (mine) {
            const double* src = prow + ((size_t)(j0 + jj) * n + i) * nx;
#pragma unroll
            for (int l = 0; l < NXB; ++l) r[l] = l < nx ? src[l] : 0.0;
        }
        if (useE) {
            const double* ep = rr.E + (size_t)j0 * nx * nw;
            for (int q = tid; q < cnt * nx * nw; q += nt) sE[q] = ep[q];
        }
        if (useR) {
            const size_t ro = (size_t)j0 * nx;
            for (int q = tid; q < cnt * nx; q += nt) { scb[q] = rr.cb[ro + q]; srb[q] = rr.rb[ro + q]; }
        }
        lds_barrier();
        if (useE) {
            for (int q = tid; q < cnt * nx; q += nt) {
                double t = 0.0;
                for (int w = 0; w < nw; ++w) t += fabs(sE[q * nw + w]);
                se1[q] = t;
            }
            lds_barrier();
        }
        if (mine) {
            double m = 0.0, s = 0.0, g = 0.0;
            if (useR) {
                const double* cb = scb + jj * nx;
                const double* rb = srb + jj * nx;
#pragma unroll
                for (int l = 0; l < NXB; ++l) {
                    if (l < nx) {
                        const double ap = fabs(r[l]);
                        m = fma(r[l], cb[l], m);
                        s = fma(ap, rb[l], s);
                        g = fma(ap, fabs(cb[l]) + rb[l], g);
                    }
                }
            }
            if (useE) {
                const double* e1 = se1 + jj * nx;
                const double* Ej = sE + (size_t)jj * nx * nw;
#pragma unroll
                for (int l = 0; l < NXB; ++l)
                    if (l < nx) g = fma(fabs(r[l]), e1[l], g);
                for (int w = 0; w < nw; ++w) {
                    double t = 0.0;
#pragma unroll
                    for (int l = 0; l < NXB; ++l)
                        if (l < nx) t = fma(r[l], Ej[l * nw + w], t);
                    s += fabs(t);
                }
            }
            am += m; as += s; ag += g;
        }
        lds_barrier();
    }
    // partial sums over the disturbance-time slots: within each wave by a
    // butterfly over the lanes of one row (when n divides the wave and every
    // lane holds a slot), then over the waves; otherwise slot by slot
    const bool wave_red = (64 % n == 0) && (jc * n == nt);
    if (wave_red) {
        double m = am, s_ = as, g = ag;
        for (int msk = n; msk < 64; msk <<= 1) {
            m += __shfl_xor(m, msk);
            s_ += __shfl_xor(s_, msk);
            g += __shfl_xor(g, msk);
        }
        const int lane = tid & 63, wv = tid >> 6;
        if (lane < n) { red[(3 * wv) * n + lane] = m; red[(3 * wv + 1) * n + lane] = s_; red[(3 * wv + 2) * n + lane] = g; }
    } else if (act) {
        red[jj * n + i] = am; red[(jc + jj) * n + i] = as; red[(2 * jc + jj) * n + i] = ag;
    }
    lds_barrier();
    if (tid < n) {
        double m = 0.0, s = 0.0, g = 0.0;
        if (wave_red) {
            for (int w = 0; w < nt / 64; ++w) { m += red[(3 * w) * n + tid]; s += red[(3 * w + 1) * n + tid]; g += red[(3 * w + 2) * n + tid]; }
        } else {
            for (int q = 0; q < jc; ++q) { m += red[q * n + tid]; s += red[(jc + q) * n + tid]; g += red[(2 * jc + q) * n + tid]; }
        }
        // rounding of the sums: at most nx + k (nw + 1) + jc additions deep, each
        // within 2^-53 of the magnitudes g; doubled for the centre's error and the
        // final additions
        const double coef = (double)(nx + k * (nw + 1) + jc + 8) * 0x1p-52;
        s = s + coef * g * (1.0 + 0x1p-50) + 0x1p-1000;
        if (MODE == ROW_NOE) {
            const double se = rr.sigE[tid];
            s = s + se;
            s = s + fabs(s) * 0x1p-52;
            if (!isfinite(se)) g = INFINITY;
        }
        if (!isfinite(g) || !isfinite(s)) { m = 0.0; s = INFINITY; }
        if (k == 0) { m = 0.0; s = 0.0; }
        mo[tid] = MODE == ROW_E ? 0.0 : m;
        so[tid] = s;
    }
    __syncthreads();
}

static int tube_jc(int nx, int nu, int nw, int mode, size_t* smem, size_t budget = SLS_ROW_LDS) {
    const int n = nx + nu;
    const size_t per_j = sizeof(double) * ((mode != ROW_NOE ? (size_t)nx * nw + nx : 0) +
                                           (mode != ROW_E ? 2 * (size_t)nx : 0) + 3 * (size_t)n);
    int jc = SLS_THREADS / n;
    while (jc > 1 && per_j * jc + 2 * n * sizeof(double) > budget) --jc;
    *smem = per_j * jc;            // tube_row's region; callers add 2 n for the row results
    return jc;
}

// register length bucket of a row of Phi
static int nx_bucket(int nx) { return nx <= 8 ? 8 : (nx <= 16 ? 16 : 32); }

template <int MODE, int NXB>
__global__ void __launch_bounds__(SLS_THREADS) sls_tube_kernel(TubeRowArgs a, double* out_sig) {
    const int k = blockIdx.x, b = blockIdx.y;
    extern __shared__ double sm[];
    const int n = a.nx + a.nu;
    double* mo = sm;
    double* so = sm + n;
    tube_row<MODE, NXB>(a, row_ref(a, b, k), k, sm + 2 * n, mo, so);
    const size_t o = ((size_t)b * a.N + k) * n;
    for (int q = threadIdx.x; q < n; q += blockDim.x) {
        if (MODE == ROW_E) {
            out_sig[o + q] = so[q];
        } else {
            a.mu[o + q] = mo[q];
            a.sigma[o + q] = so[q];
        }
    }
}

// The disturbance part sum_j |Phi_{k,j} E_j| 1 of tube row k on FP64 MFMA for
// 8 < n <= 16, nw <= 16 (smaller blocks stay on the VALU row): one workgroup per (trajectory, k), wave w takes the blocks
// j = w, w + 4, ...  Each block is one zero-padded 16 x 16 x 16 product
// (A fragments from Phi_{k,j}, B fragments from E_j, both straight from
// memory); the accumulator's entries are added up in absolute value over j,
// and |Phi| |E| is accumulated beside it for the rounding allowance.  The
// sixteen columns of each row are summed at the end.
__global__ void __launch_bounds__(256) sls_tube_e_mfma_kernel(TubeRowArgs a, double* out_sig) {
    const int k = blockIdx.x, b = blockIdx.y;
    const int nx = a.nx, nw = a.nw, N = a.N, n = nx + a.nu;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, lr = lane & 15, lq = lane >> 4;
    __shared__ double red[2][4][4][64];
    __shared__ double rows[2][16];
    sls_d4 T = {0.0, 0.0, 0.0, 0.0}, G = {0.0, 0.0, 0.0, 0.0};
    const double* prow = a.phi + (((size_t)b * N + k) * N) * n * nx;
    const double* Eb = a.E + (size_t)b * N * nx * nw;
    // fragments of block j: A[l%16][4t + l/16] from Phi_{k,j}, B[4t + l/16][l%16] from E_j;
    // the next block's are loaded while this one multiplies
    double an[4], bn[4];
    auto frag = [&](int j) {
        const double* Pj = prow + (size_t)j * n * nx;
        const double* Ej = Eb + (size_t)j * nx * nw;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int kk = 4 * t + lq;
            an[t] = (lr < n && kk < nx) ? Pj[lr * nx + kk] : 0.0;
            bn[t] = (kk < nx && lr < nw) ? Ej[kk * nw + lr] : 0.0;
        }
    };
    if (wave < k) frag(wave);
    for (int j = wave; j < k; j += 4) {
        double av[4], bv[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) { av[t] = an[t]; bv[t] = bn[t]; }
        if (j + 4 < k) frag(j + 4);
        sls_d4 D = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            D = __builtin_amdgcn_mfma_f64_16x16x4f64(av[t], bv[t], D, 0, 0, 0);
            G = __builtin_amdgcn_mfma_f64_16x16x4f64(fabs(av[t]), fabs(bv[t]), G, 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) T[i] += fabs(D[i]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) { red[0][wave][i][lane] = T[i]; red[1][wave][i][lane] = G[i]; }
    __syncthreads();
    if (tid < 32) {
        // row r = 4 i + lq' of the tile: the 16 lanes lr of group lq', element i, all waves
        const int which = tid >> 4, r = tid & 15, i = r >> 2, lqr = r & 3;
        double acc = 0.0;
        for (int w = 0; w < 4; ++w)
            for (int c = 0; c < 16; ++c) acc += red[which][w][i][lqr * 16 + c];
        rows[which][r] = acc;
    }
    __syncthreads();
    if (tid < n) {
        double sv = rows[0][tid];
        const double g = rows[1][tid];
        // depth of the sums: nx products per entry inside the MFMA, k blocks, 4 waves, 16 columns
        const double coef = (double)(nx + k * (nw + 1) + 64) * 0x1p-52;
        sv = sv + coef * g * (1.0 + 0x1p-50) + 0x1p-1000;
        if (!isfinite(g) || !isfinite(sv)) sv = INFINITY;
        if (k == 0) sv = 0.0;
        out_sig[((size_t)b * N + k) * n + tid] = sv;
    }
}

template <int MODE>
static void launch_tube(const TubeRowArgs& a, int batch, double* out_sig, hipStream_t s) {
    size_t smem;
    TubeRowArgs t = a;
    t.jc = tube_jc(a.nx, a.nu, a.nw, MODE, &smem);
    smem += 2 * (a.nx + a.nu) * sizeof(double);
    const dim3 grid((unsigned)a.N, (unsigned)batch);
    switch (nx_bucket(a.nx)) {
    case 8: hipLaunchKernelGGL((sls_tube_kernel<MODE, 8>), grid, dim3(SLS_THREADS), smem, s, t, out_sig); break;
    case 16: hipLaunchKernelGGL((sls_tube_kernel<MODE, 16>), grid, dim3(SLS_THREADS), smem, s, t, out_sig); break;
    default: hipLaunchKernelGGL((sls_tube_kernel<MODE, 32>), grid, dim3(SLS_THREADS), smem, s, t, out_sig); break;
    }
}

// ------------------------------------------------------------ disturbance error

// FP64 interval sine and cosine of [lo, hi]: library values widened by 2^-40
// relative plus 2^-100 absolute, +-1 where a critical point may lie inside
// (tested against an outward pi).
__device__ void sls_sincos(double lo, double hi, double* sl, double* sh, double* cl, double* ch) {
    const double PI_LO = 3.141592653589793115997963468544185161590576171875;
    const double PI_HI = 3.141592653589793560087173318606801331043243408203125;
    if (!(hi - lo < 2.0 * PI_LO) || fabs(lo) > 1024.0 || fabs(hi) > 1024.0) {
        *sl = -1.0; *sh = 1.0; *cl = -1.0; *ch = 1.0;
        return;
    }
    const double sa = sin(lo), sb = sin(hi), ca = cos(lo), cb = cos(hi);
    auto wdn = [](double x) { return x - fabs(x) * 0x1p-40 - 0x1p-100; };
    auto wup = [](double x) { return x + fabs(x) * 0x1p-40 + 0x1p-100; };
    double s0 = wdn(fmin(sa, sb)), s1 = wup(fmax(sa, sb));
    double c0 = wdn(fmin(ca, cb)), c1 = wup(fmax(ca, cb));
    auto may = [&](double frac) {
        const double x0 = frac * PI_LO;
        const double m = ceil((lo - x0) / (2.0 * PI_HI) - 1e-12);
        const double crit = x0 + m * 2.0 * (m >= 0 ? PI_LO : PI_HI);
        return crit <= hi + 1e-12;
    };
    if (may(0.5)) s1 = 1.0;
    if (may(-0.5)) s0 = -1.0;
    if (may(0.0)) c1 = 1.0;
    if (may(1.0)) c0 = -1.0;
    *sl = fmax(s0, -1.0); *sh = fmin(s1, 1.0);
    *cl = fmax(c0, -1.0); *ch = fmin(c1, 1.0);
}

__device__ __forceinline__ double rdn(double x) { return x - fabs(x) * 0x1p-52 - 0x1p-1000; }
__device__ __forceinline__ double rup(double x) { return x + fabs(x) * 0x1p-52 + 0x1p-1000; }

// half-width of the thrust columns' disturbance error on row l (0 off the (vx, vz) rows)
__device__ double thrust_rdist(int l, double zt, double mut, double sgt, double e0, double c) {
    const int comp = l % 6;
    if (comp != 3 && comp != 4) return 0.0;
    const double lo = rdn(zt + mut - sgt), hi = rup(zt + mut + sgt);
    if (!(lo <= hi) || !isfinite(lo) || !isfinite(hi)) return INFINITY;
    double sl, sh, cl, ch;
    sls_sincos(lo, hi, &sl, &sh, &cl, &ch);
    // vx: -c [sin], vz: c [cos]; products of the point c >= 0 rounded outward
    const double a = comp == 3 ? rdn(-c * sh) : rdn(c * cl);
    const double bq = comp == 3 ? rup(-c * sl) : rup(c * ch);
    return rup(fmax(fabs(rup(bq - e0)), fabs(rdn(a - e0))));
}

struct EDiag { double e[SLS_MAX_NX]; };

// E(z_k) = [diag(e) | thrust columns], [units][nx][nx + U]
__global__ void sls_disturbance_kernel(const double* z, EDiag e, double c, int nx, int U, int64_t units,
                                       double* E) {
    const int nw = nx + U;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= units * nx * nw) return;
    const int64_t u = q / ((int64_t)nx * nw);
    const int r = (int)((q / nw) % nx), w = (int)(q % nw);
    double val = 0.0;
    if (w < nx) val = w == r ? e.e[r] : 0.0;
    else {
        const int i = w - nx;
        const double th = z[u * nx + 6 * i + 2];
        if (r == 6 * i + 3) val = -c * sin(th);
        else if (r == 6 * i + 4) val = c * cos(th);
    }
    E[q] = val;
}

// ------------------------------------------------------------ fixed point

struct FpRowArgs {
    TubeRowArgs t;           // cbar, rbar: workspace (written here through cbar_w, rbar_w)
    double* cbar_w; double* rbar_w;
    const double* z; const double* v;
    const double* rlo_s; const double* rhi_s;   // [b][nx] bound of step k-1 (staging)
    double* zs; double* vs; double* mus; double* sgs;   // staging for the bound of step k
    double* r_lo; double* r_hi;                  // [b][N][nx] outputs (may be NULL)
    uint32_t* certified;                         // [b] (may be NULL)
    double thrust_c;                             // thrust dt / m (0: constant E)
    double pad;
    int U;
};

// Row launch of step k (k = N: only finishes step N-1).  One workgroup per trajectory.
template <int NXB>
__global__ void __launch_bounds__(SLS_THREADS) sls_fp_row_kernel(FpRowArgs a, int k) {
    const int b = blockIdx.x;
    const TubeRowArgs& t = a.t;
    const int nx = t.nx, nu = t.nu, n = nx + nu, N = t.N, nw = t.nw;
    extern __shared__ double sm[];
    double* mo = sm;
    double* so = sm + n;
    const int tid = threadIdx.x;
    if (k > 0) {
        // residual zonotope of step k-1: bound + disturbance error, outward
        const int kp = k - 1;
        for (int l = tid; l < nx; l += blockDim.x) {
            double lo = a.rlo_s[(size_t)b * nx + l], hi = a.rhi_s[(size_t)b * nx + l];
            if (a.thrust_c > 0.0) {
                const int node = l / 6, th = 6 * node + 2;
                const size_t ob = ((size_t)b * N + kp);
                const double e0 = t.E[(ob * nx + l) * nw + (nw - a.U + node)];
                const double s = thrust_rdist(l, a.z[ob * nx + th], t.mu[ob * n + th], t.sigma[ob * n + th], e0,
                                              a.thrust_c);
                if (s != 0.0) {
                    lo = rdn(lo - s);
                    hi = rup(hi + s);
                }
            }
            const size_t o = ((size_t)b * N + kp) * nx + l;
            if (a.r_lo) { a.r_lo[o] = lo; a.r_hi[o] = hi; }
            double cb = 0.5 * (lo + hi), rb = fmax(hi - cb, cb - lo);
            rb = rup(rup(rb) + a.pad);
            if (!isfinite(lo) || !isfinite(hi)) { cb = NAN; rb = INFINITY; }
            a.cbar_w[o] = cb;
            a.rbar_w[o] = rb;
        }
        __syncthreads();
    }
    if (k == N) {
        if (a.certified && tid == 0) {
            // every tube entry and residual finite: the causal pass reached C = F(C)
            bool fin = true;
            for (int q = 0; q < N * n && fin; ++q) fin = isfinite(t.sigma[(size_t)b * N * n + q]);
            for (int q = 0; q < N * nx && fin; ++q) fin = isfinite(t.rbar[(size_t)b * N * nx + q]);
            a.certified[b] = fin ? 1u : 0u;
        }
        return;
    }
    tube_row<ROW_NOE, NXB>(t, row_ref(t, b, k), k, sm + 2 * n, mo, so);
    const size_t o = ((size_t)b * N + k) * n;
    for (int q = tid; q < n; q += blockDim.x) {
        t.mu[o + q] = mo[q];
        t.sigma[o + q] = so[q];
        a.mus[(size_t)b * n + q] = mo[q];
        a.sgs[(size_t)b * n + q] = so[q];
    }
    const size_t ob = (size_t)b * N + k;
    for (int q = tid; q < nx; q += blockDim.x) a.zs[(size_t)b * nx + q] = a.z[ob * nx + q];
    for (int q = tid; q < nu; q += blockDim.x) a.vs[(size_t)b * nu + q] = a.v[ob * nu + q];
}

// Chain dynamics: the whole causal pass of one trajectory in one workgroup.
// Step k: tube row k, then the path-based bound of the unit (z_k, v_k) +
// mu_k +- sigma_k by the chain bound's node pass (U of the 256 lanes; the
// tube row sits in LDS and the bound writes its rows to LDS), then the
// residual zonotope of step k for the later rows.
struct FpChainArgs {
    TubeRowArgs t;
    double* cbar_w; double* rbar_w;
    const double* z; const double* v;
    double* r_lo; double* r_hi;
    uint32_t* certified;
    double thrust_c;
    // node-pass constants
    int U;
    double c, kL, L0, pad;
    int compact;
};

__device__ __forceinline__ void residual_row(int l, double lo, double hi, double zt, double mut, double sgt,
                                             double e0, double thrust_c, double pad, double* cb, double* rb,
                                             double* lo_o, double* hi_o) {
    if (thrust_c > 0.0) {
        const double s = thrust_rdist(l, zt, mut, sgt, e0, thrust_c);
        if (s != 0.0) {
            lo = rdn(lo - s);
            hi = rup(hi + s);
        }
    }
    *lo_o = lo;
    *hi_o = hi;
    double c = 0.5 * (lo + hi), r = fmax(hi - c, c - lo);
    r = rup(rup(r) + pad);
    if (!isfinite(lo) || !isfinite(hi)) { c = NAN; r = INFINITY; }
    *cb = c;
    *rb = r;
}

template <int NXB>
__global__ void __launch_bounds__(SLS_THREADS) sls_fp_chain_kernel(FpChainArgs a) {
    const int b = blockIdx.x;
    const TubeRowArgs& t = a.t;
    const int nx = t.nx, nu = t.nu, n = nx + nu, N = t.N, nw = t.nw, U = a.U;
    extern __shared__ double sm[];
    // the trajectory's nominal, disturbance parts, thrust entries and residual
    // zonotopes stay in LDS for the whole pass
    double* mo = sm;                    // n
    double* so = mo + n;                // n
    double* rl = so + n;                // nx
    double* rh = rl + nx;               // nx
    double* zl = rh + nx;               // N*nx
    double* vl = zl + (size_t)N * nx;   // N*nu
    double* sel = vl + (size_t)N * nu;  // N*n
    double* eth = sel + (size_t)N * n;  // N*nx  E_k entry of row l's thrust column (0 off the thrust rows)
    double* cbl = eth + (size_t)N * nx; // N*nx
    double* rbl = cbl + (size_t)N * nx; // N*nx
    SpringOut* s_sp = reinterpret_cast<SpringOut*>(rbl + (size_t)N * nx);      // [U]
    uint32_t* s_flag = reinterpret_cast<uint32_t*>(s_sp + U);                   // [2]: flags, all finite
    const size_t off = ((reinterpret_cast<uintptr_t>(s_flag + 2) - reinterpret_cast<uintptr_t>(sm)) + 15) & ~size_t(15);
    double* region = reinterpret_cast<double*>(reinterpret_cast<unsigned char*>(sm) + off);
    const int tid = threadIdx.x, bs = blockDim.x;
    const int lt = tid / U, i = tid - lt * U;
    const size_t b0 = (size_t)b * N;
    for (int q = tid; q < N * nx; q += bs) {
        zl[q] = a.z[b0 * nx + q];
        const int k = q / nx, l = q - k * nx, comp = l % 6;
        eth[q] = (a.thrust_c > 0.0 && (comp == 3 || comp == 4)) ? t.E[((b0 + k) * nx + l) * nw + (nw - U + l / 6)] : 0.0;
    }
    for (int q = tid; q < N * nu; q += bs) vl[q] = a.v[b0 * nu + q];
    for (int q = tid; q < N * n; q += bs) sel[q] = t.sigE[b0 * n + q];
    if (tid == 0) s_flag[1] = 1u;
    __syncthreads();
    RowRef rr;
    rr.E = nullptr; rr.cb = cbl; rr.rb = rbl;
    for (int k = 0; k < N; ++k) {
        rr.phi = t.phi + ((b0 + k) * N) * n * nx;
        rr.sigE = sel + (size_t)k * n;
        tube_row<ROW_NOE, NXB>(t, rr, k, region, mo, so);
        for (int q = tid; q < n; q += bs) {
            t.mu[(b0 + k) * n + q] = mo[q];
            t.sigma[(b0 + k) * n + q] = so[q];
            if (!isfinite(so[q])) s_flag[1] = 0u;
        }
        if (tid == 0) s_flag[0] = 0u;
        const TileRef t0{zl + (size_t)k * nx, vl + (size_t)k * nu, mo, so, rl, rh, nullptr, nullptr, nullptr, 1};
        NodeIn d;
        node_load(t0, U, lt, i, d);
        lds_barrier();                        // s_flag cleared
        node_pass(a, t0, d, lt, i, s_sp, s_flag);
        lds_barrier();                        // the unit's rows are in rl, rh
        for (int l = tid; l < nx; l += bs) {
            const int th = 6 * (l / 6) + 2;
            double lo, hi;
            residual_row(l, rl[l], rh[l], zl[(size_t)k * nx + th], mo[th], so[th], eth[(size_t)k * nx + l],
                         a.thrust_c, a.pad, &cbl[(size_t)k * nx + l], &rbl[(size_t)k * nx + l], &lo, &hi);
            if (!isfinite(rbl[(size_t)k * nx + l])) s_flag[1] = 0u;
            if (a.r_lo) { a.r_lo[(b0 + k) * nx + l] = lo; a.r_hi[(b0 + k) * nx + l] = hi; }
        }
        lds_barrier();                        // residual of step k in LDS for the later rows
    }
    if (a.certified && tid == 0) a.certified[b] = s_flag[1];
}

// LDS bytes of the resident part of sls_fp_chain_kernel (before its tube-row region)
static size_t fp_chain_head_bytes(int nx, int nu, int U, int N) {
    const int n = nx + nu;
    const size_t b = sizeof(double) * ((size_t)2 * n + 2 * nx + (size_t)N * (nx + nu + n + 3 * nx)) +
                     sizeof(SpringOut) * U + 2 * sizeof(uint32_t);
    return (b + 15) & ~size_t(15);
}

struct SlsWorkspace {
    std::mutex mu;
    double* buf = nullptr;
    size_t cap = 0;
    WsFence fence;
};
static SlsWorkspace g_sls;

static bool dims_ok(int nx, int nu) { return nx >= 1 && nx <= SLS_MAX_NX && nu >= 0 && nu <= SLS_MAX_NU; }

}  // namespace leb

using namespace leb;

extern "C" int leb_sls_responses(int32_t nx, int32_t nu, int32_t batch, int32_t N, const double* A, const double* B,
                                 const double* qx, const double* qu, double* K, double* phi, void* stream) {
    if (!dims_ok(nx, nu) || nu < 1 || batch < 0 || N < 0) return LEB_EINVAL;
    if (batch > 65535 || N > 65535) return LEB_ENOTSUP;
    if ((int64_t)batch * N * N == 0) return LEB_OK;
    if (!A || !B || !qx || !qu || !K || !phi) return LEB_EINVAL;
    const void* ptrs[] = {A, B, qx, qu, K, phi};
    for (const void* p : ptrs)
        if (!aligned8(p)) return LEB_EINVAL;
    RiccatiArgs a;
    a.A = A; a.B = B; a.qx = qx; a.qu = qu; a.K = K; a.phi = phi;
    a.nx = nx; a.nu = nu; a.N = N;
    const int threads = min(SLS_THREADS, 64 * ((nx * nx + 63) / 64));
    // registers per thread that hold one step's prefetch
    const int step = max(nx * nx + 2 * nx * nu, nx * (nx + nu) + nx + nu);
    const bool small = nu <= 4 && step <= 2 * threads;
    if (!small && step > SLS_PF * threads) return LEB_ENOTSUP;
    const dim3 grid((unsigned)N, (unsigned)batch);
    const size_t sm = riccati_smem(nx, nu);
    hipStream_t st = (hipStream_t)stream;
    if (nx > 8 && nx <= 16 && nu <= 4)
        hipLaunchKernelGGL((sls_riccati_mfma_kernel<4>), grid, dim3(64), 0, st, a);
    else if (nx == 6 && nu == 2 && threads == 64)
        hipLaunchKernelGGL((sls_riccati_kernel<4, 2, 6, 2>), grid, dim3(threads), sm, st, a);
    else if (small)
        hipLaunchKernelGGL((sls_riccati_kernel<4, 2>), grid, dim3(threads), sm, st, a);
    else
        hipLaunchKernelGGL((sls_riccati_kernel<SLS_MAX_NU, SLS_PF>), grid, dim3(threads), sm, st, a);
    return hipGetLastError() == hipSuccess ? LEB_OK : LEB_EDEVICE;
}

extern "C" int leb_sls_tube_map(int32_t nx, int32_t nu, int32_t nw, int32_t batch, int32_t N, const double* phi,
                                const double* E, const double* c_bar, const double* rho_bar, double* mu,
                                double* sigma, void* stream) {
    if (!dims_ok(nx, nu) || nw < 0 || nw > SLS_MAX_NW || batch < 0 || N < 0) return LEB_EINVAL;
    if (batch > 65535 || N > 65535) return LEB_ENOTSUP;
    if ((int64_t)batch * N == 0) return LEB_OK;
    if (!phi || (nw > 0 && !E) || !c_bar || !rho_bar || !mu || !sigma) return LEB_EINVAL;
    const void* ptrs[] = {phi, E, c_bar, rho_bar, mu, sigma};
    for (const void* p : ptrs)
        if (p && !aligned8(p)) return LEB_EINVAL;
    TubeRowArgs a;
    a.phi = phi; a.E = E; a.cbar = c_bar; a.rbar = rho_bar; a.mu = mu; a.sigma = sigma; a.sigE = nullptr;
    a.nx = nx; a.nu = nu; a.nw = nw; a.N = N;
    launch_tube<ROW_FULL>(a, batch, nullptr, (hipStream_t)stream);
    return hipGetLastError() == hipSuccess ? LEB_OK : LEB_EDEVICE;
}

extern "C" int leb_linearize(const leb_dynamics* dyn, int32_t batch, int32_t N, const double* z, const double* v,
                             const double* e, double thrust, double* A, double* B, double* E, void* stream) {
    int rc = check_dynamics(dyn);
    if (rc != LEB_OK) return rc;
    if (dyn->kind != LEB_DYN_PQUAD_CHAIN) return LEB_ENOTSUP;
    if (batch < 0 || N < 0 || !(thrust >= 0.0) || !isfinite(thrust)) return LEB_EINVAL;
    const int64_t units = (int64_t)batch * N;
    if (units == 0) return LEB_OK;
    if (!z || !v || !A || !B || (E && !e)) return LEB_EINVAL;
    const void* ptrs[] = {z, v, A, B, E};
    for (const void* p : ptrs)
        if (p && !aligned8(p)) return LEB_EINVAL;
    const int nx = dyn->nx, U = dyn->n_units;
    if (units * nx * (nx + dyn->nu + nx + U) > ((int64_t)1 << 46)) return LEB_EINVAL;
    EDiag ed;
    if (E) {
        if (nx > SLS_MAX_NX) return LEB_ENOTSUP;
        for (int i = 0; i < nx; ++i) {
            if (!(e[i] >= 0.0) || !isfinite(e[i])) return LEB_EINVAL;
            ed.e[i] = e[i];
        }
    }
    hipStream_t s = (hipStream_t)stream;
    if ((rc = launch_chain_jacobians(dyn, units, z, v, A, B, s))) return rc;
    if (!E) return LEB_OK;
    const int64_t cnt = units * nx * (nx + U);
    hipLaunchKernelGGL(sls_disturbance_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, z, ed,
                       thrust * dyn->dt / dyn->m, nx, U, units, E);
    return hipGetLastError() == hipSuccess ? LEB_OK : LEB_EDEVICE;
}

extern "C" int leb_sls_fixed_point(const leb_dynamics* dyn, int32_t batch, int32_t N, const double* z,
                                   const double* v, const double* phi, int32_t nw, const double* E, double thrust,
                                   double pad, double* mu, double* sigma, double* r_lo, double* r_hi,
                                   uint32_t* certified, void* stream) {
    int rc = check_dynamics(dyn);
    if (rc != LEB_OK) return rc;
    const int nx = dyn->nx, nu = dyn->nu, n = nx + nu;
    if (!dims_ok(nx, nu) || nw < 0 || nw > SLS_MAX_NW || batch < 0 || N < 0) return LEB_EINVAL;
    if (!(pad >= 0.0) || !isfinite(pad) || !(thrust >= 0.0) || !isfinite(thrust)) return LEB_EINVAL;
    const bool chain = dyn->kind == LEB_DYN_PQUAD_CHAIN;
    if (dyn->kind == LEB_DYN_LINEAR || dyn->kind == LEB_DYN_QUADRATIC || dyn->kind == LEB_DYN_SINCOS)
        return LEB_ENOTSUP;
    if (thrust > 0.0 && (!chain || nw < dyn->n_units)) return LEB_EINVAL;
    if (batch > 65535) return LEB_ENOTSUP;
    if ((int64_t)batch * N == 0) return LEB_OK;
    if (!z || (nu > 0 && !v) || !phi || (nw > 0 && !E) || !mu || !sigma || (!r_lo != !r_hi)) return LEB_EINVAL;
    const void* ptrs[] = {z, v, phi, E, mu, sigma, r_lo, r_hi};
    for (const void* p : ptrs)
        if (p && !aligned8(p)) return LEB_EINVAL;
    if (certified && (reinterpret_cast<uintptr_t>(certified) & 3u)) return LEB_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lock(g_sls.mu);
    // cbar, rbar [b][N][nx]; sigE [b][N][n]; staging zs [b][nx], vs [b][nu], mus, sgs [b][n], rlo_s, rhi_s [b][nx]
    const size_t need = (size_t)batch * (2 * (size_t)N * nx + (size_t)N * n + nx + nu + 2 * n + 2 * nx) + 1;
    if (need > g_sls.cap) {
        if (g_sls.buf) (void)hipFree(g_sls.buf);
        g_sls.buf = nullptr;
        g_sls.cap = 0;
        if (hipMalloc(&g_sls.buf, need * sizeof(double)) != hipSuccess) return LEB_ENOMEM;
        g_sls.cap = need;
    }
    if ((rc = g_sls.fence.enter(s))) return rc;
    WsFenceScope leave{g_sls.fence, s};
    double* p = g_sls.buf;
    auto take = [&](size_t cnt) { double* q = p; p += cnt; return q; };
    FpRowArgs a;
    a.t.phi = phi; a.t.E = E; a.t.mu = mu; a.t.sigma = sigma;
    a.cbar_w = take((size_t)batch * N * nx);
    a.rbar_w = take((size_t)batch * N * nx);
    a.t.cbar = a.cbar_w;
    a.t.rbar = a.rbar_w;
    a.t.nx = nx; a.t.nu = nu; a.t.nw = nw; a.t.N = N;
    // the disturbance part of every tube entry first: it does not depend on the bounds,
    // so it runs over all (trajectory, step) rows at once
    double* sigE = take((size_t)batch * N * n);
    a.t.sigE = sigE;
    if (n > 8 && n <= 16 && nw <= 16 && nw > 0)
        hipLaunchKernelGGL(sls_tube_e_mfma_kernel, dim3((unsigned)N, (unsigned)batch), dim3(256), 0, s, a.t, sigE);
    else
        launch_tube<ROW_E>(a.t, batch, sigE, s);
    size_t smem;
    a.t.jc = tube_jc(nx, nu, nw, ROW_NOE, &smem);
    smem += 2 * n * sizeof(double);
    const int nxb = nx_bucket(nx);
    a.zs = take((size_t)batch * nx);
    a.vs = take((size_t)batch * nu);
    a.mus = take((size_t)batch * n);
    a.sgs = take((size_t)batch * n);
    double* rlo_s = take((size_t)batch * nx);
    double* rhi_s = take((size_t)batch * nx);
    a.rlo_s = rlo_s; a.rhi_s = rhi_s;
    a.z = z; a.v = v; a.r_lo = r_lo; a.r_hi = r_hi; a.certified = certified;
    a.thrust_c = thrust > 0.0 ? thrust * dyn->dt / dyn->m : 0.0;
    a.pad = pad;
    a.U = chain ? dyn->n_units : 0;
    // chains whose trajectory data fits in LDS beside a tube-row region: the whole
    // causal pass in one launch (one workgroup per trajectory)
    const size_t head = chain ? fp_chain_head_bytes(nx, nu, dyn->n_units, N) : 0;
    size_t region = 0;
    int jc_res = 0;
    if (chain && head < SLS_LDS_MAX) {
        jc_res = tube_jc(nx, nu, nw, ROW_NOE, &region, SLS_LDS_MAX - head);
        if (head + region > SLS_LDS_MAX) jc_res = 0;
    }
    if (jc_res > 0) {
        FpChainArgs c;
        c.t = a.t;
        c.t.jc = jc_res;
        c.cbar_w = a.cbar_w; c.rbar_w = a.rbar_w;
        c.z = z; c.v = v; c.r_lo = r_lo; c.r_hi = r_hi; c.certified = certified;
        c.thrust_c = a.thrust_c;
        c.U = dyn->n_units;
        c.c = dyn->dt / dyn->m; c.kL = dyn->k_spring * dyn->rest_len; c.L0 = dyn->rest_len; c.pad = pad;
        c.compact = 0;
        const dim3 g((unsigned)batch), bl(SLS_THREADS);
        if (nxb == 8) hipLaunchKernelGGL(sls_fp_chain_kernel<8>, g, bl, head + region, s, c);
        else if (nxb == 16) hipLaunchKernelGGL(sls_fp_chain_kernel<16>, g, bl, head + region, s, c);
        else hipLaunchKernelGGL(sls_fp_chain_kernel<32>, g, bl, head + region, s, c);
        return hipGetLastError() == hipSuccess ? LEB_OK : LEB_EDEVICE;
    }
    // otherwise one row launch and one bound launch per step
    for (int k = 0; k <= N; ++k) {
        const dim3 g((unsigned)batch), bl(SLS_THREADS);
        if (nxb == 8) hipLaunchKernelGGL(sls_fp_row_kernel<8>, g, bl, smem, s, a, k);
        else if (nxb == 16) hipLaunchKernelGGL(sls_fp_row_kernel<16>, g, bl, smem, s, a, k);
        else hipLaunchKernelGGL(sls_fp_row_kernel<32>, g, bl, smem, s, a, k);
        if (k == N) break;
        rc = chain ? launch_pbh_chain(dyn, batch, a.zs, a.vs, a.mus, a.sgs, rlo_s, rhi_s, nullptr, nullptr, 0.0,
                                      nullptr, s)
                   : launch_small_dyn(dyn, LEB_IH_PATH, batch, a.zs, a.vs, a.mus, a.sgs, rlo_s, rhi_s, nullptr,
                                      nullptr, 0.0, nullptr, s);
        if (rc) return rc;
    }
    return hipGetLastError() == hipSuccess ? LEB_OK : LEB_EDEVICE;
}
