// mlp.hip -- BF16 MFMA kernels of the learned warm-start MLP: fused
// forward, GEMM-based backward, MSE, Adam.
//
// Network: widths [d_0, ..., d_L], GELU after every hidden layer, FP32
// master parameters, BF16 operands with FP32 accumulation:
//   a_0 = bf16(x);  z_l = bf16(W_l) a_{l-1} + b_l;  a_l = bf16(gelu(z_l));
//   y = bf16(W_L) a_{L-1} + b_L.
// Backward (of sum(dy . y)): g_L = bf16(dy); dW_l = sum_b g_l a_{l-1}^T;
//   db_l = sum_b dz_l; dz_{l-1} = (bf16(W_l)^T g_l) gelu'(z_{l-1});
//   g_{l-1} = bf16(dz_{l-1}).
// Adam (Kingma and Ba, Algorithm 1) updates the FP32 parameters, then the
// BF16 copies are refreshed.  gelu(z) = z Phi(z) is evaluated in FP32 with
// a published approximation of erf (below), well inside BF16 rounding.
//
// MFMA: v_mfma_f32_16x16x32_bf16.  Lane l supplies A[l%16][8(l/16)+j] and
// B[8(l/16)+j][l%16] (j = 0..7) and receives D[4(l/16)+i][l%16] (i = 0..3).
// Every operand is stored with k contiguous, so each fragment is one
// 16-byte load: activations [row][k], weights W~ [out][in] (forward) and
// W~^T [in][out] (backward), and for the weight gradients the transposed
// activations a^T [k][batch] and g^T [out][batch].
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "leb.h"
#include "chain_features.hpp"
#include "leb_internal.hpp"

namespace leb {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

constexpr int MLP_MAX_LAYERS = 8;
constexpr int MLP_MAX_WIDTH = 256;
constexpr int FWD_ROWS = 64;            // rows (samples) per forward workgroup
// LDS row stride (BF16) of the forward activation tile: the widest layer the
// variant serves (128 or 256) + 8, which skews the rows over the banks
constexpr int fwd_lda(int ct) { return ct == 2 ? 136 : 264; }
constexpr size_t fwd_smem(int ct) { return 2 * (size_t)FWD_ROWS * fwd_lda(ct) * 2; }

// Standard normal CDF Phi(z) = (1 + erf(z / sqrt 2)) / 2 and exp(-z^2 / 2),
// with erf from Abramowitz and Stegun, Handbook of Mathematical Functions,
// formula 7.1.26 (|error| <= 1.5e-7): erf(x) ~ 1 - (a1 t + ... + a5 t^5)
// exp(-x^2), t = 1 / (1 + p x), x >= 0; odd extension for x < 0.
__device__ __forceinline__ void normal_cdf(float z, float* Phi, float* ex) {
    const float u = fabsf(z) * 0.70710678118654752f;
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, u, 1.0f));
    const float e = __builtin_amdgcn_exp2f(z * z * -0.72134752044448170f);     // exp(-z^2 / 2)
    const float poly =
        t * fmaf(t, fmaf(t, fmaf(t, fmaf(t, 1.061405429f, -1.453152027f), 1.421413741f), -0.284496736f),
                 0.254829592f);
    const float erf_abs = fmaf(-poly, e, 1.0f);
    *Phi = fmaf(0.5f, copysignf(erf_abs, z), 0.5f);
    *ex = e;
}
// GELU of the training forward: z Phi(z) with Phi from normal_cdf, the same
// approximation the backward differentiates.
__device__ __forceinline__ float gelu_train_f(float z) {
    float P, e;
    normal_cdf(z, &P, &e);
    return z * P;
}
// GELU of inference: z Phi(z) = max(z, 0) - |z| erfc(|z| / sqrt 2) / 2, with erfc from
// Abramowitz and Stegun, formula 7.1.28 (|error of erf| <= 3e-7):
// erf(x) ~ 1 - (1 + a1 x + ... + a6 x^6)^-16, x >= 0 -- one reciprocal and no
// exponential.  The coefficients below are c a_i / sqrt(2)^i with c = 2^(1/16):
// the polynomial is evaluated at |z| and its 16th power is 2 (1 + ...)^16, so
// the correction |z| / (2 (1 + ...)^16) is one fma; a large |z| drives the
// power to +inf and the correction to 0.  max(z, 0) is a median of three.
__device__ __forceinline__ float gelu_f(float z) {
    const float x = fabsf(z);
    float p = fmaf(x, 5.62129966e-6f, 5.10552090e-5f);
    p = fmaf(x, p, 3.96861370e-5f);
    p = fmaf(x, p, 3.42273924e-3f);
    p = fmaf(x, p, 2.20769985e-2f);
    p = fmaf(x, p, 5.20751630e-2f);
    p = fmaf(x, p, 1.04427378f);
    p = p * p;
    p = p * p;
    p = p * p;
    p = p * p;
    return fmaf(-x, __builtin_amdgcn_rcpf(p), __builtin_amdgcn_fmed3f(z, 0.0f, INFINITY));
}
__device__ __forceinline__ float gelu_grad_f(float z) {
    float P, e;
    normal_cdf(z, &P, &e);
    return P + z * e * 0.39894228040143268f;
}

static inline int pad32(int x) { return (x + 31) & ~31; }
static inline int pad16(int x) { return (x + 15) & ~15; }

struct MlpLayout {
    int L;
    int w[MLP_MAX_LAYERS + 1];     // true widths
    int kp[MLP_MAX_LAYERS];        // padded input width of layer l (multiple of 32)
    int np[MLP_MAX_LAYERS];        // padded output width of layer l (multiple of 32)
    int64_t poff[MLP_MAX_LAYERS];  // offset of W_l in the flat FP32 parameters (b_l follows)
    int64_t woff[MLP_MAX_LAYERS];  // offset of W~_l [np][kp] and W~_l^T [kp][np] in the BF16 copies
    int64_t nparams, nw;
};

// ---------------------------------------------------------------- forward

struct FwdArgs {
    MlpLayout G;
    const __bf16* Wt;         // W~_l [np][kp] per layer
    const float* params;      // biases b_l
    const float* x;           // [B][d0]
    float* y;                 // [B][dL]
    float* zsave;             // optional [L-1][B][np]   pre-activations
    __bf16* aT;               // optional [L][MAX_WIDTH][B]  a_l^T for l = 0..L-1
    int B;
    // chain surrogate sweep (FWD_CHAIN): rows are (unit, node) of a chain tube
    const double *cz, *cv, *cmu, *csg;
    double *cbar, *rbar;      // all 6 rows of each node, or (compact) rows 3, 4: [unit][U][2]
    int U;
    int compact;
    int sg_period;            // > 0: csg holds one trajectory's tube, unit u reads row u % sg_period
    double L0, pad;
};

enum { FWD_PLAIN = 0, FWD_SAVE = 1, FWD_CHAIN = 2 };

// One workgroup (4 waves) carries 64 rows through every layer.  The
// activation tile lives in LDS ([64][ldA] BF16, ldA = fwd_lda(CT)); weight
// fragments are read from global memory (L2-resident).  Wave w owns the
// 16-feature output tiles w, w+4, ..., up to CT of them, over all four
// 16-row tiles.  The MFMA computes the transposed tile, D = W~ a^T (weights
// as the A operand, activations as B), so each lane ends with 4
// consecutive features of one row: the epilogue writes 8 bytes per lane
// and tile.  The accumulators start at the bias; padded weight rows and
// biases are zero, so padded features come out as gelu(0) = 0 without a
// test.  The next layer's first weight chunk and bias are in flight during
// each epilogue.
//
// FWD_CHAIN: the rows are the nodes of a chain tube; the inputs are the
// chain surrogate's features, computed in the staging step, and the output
// (log-bounds of the vx, vz rows) is decoded into the residual zonotope in
// place of y: one kernel per surrogate sweep.
template <int CT, int MODE>
__global__ void __launch_bounds__(256) mlp_fwd_kernel(FwdArgs A) {
    constexpr bool SAVE = MODE == FWD_SAVE;
    __shared__ __align__(16) float sy[FWD_ROWS][LEB_CHAIN_OUTPUTS];
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int ldA = fwd_lda(CT);
    __bf16* buf0 = reinterpret_cast<__bf16*>(smem);
    __bf16* buf1 = buf0 + FWD_ROWS * ldA;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int row0 = blockIdx.x * FWD_ROWS;
    const MlpLayout& G = A.G;
    const int lr = lane & 15, lk = 8 * (lane >> 4), lf = 4 * (lane >> 4);
    // k-steps of 32 per weight chunk (registers: KS * CT fragments)
    constexpr int KS = CT == 2 ? 4 : 2;
    // weight fragments of chunk kc of layer l (and, for kc = 0, the bias of
    // the 4 features each lane accumulates in each slot)
    auto fetch = [&](int l, int kc, bf16x8 (&bb)[KS][CT], f32x4 (&bias_r)[CT]) {
        const int kp = G.kp[l], nout = G.w[l + 1];
        const int ntc = (l == G.L - 1) ? (nout + 15) / 16 : G.np[l] / 16;
        const int ns = __builtin_amdgcn_readfirstlane((ntc - wave + 3) >> 2);
        const __bf16* W = A.Wt + G.woff[l];
        const float* bias = A.params + G.poff[l] + (int64_t)nout * G.w[l];
#pragma unroll
        for (int s = 0; s < CT; ++s) {
            if (s >= ns) continue;
            const int ct = wave + 4 * s;
            const __bf16* wr = W + (int64_t)(ct * 16 + lr) * kp + lk + kc;
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
                if (kc + 32 * ks < kp) bb[ks][s] = *reinterpret_cast<const bf16x8*>(wr + 32 * ks);
            if (kc == 0) {
                const int c = ct * 16 + lf;
#pragma unroll
                for (int i = 0; i < 4; ++i) bias_r[s][i] = c + i < nout ? bias[c + i] : 0.0f;
            }
        }
    };
    bf16x8 b[KS][CT];
    f32x4 bnext[CT];
    fetch(0, 0, b, bnext);
    // stage a_0 = bf16(x), zero padded
    if (MODE == FWD_CHAIN) {
        if (tid < FWD_ROWS) {
            const int row = row0 + tid;
            float f[LEB_CHAIN_FEATURES];
            if (row < A.B) {
                const int U = A.U, nx = 6 * U, nu = 2 * U, n = nx + nu;
                const int u = row / U, i = row - u * U;
                const int us = A.sg_period > 0 ? u % A.sg_period : u;
                chain_node_features(A.cz + (int64_t)u * nx, A.cv + (int64_t)u * nu,
                                    A.cmu ? A.cmu + (int64_t)u * n : nullptr, A.csg + (int64_t)us * n, i, U, A.L0, f);
            } else {
#pragma unroll
                for (int k = 0; k < LEB_CHAIN_FEATURES; ++k) f[k] = 0.0f;
            }
#pragma unroll
            for (int k = 0; k < LEB_CHAIN_FEATURES; k += 8) {
                bf16x8 v;
#pragma unroll
                for (int j = 0; j < 8; ++j) v[j] = (__bf16)f[k + j];
                *reinterpret_cast<bf16x8*>(buf0 + tid * ldA + k) = v;
            }
        }
    } else {
        const int d0 = G.w[0], k0 = G.kp[0];
        for (int idx = tid; idx < FWD_ROWS * k0; idx += 256) {
            const int r = idx / k0, k = idx - r * k0;
            const int row = row0 + r;
            const float v = (row < A.B && k < d0) ? A.x[(int64_t)row * d0 + k] : 0.0f;
            const __bf16 bv = (__bf16)v;
            buf0[r * ldA + k] = bv;
            if (SAVE && row < A.B) A.aT[(int64_t)k * A.B + row] = bv;   // a_0^T
        }
    }
    __syncthreads();
    __bf16* cur = buf0;
    __bf16* nxt = buf1;
    for (int l = 0; l < G.L; ++l) {
        const int kp = G.kp[l], nout = G.w[l + 1];
        const bool last = (l == G.L - 1);
        // feature tiles of this layer (the output layer stops at its true width)
        const int ntc = last ? (nout + 15) / 16 : G.np[l] / 16;
        const int ns = __builtin_amdgcn_readfirstlane((ntc - wave + 3) >> 2);   // slots of this wave (may be <= 0)
        f32x4 acc[CT][4];
#pragma unroll
        for (int s = 0; s < CT; ++s)
#pragma unroll
            for (int rt = 0; rt < 4; ++rt) acc[s][rt] = bnext[s];
        if (ns > 0) {
            // the first chunk was fetched before the previous layer's epilogue
            for (int kc = 0; kc < kp; kc += 32 * KS) {
                if (kc > 0) fetch(l, kc, b, bnext);
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) {
                    const int k = kc + 32 * ks;
                    if (k >= kp) break;
                    bf16x8 a[4];
#pragma unroll
                    for (int rt = 0; rt < 4; ++rt)
                        a[rt] = *reinterpret_cast<const bf16x8*>(cur + (rt * 16 + lr) * ldA + k + lk);
#pragma unroll
                    for (int s = 0; s < CT; ++s)
                        if (s < ns)
#pragma unroll
                            for (int rt = 0; rt < 4; ++rt)
                                acc[s][rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[ks][s], a[rt], acc[s][rt], 0, 0, 0);
                }
            }
        }
        // next layer's first weight chunk and bias, in flight during this epilogue
        if (!last) fetch(l + 1, 0, b, bnext);
        // lane holds pre-activations of features c..c+3 of row rt * 16 + lr
        if (last) {
#pragma unroll
            for (int s = 0; s < CT; ++s) {
                if (s >= ns) continue;
                const int c = (wave + 4 * s) * 16 + lf;
#pragma unroll
                for (int rt = 0; rt < 4; ++rt) {
                    const int r = rt * 16 + lr;
                    const int row = row0 + r;
                    if (MODE == FWD_CHAIN) {
                        if (c == 0) *reinterpret_cast<f32x4*>(&sy[r][0]) = acc[s][rt];
                    } else if (row < A.B) {
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            if (c + i < nout) A.y[(int64_t)row * nout + c + i] = acc[s][rt][i];
                    }
                }
            }
        } else {
#pragma unroll
            for (int s = 0; s < CT; ++s) {
                if (s >= ns) continue;
                const int c = (wave + 4 * s) * 16 + lf;
#pragma unroll
                for (int rt = 0; rt < 4; ++rt) {
                    const int r = rt * 16 + lr;
                    bf16x4 av;
#pragma unroll
                    for (int i = 0; i < 4; ++i) av[i] = (__bf16)(SAVE ? gelu_train_f(acc[s][rt][i]) : gelu_f(acc[s][rt][i]));
                    *reinterpret_cast<bf16x4*>(nxt + r * ldA + c) = av;
                    if (SAVE) {
                        const int row = row0 + r;
                        if (row < A.B) {
                            *reinterpret_cast<f32x4*>(A.zsave + ((int64_t)l * A.B + row) * MLP_MAX_WIDTH + c) = acc[s][rt];
#pragma unroll
                            for (int i = 0; i < 4; ++i)
                                A.aT[((int64_t)(l + 1) * MLP_MAX_WIDTH + c + i) * A.B + row] = av[i];
                        }
                    }
                }
            }
        }
        __syncthreads();
        __bf16* t_ = cur; cur = nxt; nxt = t_;
    }
    if (MODE == FWD_CHAIN) {
        if (A.compact) {
            // decode: rows 3 and 4 of each node (row = u U + i, so [row][2])
            if (tid < 2 * FWD_ROWS) {
                const int r = tid >> 1, w = tid & 1;
                const int row = row0 + r;
                if (row < A.B) {
                    double c, rad;
                    chain_decode_row(sy[r][2 * w], sy[r][2 * w + 1], &c, &rad);
                    A.cbar[(int64_t)row * 2 + w] = c;
                    A.rbar[(int64_t)row * 2 + w] = rad + A.pad;
                }
            }
            return;
        }
        // decode: the 6 residual rows of each node, (0, pad) on the affine rows
        for (int idx = tid; idx < 6 * FWD_ROWS; idx += 256) {
            const int r = idx / 6, rc = idx - 6 * r;
            const int row = row0 + r;
            if (row >= A.B) continue;
            const int U = A.U, u = row / U, i = row - u * U;
            double c = 0.0, rad = 0.0;
            if (rc == 3 || rc == 4) chain_decode_row(sy[r][2 * (rc - 3)], sy[r][2 * (rc - 3) + 1], &c, &rad);
            const int64_t o = (int64_t)u * 6 * U + 6 * i + rc;
            A.cbar[o] = c;
            A.rbar[o] = rad + A.pad;
        }
    }
}

// ---------------------------------------------------------------- GEMM  C = A Bt^T

struct GemmArgs {
    const __bf16* A; int64_t lda;    // [M][K], k contiguous
    const __bf16* Bt; int64_t ldb;   // [N][K], k contiguous
    int M, N, K;                     // K a multiple of 32; operands hold zeros beyond their true extent
    // epilogue
    float* C; int64_t ldc;           // FP32 [M][N] (rows < Mst, cols < Nst stored)
    int Mst, Nst;
    const float* Z; int64_t ldz;     // optional: C <- C * gelu'(Z) and also emit BF16 copies
    __bf16* G; int64_t ldg;          // BF16 [M][..] of the (scaled) result, zero where col >= Nst
    __bf16* GT; int64_t ldgt;        // BF16 transposed [N][..], zero where col >= Nst
};

// 64 x 64 output tile per workgroup, 4 waves of 32 x 32 (2 x 2 MFMA
// tiles); K in steps of 32 staged through LDS.
__global__ void __launch_bounds__(256) mlp_gemm_kernel(GemmArgs P) {
    __shared__ __align__(16) __bf16 sA[64][40];
    __shared__ __align__(16) __bf16 sB[64][40];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    f32x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    // staging: 64 rows x 32 k = 256 chunks of 8 BF16; one chunk per thread per operand
    const int sr = tid >> 2, sk = (tid & 3) * 8;
    for (int k = 0; k < P.K; k += 32) {
        bf16x8 va = bf16x8{}, vb = bf16x8{};
        if (m0 + sr < P.M) va = *reinterpret_cast<const bf16x8*>(P.A + (int64_t)(m0 + sr) * P.lda + k + sk);
        if (n0 + sr < P.N) vb = *reinterpret_cast<const bf16x8*>(P.Bt + (int64_t)(n0 + sr) * P.ldb + k + sk);
        __syncthreads();
        *reinterpret_cast<bf16x8*>(&sA[sr][sk]) = va;
        *reinterpret_cast<bf16x8*>(&sB[sr][sk]) = vb;
        __syncthreads();
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const bf16x8 fa = *reinterpret_cast<const bf16x8*>(&sA[wm + a * 16 + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const bf16x8 fb = *reinterpret_cast<const bf16x8*>(&sB[wn + b * 16 + (lane & 15)][8 * (lane >> 4)]);
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, fb, acc[a][b], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int m = m0 + wm + a * 16 + 4 * (lane >> 4) + i;
                const int n = n0 + wn + b * 16 + (lane & 15);
                if (m >= P.M || n >= P.N) continue;
                float v = acc[a][b][i];
                const bool in = m < P.Mst && n < P.Nst;
                if (P.Z) v = in ? v * gelu_grad_f(P.Z[(int64_t)m * P.ldz + n]) : 0.0f;
                if (in && P.C) P.C[(int64_t)m * P.ldc + n] = v;
                if (P.G) P.G[(int64_t)m * P.ldg + n] = (__bf16)(in ? v : 0.0f);
                if (P.GT) P.GT[(int64_t)n * P.ldgt + m] = (__bf16)(in ? v : 0.0f);
            }
}

// ---------------------------------------------------------------- small kernels

// dz = dy = 2 (y - t) / (B d) in [B][ldw] (zero beyond d), G = bf16(dy)
// [B][ldw], GT [ldw][B]; per-block partial sums of (y - t)^2
__global__ void __launch_bounds__(256) mse_kernel(const float* y, const float* t, int B, int d, int ldw, float* dz,
                                                  __bf16* G, __bf16* GT, float* partial) {
    __shared__ float red[256];
    const int64_t total = (int64_t)B * ldw;
    const float scale = 2.0f / ((float)B * (float)d);
    float acc = 0.0f;
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < total; q += (int64_t)gridDim.x * 256) {
        const int b = (int)(q / ldw), c = (int)(q - (int64_t)b * ldw);
        float g = 0.0f;
        if (c < d) {
            const float diff = y[(int64_t)b * d + c] - t[(int64_t)b * d + c];
            acc += diff * diff;
            g = scale * diff;
        }
        const __bf16 gb = (__bf16)g;
        dz[q] = g;
        G[q] = gb;
        GT[(int64_t)c * B + b] = gb;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) sum_kernel(const float* partial, int n, float scale, float* out) {
    __shared__ float red[256];
    float acc = 0.0f;
    for (int q = threadIdx.x; q < n; q += 256) acc += partial[q];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0] * scale;
}

// db[c] = sum_b X[b][c] (c < n), one workgroup per 64 columns, fixed order
// Column sums of X [B][n] (row stride ldx): a workgroup takes 4 columns, its
// 256 lanes 64 row phases of each (every lane's loads in flight together),
// then a fixed-order tree over the phases.
__global__ void __launch_bounds__(256) colsum_kernel(const float* X, int64_t ldx, int B, int n, float* db) {
    __shared__ float red[64][4];
    const int cq = threadIdx.x & 3, part = threadIdx.x >> 2;
    const int c = blockIdx.x * 4 + cq;
    const int cc = c < n ? c : 0;
    float acc = 0.0f;
    for (int b0 = part; b0 < B; b0 += 8 * 64) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int b = b0 + 64 * u;
            const float x = X[(int64_t)(b < B ? b : 0) * ldx + cc];
            v[u] = b < B ? x : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += v[u];
    }
    red[part][cq] = acc;
    __syncthreads();
    for (int h = 32; h > 0; h >>= 1) {
        if (part < h) red[part][cq] += red[part + h][cq];
        __syncthreads();
    }
    if (part == 0 && c < n) db[c] = red[0][cq];
}

// Adam with the step-dependent factors formed on the host in FP64:
// lr_t = lr / (1 - b1^t), isc2 = 1 / sqrt(1 - b2^t), ob = 1 - b (so that
// 1 - 0.999 is not formed in FP32).
__global__ void adam_kernel(float* p, const float* g, float* m, float* v, int64_t n, float b1, float ob1, float b2,
                            float ob2, float lr_t, float isc2, float eps) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const float gq = g[q];
    const float mq = b1 * m[q] + ob1 * gq;
    const float vq = b2 * v[q] + ob2 * gq * gq;
    m[q] = mq;
    v[q] = vq;
    p[q] = p[q] - lr_t * mq / (sqrtf(vq) * isc2 + eps);
}

// BF16 copies of the weights: W~ [np][kp] and W~^T [kp][np], zero padded
__global__ void mlp_convert_kernel(MlpLayout G, const float* params, __bf16* Wt, __bf16* WtT) {
    const int l = blockIdx.y;
    if (l >= G.L) return;
    const int kp = G.kp[l], np = G.np[l], in = G.w[l], out = G.w[l + 1];
    const float* W = params + G.poff[l];
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < kp * np; q += gridDim.x * blockDim.x) {
        const int o = q / kp, i = q - o * kp;
        const __bf16 v = (__bf16)((o < out && i < in) ? W[(int64_t)o * in + i] : 0.0f);
        Wt[G.woff[l] + q] = v;
        WtT[G.woff[l] + (int64_t)i * np + o] = v;
    }
}

static unsigned nb(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

}  // namespace leb

using namespace leb;

// ---------------------------------------------------------------- object

struct leb_surrogate_s {
    MlpLayout G;
    bool narrow = true;        // every layer at most 128 wide: the CT = 2 forward variants
    float* params = nullptr;   // device FP32, flat
    float* m = nullptr;
    float* v = nullptr;
    float* grads = nullptr;
    __bf16* Wt = nullptr;      // [sum np kp]
    __bf16* WtT = nullptr;
    // training workspace, grown on demand (batch rows)
    int cap = 0;
    float* zsave = nullptr;    // [L-1][B][MAX_WIDTH]
    __bf16* aT = nullptr;      // [L][MAX_WIDTH][B]
    float* y = nullptr;        // [B][dL]
    float* dz[2] = {nullptr, nullptr};     // [B][MAX_WIDTH]
    __bf16* g[2] = {nullptr, nullptr};     // [B][MAX_WIDTH]
    __bf16* gT[2] = {nullptr, nullptr};    // [MAX_WIDTH][B]
    float* partial = nullptr;              // [1024]
    std::mutex mu;
};

static void sur_free_ws(leb_surrogate_s* s) {
    void* ps[] = {s->zsave, s->aT, s->y, s->dz[0], s->dz[1], s->g[0], s->g[1], s->gT[0], s->gT[1], s->partial};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    s->zsave = nullptr; s->aT = nullptr; s->y = nullptr; s->partial = nullptr;
    for (int q = 0; q < 2; ++q) { s->dz[q] = nullptr; s->g[q] = nullptr; s->gT[q] = nullptr; }
    s->cap = 0;
}

static int sur_ws(leb_surrogate_s* s, int B) {
    if (B <= s->cap) return LEB_OK;
    sur_free_ws(s);
    const int L = s->G.L;
    const size_t W = MLP_MAX_WIDTH;
    bool ok = hipMalloc(&s->zsave, (size_t)(L > 1 ? L - 1 : 1) * B * W * sizeof(float)) == hipSuccess &&
              hipMalloc(&s->aT, (size_t)L * W * B * sizeof(__bf16)) == hipSuccess &&
              hipMalloc(&s->y, (size_t)B * s->G.w[L] * sizeof(float)) == hipSuccess &&
              hipMalloc(&s->partial, 1024 * sizeof(float)) == hipSuccess;
    for (int q = 0; q < 2 && ok; ++q)
        ok = hipMalloc(&s->dz[q], (size_t)B * W * sizeof(float)) == hipSuccess &&
             hipMalloc(&s->g[q], (size_t)B * W * sizeof(__bf16)) == hipSuccess &&
             hipMalloc(&s->gT[q], (size_t)W * B * sizeof(__bf16)) == hipSuccess;
    if (!ok) { sur_free_ws(s); return LEB_ENOMEM; }
    s->cap = B;
    return LEB_OK;
}

extern "C" int leb_surrogate_create(int32_t n_layers, const int32_t* widths, const float* params_host,
                                    leb_surrogate* out) {
    if (!out || !widths || !params_host || n_layers < 1 || n_layers > MLP_MAX_LAYERS) return LEB_EINVAL;
    *out = nullptr;
    for (int l = 0; l <= n_layers; ++l)
        if (widths[l] < 1 || widths[l] > MLP_MAX_WIDTH) return LEB_EINVAL;
    leb_surrogate_s* s = new (std::nothrow) leb_surrogate_s;
    if (!s) return LEB_ENOMEM;
    MlpLayout& G = s->G;
    memset(&G, 0, sizeof(G));
    G.L = n_layers;
    int64_t po = 0, wo = 0;
    for (int l = 0; l <= n_layers; ++l) G.w[l] = widths[l];
    for (int l = 0; l < n_layers; ++l) {
        G.kp[l] = pad32(widths[l]);
        G.np[l] = pad32(widths[l + 1]);
        G.poff[l] = po;
        po += (int64_t)widths[l] * widths[l + 1] + widths[l + 1];
        G.woff[l] = wo;
        wo += (int64_t)G.kp[l] * G.np[l];
    }
    G.nparams = po;
    G.nw = wo;
    int widest = 0;
    for (int l = 0; l < n_layers; ++l) widest = widest > G.kp[l] ? widest : G.kp[l];
    for (int l = 0; l < n_layers; ++l) widest = widest > G.np[l] ? widest : G.np[l];
    s->narrow = widest <= 128;
    const size_t smem = fwd_smem(s->narrow ? 2 : 4);
    const void* fns[] = {(const void*)mlp_fwd_kernel<2, FWD_PLAIN>, (const void*)mlp_fwd_kernel<2, FWD_SAVE>,
                         (const void*)mlp_fwd_kernel<2, FWD_CHAIN>, (const void*)mlp_fwd_kernel<4, FWD_PLAIN>,
                         (const void*)mlp_fwd_kernel<4, FWD_SAVE>, (const void*)mlp_fwd_kernel<4, FWD_CHAIN>};
    bool attr_ok = true;
    if (smem > 65536)
        for (const void* f : fns)
            attr_ok = attr_ok &&
                      hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem) == hipSuccess;
    if (!attr_ok) {
        delete s;
        return LEB_EDEVICE;
    }
    const size_t pb = (size_t)po * sizeof(float);
    bool ok = hipMalloc(&s->params, pb) == hipSuccess && hipMalloc(&s->m, pb) == hipSuccess &&
              hipMalloc(&s->v, pb) == hipSuccess && hipMalloc(&s->grads, pb) == hipSuccess &&
              hipMalloc(&s->Wt, (size_t)wo * sizeof(__bf16)) == hipSuccess &&
              hipMalloc(&s->WtT, (size_t)wo * sizeof(__bf16)) == hipSuccess;
    ok = ok && hipMemcpy(s->params, params_host, pb, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemset(s->m, 0, pb) == hipSuccess && hipMemset(s->v, 0, pb) == hipSuccess;
    if (ok) {
        hipLaunchKernelGGL(mlp_convert_kernel, dim3(64, n_layers), dim3(256), 0, 0, G, s->params, s->Wt, s->WtT);
        ok = hipGetLastError() == hipSuccess && hipDeviceSynchronize() == hipSuccess;
    }
    if (!ok) {
        leb_surrogate_destroy(s);
        return LEB_ENOMEM;
    }
    *out = s;
    return LEB_OK;
}

extern "C" int leb_surrogate_destroy(leb_surrogate s) {
    if (!s) return LEB_OK;
    void* ps[] = {s->params, s->m, s->v, s->grads, s->Wt, s->WtT};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    sur_free_ws(s);
    delete s;
    return LEB_OK;
}

extern "C" int leb_surrogate_params(leb_surrogate s, float* params_host) {
    if (!s || !params_host) return LEB_EINVAL;
    std::lock_guard<std::mutex> lock(s->mu);
    if (hipDeviceSynchronize() != hipSuccess) return LEB_EDEVICE;
    return hipMemcpy(params_host, s->params, (size_t)s->G.nparams * sizeof(float), hipMemcpyDeviceToHost) ==
                   hipSuccess
               ? LEB_OK
               : LEB_EDEVICE;
}

extern "C" int64_t leb_surrogate_n_params(leb_surrogate s) { return s ? s->G.nparams : -1; }

extern "C" int leb_surrogate_dims(leb_surrogate s, int32_t* d_in, int32_t* d_out) {
    if (!s) return LEB_EINVAL;
    if (d_in) *d_in = s->G.w[0];
    if (d_out) *d_out = s->G.w[s->G.L];
    return LEB_OK;
}

static int fwd_dispatch(leb_surrogate_s* s, const FwdArgs& a, int mode, hipStream_t st) {
    const size_t smem = fwd_smem(s->narrow ? 2 : 4);
    const dim3 g(nb(a.B, FWD_ROWS)), t(256);
    if (s->narrow) {
        if (mode == FWD_SAVE) hipLaunchKernelGGL((mlp_fwd_kernel<2, FWD_SAVE>), g, t, smem, st, a);
        else if (mode == FWD_CHAIN) hipLaunchKernelGGL((mlp_fwd_kernel<2, FWD_CHAIN>), g, t, smem, st, a);
        else hipLaunchKernelGGL((mlp_fwd_kernel<2, FWD_PLAIN>), g, t, smem, st, a);
    } else {
        if (mode == FWD_SAVE) hipLaunchKernelGGL((mlp_fwd_kernel<4, FWD_SAVE>), g, t, smem, st, a);
        else if (mode == FWD_CHAIN) hipLaunchKernelGGL((mlp_fwd_kernel<4, FWD_CHAIN>), g, t, smem, st, a);
        else hipLaunchKernelGGL((mlp_fwd_kernel<4, FWD_PLAIN>), g, t, smem, st, a);
    }
    return hipGetLastError() == hipSuccess ? LEB_OK : LEB_EDEVICE;
}

static int fwd_launch(leb_surrogate_s* s, int B, const float* x, float* y, bool save, hipStream_t st) {
    FwdArgs a = {};
    a.G = s->G; a.Wt = s->Wt; a.params = s->params; a.x = x; a.y = y; a.B = B;
    a.zsave = save ? s->zsave : nullptr;
    a.aT = save ? s->aT : nullptr;
    return fwd_dispatch(s, a, save ? FWD_SAVE : FWD_PLAIN, st);
}

namespace leb {
// One surrogate sweep over a chain tube: features -> MLP -> (c_bar, rho_bar) for
// every (unit, node): the decoded bound on rows 6i+3, 6i+4, (0, pad) elsewhere.
int surrogate_chain_sweep(leb_surrogate s, const double* z, const double* v, const double* mu, const double* sigma,
                          int nodes, int U, double L0, double pad, double* cbar, double* rbar, hipStream_t st,
                          bool compact, int sg_period) {
    if (s->G.w[0] != LEB_CHAIN_FEATURES || s->G.w[s->G.L] != LEB_CHAIN_OUTPUTS) return LEB_EINVAL;
    if (nodes == 0) return LEB_OK;
    FwdArgs a = {};
    a.G = s->G; a.Wt = s->Wt; a.params = s->params; a.B = nodes;
    a.cz = z; a.cv = v; a.cmu = mu; a.csg = sigma; a.cbar = cbar; a.rbar = rbar; a.U = U; a.L0 = L0; a.pad = pad;
    a.compact = compact ? 1 : 0;
    a.sg_period = sg_period;
    return fwd_dispatch(s, a, FWD_CHAIN, st);
}
}  // namespace leb

extern "C" int leb_mlp_fwd_bf16(leb_surrogate s, int32_t batch, const float* x, float* y, void* stream) {
    if (!s || batch < 0) return LEB_EINVAL;
    if (batch == 0) return LEB_OK;
    if (!x || !y || !aligned8(x) || !aligned8(y)) return LEB_EINVAL;
    return fwd_launch(s, batch, x, y, false, (hipStream_t)stream);
}

// backward of sum(dy . y) from the saved forward (zsave, aT) and g_L in g[0]/gT[0]
static int bwd_core(leb_surrogate_s* s, int B, float* grads, hipStream_t st) {
    const MlpLayout& G = s->G;
    const int W = MLP_MAX_WIDTH;
    int cur = 0;
    for (int l = G.L - 1; l >= 0; --l) {
        const int in = G.w[l], out = G.w[l + 1];
        float* dW = grads + G.poff[l];
        float* db = dW + (int64_t)in * out;
        // dW_l [out][in] = g_l^T a_{l-1}: A = gT [out][B], Bt = aT_{l} [in][B], K = B
        GemmArgs p{};
        p.A = s->gT[cur]; p.lda = B;
        p.Bt = s->aT + (int64_t)l * W * B; p.ldb = B;
        p.M = out; p.N = in; p.K = B;
        p.C = dW; p.ldc = in; p.Mst = out; p.Nst = in;
        hipLaunchKernelGGL(mlp_gemm_kernel, dim3(nb(in, 64), nb(out, 64)), dim3(256), 0, st, p);
        // db_l = column sums of dz_l
        hipLaunchKernelGGL(colsum_kernel, dim3(nb(out, 4)), dim3(256), 0, st, s->dz[cur], (int64_t)W, B, out, db);
        if (l > 0) {
            // dz_{l-1} = (g_l W~_l) * gelu'(z_{l-1}): A = g [B][np_l], Bt = W~_l^T [kp_l][np_l]
            GemmArgs q{};
            q.A = s->g[cur]; q.lda = W;
            q.Bt = s->WtT + G.woff[l]; q.ldb = G.np[l];
            q.M = B; q.N = G.kp[l]; q.K = G.np[l];
            q.C = s->dz[cur ^ 1]; q.ldc = W; q.Mst = B; q.Nst = in;
            q.Z = s->zsave + (int64_t)(l - 1) * B * W; q.ldz = W;
            q.G = s->g[cur ^ 1]; q.ldg = W;
            q.GT = s->gT[cur ^ 1]; q.ldgt = B;
            hipLaunchKernelGGL(mlp_gemm_kernel, dim3(nb(G.kp[l], 64), nb(B, 64)), dim3(256), 0, st, q);
            cur ^= 1;
        }
    }
    return hipGetLastError() == hipSuccess ? LEB_OK : LEB_EDEVICE;
}

// g_L, gT_L and dz_L from dy [B][dL]
__global__ void dy_stage_kernel(const float* dy, int B, int d, float* dz, __bf16* G, __bf16* GT, int ldw) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)B * ldw;
    if (q >= total) return;
    const int b = (int)(q / ldw), c = (int)(q - (int64_t)b * ldw);
    const float v = c < d ? dy[(int64_t)b * d + c] : 0.0f;
    const __bf16 gb = (__bf16)v;
    dz[q] = v;
    G[q] = gb;
    GT[(int64_t)c * B + b] = gb;
}

extern "C" int leb_mlp_bwd_bf16(leb_surrogate s, int32_t batch, const float* x, const float* dy, float* grads,
                                void* stream) {
    if (!s || batch < 0) return LEB_EINVAL;
    if (batch == 0) return LEB_OK;
    if (!x || !dy || !grads || (batch & 31)) return LEB_EINVAL;
    std::lock_guard<std::mutex> lock(s->mu);
    hipStream_t st = (hipStream_t)stream;
    int rc = sur_ws(s, batch);
    if (rc) return rc;
    if ((rc = fwd_launch(s, batch, x, s->y, true, st))) return rc;
    hipLaunchKernelGGL(dy_stage_kernel, dim3(nb((int64_t)batch * MLP_MAX_WIDTH)), dim3(256), 0, st, dy, batch,
                       s->G.w[s->G.L], s->dz[0], s->g[0], s->gT[0], MLP_MAX_WIDTH);
    return bwd_core(s, batch, grads, st);
}

static int adam_launch(leb_surrogate_s* s, const float* grads, int step, double lr, double b1, double b2, double eps,
                       hipStream_t st) {
    const double c1 = 1.0 - pow(b1, step), c2 = 1.0 - pow(b2, step);
    hipLaunchKernelGGL(adam_kernel, dim3(nb(s->G.nparams)), dim3(256), 0, st, s->params, grads, s->m, s->v,
                       s->G.nparams, (float)b1, (float)(1.0 - b1), (float)b2, (float)(1.0 - b2), (float)(lr / c1),
                       (float)(1.0 / sqrt(c2)), (float)eps);
    hipLaunchKernelGGL(mlp_convert_kernel, dim3(64, s->G.L), dim3(256), 0, st, s->G, s->params, s->Wt, s->WtT);
    return hipGetLastError() == hipSuccess ? LEB_OK : LEB_EDEVICE;
}

extern "C" int leb_adam_step(leb_surrogate s, const float* grads, int32_t step, double lr, double beta1,
                             double beta2, double eps, void* stream) {
    if (!s || !grads || step < 1 || !(lr >= 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) ||
        !(eps > 0.0))
        return LEB_EINVAL;
    std::lock_guard<std::mutex> lock(s->mu);
    return adam_launch(s, grads, step, lr, beta1, beta2, eps, (hipStream_t)stream);
}

extern "C" int leb_surrogate_train_step(leb_surrogate s, int32_t batch, const float* x, const float* t,
                                        int32_t step, double lr, float* loss, void* stream) {
    if (!s || !x || !t || batch <= 0 || (batch & 31) || step < 1 || !(lr >= 0.0)) return LEB_EINVAL;
    std::lock_guard<std::mutex> lock(s->mu);
    hipStream_t st = (hipStream_t)stream;
    int rc = sur_ws(s, batch);
    if (rc) return rc;
    if ((rc = fwd_launch(s, batch, x, s->y, true, st))) return rc;
    const int d = s->G.w[s->G.L];
    const int nblocks = 256;
    hipLaunchKernelGGL(mse_kernel, dim3(nblocks), dim3(256), 0, st, s->y, t, batch, d, MLP_MAX_WIDTH, s->dz[0],
                       s->g[0], s->gT[0], s->partial);
    if (loss)
        hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, st, s->partial, nblocks, 1.0f / ((float)batch * d), loss);
    if ((rc = bwd_core(s, batch, s->grads, st))) return rc;
    return adam_launch(s, s->grads, step, lr, 0.9, 0.999, 1e-8, st);
}
