// nn.hip -- linearization-error bound for ReLU-MLP dynamics (section IV.B).
//
// Dynamics f(x, u) = x + g([x; u]) (or g alone), g a ReLU MLP
//   z_l = W_l a_{l-1} + b_l, a_l = relu(z_l), g = z_L.
// CROWN (Theorem "CROWN bounds", Zhang et al. Thm 3.2) gives affine bounds
// W_lo a + b_lo <= g(a) <= W_hi a + b_hi over the box; Theorem 2 turns them
// into the remainder bound with the local Jacobian J = J_g(a~):
//   r_hi = max_X (W_hi - J) a + J a~ - g(a~) + b_hi, r_lo = min_X (...lo...).
// Relaxations per neuron from pre-activation bounds [l, u]: active (l >= 0)
// identity, inactive (u <= 0) zero, unstable: upper line s z + t with
// s = u/(u-l), t = -s l, lower line a z with a = 1 iff u >= -l.  First-layer
// bounds are exact; every later hidden layer gets its own full CROWN pass.
//
// GPU design.  Each backward substitution step
//     Lambda_next = (Lambda (.) S) W_l      (S sign-selected slopes)
// is a batched dense contraction run on FP64 MFMA (v_mfma_f64_16x16x4):
// the left operand is generated on the fly from Lambda and the per-box
// slopes, the shared weight tile is staged through LDS, and the per-row bias
// (intercepts, Omega b_l) and rounding-term weights are accumulated while
// the operand is generated.  The upper, lower and Jacobian chains of one
// box share the same kernel (modes), the Jacobian chain using S = 1[z^ > 0].
//
// Soundness in floating point: every FP64 dot product of length <= 300 has
// error <= 2^-44.8 times the dot product of absolute values.  Each bound
// adds 2^-40 times the absolute-value dot products of every step (computed
// alongside as matrix-vector products), covering the relaxation scaling,
// the contraction, the bias sums, the concretisation, the nominal forward
// pass and the Jacobian chain.  Upper-line slopes are rounded up so the
// computed line stays above the ReLU on [l, u].
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "leb.h"
#include "leb_internal.hpp"

#include "nn_net.hpp"

namespace leb {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr double RT = 0x1p-40;   // rounding allowance factor
constexpr int NN_CHUNK = 4096;   // boxes per pass
constexpr uint32_t NN_UNSTABLE = 1u << 31;   // private per-box bit: some neuron is unstable

}  // namespace leb

namespace leb {

// ------------------------------------------------------------------ prep

struct PrepArgs {
    const double* z; const double* v; const double* mu; const double* sigma;
    int64_t u0; int nbox;
    int L; int w[NN_MAXL + 1]; int nx, nu;
    const double* W[NN_MAXL]; const double* WT[NN_MAXL]; const double* b[NN_MAXL];
    // outputs (chunk-local)
    double* alpha; double* c; double* rho;                 // [box][w0]
    double* zhat;                                          // [L-1][box][W]
    double* lo; double* hi;                                // [L-1][box][W] (layer 1 filled here)
    double* g; double* eg;                                 // [box][m]
    uint32_t* flags;                                       // [box]
};

// one workgroup (256 lanes) per box
__global__ void __launch_bounds__(256) nn_prep_kernel(PrepArgs A) {
    __shared__ double s_a[NN_MAXW], s_m[NN_MAXW], s_v[NN_MAXW];
    __shared__ double s_c[NN_MAXW], s_r[NN_MAXW], s_al[NN_MAXW];
    __shared__ uint32_t s_flag;
    const int box = blockIdx.x, q = threadIdx.x;
    const int64_t unit = A.u0 + box;
    const int n0 = A.w[0], m = A.w[A.L];
    if (q == 0) s_flag = 0;
    __syncthreads();
    if (q < n0) {
        const double x = q < A.nx ? A.z[unit * A.nx + q] : A.v[unit * A.nu + (q - A.nx)];
        const double sg = A.sigma[unit * n0 + q];
        const double mu = A.mu ? A.mu[unit * n0 + q] : 0.0;
        uint32_t f = 0;
        if (!isfinite(x) || !isfinite(sg) || !isfinite(mu) || !(sg >= 0.0)) f |= LEB_FLAG_BAD_INPUT;
        if (fabs(mu) > sg) f |= LEB_FLAG_HULL_EXTENDED;
        if (f) atomicOr(&s_flag, f);
        // box = hull({a~}, a~ + mu +/- sigma): centre and half-width, widened
        // so the FP64 box encloses the exact one
        const double dlo = fmin(mu - sg, 0.0), dhi = fmax(mu + sg, 0.0);
        const double cc = x + 0.5 * (dlo + dhi);
        double rr = 0.5 * (dhi - dlo);
        rr = rr + rr * 0x1p-50 + (fabs(x) + fabs(dlo) + fabs(dhi)) * 0x1p-51;
        s_al[q] = x; s_c[q] = cc; s_r[q] = rr;
        s_a[q] = x;                                   // forward input
        s_m[q] = fabs(x);                             // magnitude chain (nominal pass error)
        s_v[q] = fabs(cc - x) + rr;                   // |a - a~| bound (Jacobian error)
        A.alpha[box * n0 + q] = x; A.c[box * n0 + q] = cc; A.rho[box * n0 + q] = rr;
    }
    __syncthreads();
    // first layer bounds, exact affine image of the box
    {
        const int h = A.w[1];
        if (q < h) {
            const double* Wr = A.W[0] + (size_t)q * n0;
            double lin = A.b[0][q], mag = 0.0, abs_ = fabs(A.b[0][q]);
            for (int k = 0; k < n0; ++k) {
                lin = __builtin_fma(Wr[k], s_c[k], lin);
                mag = __builtin_fma(fabs(Wr[k]), s_r[k], mag);
                abs_ = __builtin_fma(fabs(Wr[k]), fabs(s_c[k]), abs_);
            }
            const double err = RT * (abs_ + mag + fabs(lin));
            A.lo[(size_t)box * NN_MAXW + q] = lin - mag - err;
            A.hi[(size_t)box * NN_MAXW + q] = lin + mag + err;
        }
    }
    // nominal forward pass, magnitude chains (nominal error, Jacobian error)
    for (int l = 0; l < A.L; ++l) {
        const int in = A.w[l], out = A.w[l + 1];
        double z = 0.0, mz = 0.0, vz = 0.0;
        if (q < out) {
            const double* WT = A.WT[l];
            z = A.b[l][q];
            mz = fabs(A.b[l][q]);
            // eight k at a time, the weight loads of a group issued before its sums
            int k = 0;
            for (; k + 8 <= in; k += 8) {
                double wv[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) wv[u] = WT[(size_t)(k + u) * out + q];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    z = __builtin_fma(wv[u], s_a[k + u], z);
                    mz = __builtin_fma(fabs(wv[u]), s_m[k + u], mz);
                    vz = __builtin_fma(fabs(wv[u]), s_v[k + u], vz);
                }
            }
            for (; k < in; ++k) {
                const double wk = WT[(size_t)k * out + q];
                z = __builtin_fma(wk, s_a[k], z);
                mz = __builtin_fma(fabs(wk), s_m[k], mz);
                vz = __builtin_fma(fabs(wk), s_v[k], vz);
            }
        }
        __syncthreads();
        if (q < out) {
            if (l < A.L - 1) {
                const bool on = z > 0.0;
                A.zhat[((size_t)l * A.nbox + box) * NN_MAXW + q] = z;
                s_a[q] = on ? z : 0.0;
                s_m[q] = mz;
                s_v[q] = on ? vz : 0.0;
            } else {
                A.g[box * m + q] = z;
                // |g^ - g| and |(J^ - J)(a - a~)| allowances
                A.eg[box * m + q] = RT * (mz + vz);
            }
        }
        __syncthreads();
    }
    if (q == 0) A.flags[box] = s_flag;
}

// ---------------------------------------------------------------- relax

struct RelaxArgs {
    const double* lo; const double* hi;     // [box][W] of layer l
    const double* amax_prev;                // [box][W] of layer l-1, or NULL (input layer: |c| + rho)
    const double* c; const double* rho;     // [box][w0]
    const double* WT;                       // layer l transposed [w[l-1]][w[l]]
    const double* b;                        // [w[l]]
    const double* zhat;                     // [box][W]
    int in, out, n0;
    double* s; double* t; double* a; double* D; double* e; double* amax;   // [box][W]
    uint32_t* boxflags;                     // [box]
};

// sound relaxation coefficients and rounding weights e = zmax + |W| amax_prev + |b| + |t|
__global__ void __launch_bounds__(256) nn_relax_kernel(RelaxArgs A) {
    __shared__ double s_am[NN_MAXW];
    const int box = blockIdx.x, q = threadIdx.x;
    if (q < A.in) {
        if (A.amax_prev) s_am[q] = A.amax_prev[(size_t)box * NN_MAXW + q];
        else s_am[q] = fabs(A.c[box * A.n0 + q]) + A.rho[box * A.n0 + q];
    }
    __syncthreads();
    const size_t o = (size_t)box * NN_MAXW + q;
    const bool unstable = q < A.out && A.lo[o] < 0.0 && A.hi[o] > 0.0;
    if (__syncthreads_or(unstable) && q == 0) atomicOr(&A.boxflags[box], NN_UNSTABLE);
    if (q >= A.out) return;
    const double l = A.lo[o], u = A.hi[o];
    double s, t, a;
    if (l >= 0.0) { s = 1.0; t = 0.0; a = 1.0; }
    else if (u <= 0.0) { s = 0.0; t = 0.0; a = 0.0; }
    else {
        s = u / (u - l);
        s = s + s * 0x1p-50;             // rounded up: the line stays above relu on [l, u]
        t = -s * l;
        t = t + t * 0x1p-50;
        a = (u >= -l) ? 1.0 : 0.0;
    }
    double wa = 0.0;
    int k = 0;
    for (; k + 8 <= A.in; k += 8) {           // the weight loads of a group issued before its sums
        double wv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) wv[u] = A.WT[(size_t)(k + u) * A.out + q];
#pragma unroll
        for (int u = 0; u < 8; ++u) wa = __builtin_fma(fabs(wv[u]), s_am[k + u], wa);
    }
    for (; k < A.in; ++k) wa = __builtin_fma(fabs(A.WT[(size_t)k * A.out + q]), s_am[k], wa);
    A.s[o] = s; A.t[o] = t; A.a[o] = a;
    A.D[o] = A.zhat[o] > 0.0 ? 1.0 : 0.0;
    A.e[o] = fmax(fabs(l), fabs(u)) + wa + fabs(A.b[q]) + fabs(t);
    A.amax[o] = fmax(u, 0.0);
}

// ---------------------------------------------------------- fused chain
//
// The whole backward substitution of one target layer k, for one box, one
// mode and a block of 16 target rows, in one workgroup:
//   Lambda_{j-1} = (Lambda_j (.) S_j) W_j,   j = k-1, ..., 1,   Lambda_k = rows of W_k,
//   beta += sum_i (Lambda_j t_sel)_i + (Omega_j b_j),   eps += |Lambda_j| e_j,
// with Lambda kept in LDS between the steps (never in HBM).  The product is
// formed transposed on FP64 MFMA (v_mfma_f64_16x16x4): Lambda^T_{j-1} =
// W_j^T Omega^T, so the accumulator of one step (lane l holds element
// [4i + l/16][l%16] of a 16 x 16 tile) is stored to LDS in the layout the
// next step reads its B operand from (lane l supplies B[l/16][l%16]).  A
// operands are W_j columns read from L2, 16 consecutive values per k.
// Neurons of layer j that are stably inactive (u <= 0) have zero slopes and
// intercepts in every mode, so their columns of Omega_j are exactly 0: each
// step runs over the workgroup's list of the other neurons only.
// Wave w produces the output tiles w, w + 4, ... of each step; wave 0 also
// sums the bias and rounding terms of its rows.
struct ChainArgs {
    const double* WTt;             // target layer k, transposed: [w_{k-1}][M] (shared by every box)
    const double* bt;              // [M]
    const double* W[NN_MAXL];      // layer j at W[j-1]: [w_j][w_{j-1}]
    const double* b[NN_MAXL];
    int w[NN_MAXL + 1];
    int k, M, nbox;
    // per-box vectors of hidden layer j (1-based) at base + (j - 1) * lstride + box * NN_MAXW
    const double* s; const double* t; const double* a; const double* D; const double* e; const double* hi;
    size_t lstride;
    double* C;                     // [mode][box][M][w_0]
    double* beta; double* eps;     // [mode][box][M]
};

constexpr size_t CHAIN_STATE_BYTES = (size_t)NN_MAXW * 16 * sizeof(double);
constexpr int CHAIN_PAD = NN_MAXW + 8;               // listed neurons, padded past the last k-step read

__global__ void __launch_bounds__(256) nn_chain_kernel(ChainArgs A) {
    extern __shared__ double cst[];                    // [NN_MAXW][16]: Lambda^T of this block
    __shared__ double cv[5][CHAIN_PAD];                // slope x >= 0, slope x < 0, intercept, bias, e (list order)
    __shared__ int sk[CHAIN_PAD];                      // neurons of layer j that are not stably inactive
    __shared__ int scnt[4];
    __shared__ double spart[768];                      // partial tiles of the k-slices; then the row sums
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = lane & 15, g = lane >> 4;
    const int mode = blockIdx.y, box = blockIdx.z;
    const int K0 = A.w[A.k - 1];
    // intercept of the selected line: upper mode on x >= 0, lower mode on x < 0
    const bool t_on_pos = mode == 0, t_on_neg = mode == 1;
    // list the neurons of layer j that are not stably inactive and stage this
    // mode's slopes, intercept, bias and rounding weight of each, in list order
    int Kc = 0;
    auto prepare = [&](int j) {
        const int K = A.w[j];
        const size_t vo = (size_t)(j - 1) * A.lstride + (size_t)box * NN_MAXW;
        const bool keep = tid < K && A.hi[vo + tid] > 0.0;
        const uint64_t bal = __ballot(keep);
        if (lane == 0) scnt[wave] = __popcll(bal);
        __syncthreads();                               // counts (and the previous step's state) written
        int off = 0;
        Kc = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) { off += q < wave ? scnt[q] : 0; Kc += scnt[q]; }
        if (keep) sk[off + __popcll(bal & ((1ull << lane) - 1ull))] = tid;
        if (tid >= Kc) sk[tid] = 0;                    // padding (its x is forced to 0)
        if (tid < CHAIN_PAD - 256) sk[256 + tid] = 0;
        __syncthreads();
        for (int q = tid; q < CHAIN_PAD; q += 256) {
            const int k = sk[q];
            const size_t o = vo + k;
            const double s_ = A.s[o], a_ = A.a[o];
            cv[0][q] = mode == 0 ? s_ : (mode == 1 ? a_ : A.D[o]);
            cv[1][q] = mode == 0 ? a_ : (mode == 1 ? s_ : A.D[o]);
            cv[2][q] = mode == 2 ? 0.0 : A.t[o];
            cv[3][q] = A.b[j - 1][k];
            cv[4][q] = A.e[o];
        }
        __syncthreads();
    };
    // a target with one step (k = 2) runs every 16-row block in this workgroup with
    // one list; deeper targets run one block per workgroup
    const bool single = A.k == 2;
    const int nrb = (A.M + 15) / 16;
    if (single) prepare(1);
    for (int rb = single ? 0 : blockIdx.x; rb < (single ? nrb : blockIdx.x + 1); ++rb) {
    const int row0 = 16 * rb;
    // Lambda_k: rows row0 .. row0 + 15 of W_k (zero past M), read from W_k^T so that
    // both the loads and the LDS stores are consecutive
    for (int q = tid; q < 16 * K0; q += 256) {
        const int kk = q >> 4, rr = q & 15;
        const bool ok = row0 + rr < A.M;
        const double x = A.WTt[ok ? (size_t)kk * A.M + row0 + rr : 0];
        cst[q] = ok ? x : 0.0;
    }
    if (single) __syncthreads();                       // (otherwise prepare() waits for the state)
    double pb = 0.0, pe = 0.0;
    for (int j = A.k - 1; j >= 1; --j) {
        const int N = A.w[j - 1];
        const double* Wj = A.W[j - 1];
        if (!single) prepare(j);
        // work split: ntile >= 3: wave w owns tiles w, w + 4, ... over all k; ntile 2 or
        // 1: the waves split the k-steps of the tile(s) into 2 or 4 slices
        const int ntile = N / 16;
        const int nslice = ntile >= 3 ? 1 : 4 / ntile;
        const int slice = wave / (4 / nslice);
        const int tfirst = ntile >= 3 ? wave : wave % ntile;
        const int nmine = tfirst < ntile ? (ntile >= 3 ? (ntile - wave + 3) / 4 : 1) : 0;
        const bool sums = tfirst == 0;                 // the waves of tile 0 sum the row terms of their slice
        d4 acc[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i] = d4{0.0, 0.0, 0.0, 0.0};
        if (nmine > 0) {
            // k-step covers list positions c0 .. c0 + 3 (lane group g takes c0 + g);
            // this wave runs c0 = 4 slice, 4 slice + 4 nslice, ...; the operands of the
            // next k-step (W columns from L2, the state and vectors from LDS) are read
            // while this one's MFMAs run
            const int stride = 4 * nslice;
            double wn[4], xn, psn, nsn, tn, bn, en;
            auto load = [&](int c0) {
                const int c = c0 + g;
                const int k = sk[c];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int tt = i < nmine ? tfirst + 4 * i : tfirst;
                    wn[i] = Wj[(size_t)k * N + 16 * tt + r];
                }
                xn = c < Kc ? cst[k * 16 + r] : 0.0;
                psn = cv[0][c]; nsn = cv[1][c]; tn = cv[2][c]; bn = cv[3][c]; en = cv[4][c];
            };
            load(4 * slice);
            for (int c0 = 4 * slice; c0 < Kc; c0 += stride) {
                double wc[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) wc[i] = wn[i];
                const double x = xn, ps = psn, ns = nsn, tv = tn, bb = bn, ee = en;
                load(c0 + stride < Kc ? c0 + stride : c0);     // the last one re-reads in bounds
                const bool pos = x >= 0.0;
                const double om = x * (pos ? ps : ns);
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (i < nmine) acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(wc[i], om, acc[i], 0, 0, 0);
                if (sums) {
                    if (pos ? t_on_pos : t_on_neg) pb = __builtin_fma(x, tv, pb);
                    pb = __builtin_fma(om, bb, pb);
                    pe = __builtin_fma(fabs(x), ee, pe);
                }
            }
        }
        // slices 1.. hand their partial tiles to slice 0 (added in slice order); every
        // read of the state is done before it is overwritten
        const int pidx = nslice == 4 ? slice - 1 : tfirst;
        if (nslice > 1 && slice > 0 && nmine > 0) {
#pragma unroll
            for (int q = 0; q < 4; ++q) spart[pidx * 256 + q * 64 + lane] = acc[0][q];
        }
        __syncthreads();
        if (nslice > 1 && slice == 0 && nmine > 0) {
            for (int sl = 1; sl < nslice; ++sl) {
                const int pi = nslice == 4 ? sl - 1 : tfirst;
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[0][q] += spart[pi * 256 + q * 64 + lane];
            }
        }
        if (slice == 0) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (i >= nmine) break;
                const int tt = tfirst + 4 * i;
#pragma unroll
                for (int q = 0; q < 4; ++q) cst[(16 * tt + 4 * q + g) * 16 + r] = acc[i][q];
            }
        }
        __syncthreads();                               // the next step reads the state just written
    }
    // Lambda_0 rows of this block, and the bias and rounding sums of each row
    const int n0 = A.w[0];
    const size_t cbase = ((size_t)mode * A.nbox + box) * A.M;
    for (int q = tid; q < 16 * n0; q += 256) {
        const int rr = q / n0, n = q - rr * n0;
        if (row0 + rr < A.M) A.C[(cbase + row0 + rr) * n0 + n] = cst[n * 16 + rr];
    }
    spart[wave * 64 + lane] = pb;
    spart[256 + wave * 64 + lane] = pe;
    __syncthreads();
    if (tid < 16 && row0 + tid < A.M) {
        double b_ = 0.0, e_ = 0.0;
        for (int w = 0; w < 4; ++w)
            for (int q = 0; q < 4; ++q) { b_ += spart[w * 64 + tid + 16 * q]; e_ += spart[256 + w * 64 + tid + 16 * q]; }
        const double bt = A.bt[row0 + tid];
        A.beta[cbase + row0 + tid] = bt + b_;
        A.eps[cbase + row0 + tid] = e_ + fabs(bt);
    }
    __syncthreads();                                   // the next block reuses the state and sums
    }
}

// A target with a single step (k = 2) whose input layer is 16 wide:
//   Lambda_0 = (W_2 (.) S_1) W_1   ([w_2] x [16]) for one box and mode,
// every 16-row block in this workgroup.  The listed neurons of layer 1 are the
// same for every block, so each lane loads the W_1 values of all its k-steps
// once (up to 16 in registers, all in flight together); the k-steps of a block
// are split over the four waves (slices) and summed in slice order.  The next
// block's rows of W_2 are loaded while this block's MFMAs run.
__global__ void __launch_bounds__(256) nn_chain1_kernel(ChainArgs A) {
    extern __shared__ double cst[];                    // [NN_MAXW][16]: Omega^T of the current block
    __shared__ double cv[5][CHAIN_PAD];
    __shared__ int sk[CHAIN_PAD];
    __shared__ int scnt[4];
    __shared__ double spart[768];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = lane & 15, g = lane >> 4;
    const int mode = blockIdx.y, box = blockIdx.z;
    const int K = A.w[1], M = A.M;
    const double* W1 = A.W[0];                         // [w_1][16]
    const size_t vo = (size_t)box * NN_MAXW;
    // the listed neurons of layer 1 and this mode's vectors
    const bool keep = tid < K && A.hi[vo + tid] > 0.0;
    const uint64_t bal = __ballot(keep);
    if (lane == 0) scnt[wave] = __popcll(bal);
    __syncthreads();
    int off = 0, Kc = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) { off += q < wave ? scnt[q] : 0; Kc += scnt[q]; }
    if (keep) sk[off + __popcll(bal & ((1ull << lane) - 1ull))] = tid;
    if (tid >= Kc) sk[tid] = 0;
    if (tid < CHAIN_PAD - 256) sk[256 + tid] = 0;
    __syncthreads();
    for (int q = tid; q < CHAIN_PAD; q += 256) {
        const int k = sk[q];
        const size_t o = vo + k;
        const double s_ = A.s[o], a_ = A.a[o];
        cv[0][q] = mode == 0 ? s_ : (mode == 1 ? a_ : A.D[o]);
        cv[1][q] = mode == 0 ? a_ : (mode == 1 ? s_ : A.D[o]);
        cv[2][q] = mode == 2 ? 0.0 : A.t[o];
        cv[3][q] = A.b[0][k];
        cv[4][q] = A.e[o];
    }
    // this lane's W_1 values: k-step m of slice `wave` covers list positions
    // 4 wave + 16 m .. + 3, lane group g takes + g
    double wv[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        const int c = 4 * wave + 16 * m + g;
        const double x = W1[(size_t)sk[c < CHAIN_PAD ? c : 0] * 16 + r];
        wv[m] = c < Kc ? x : 0.0;
    }
    const bool t_on_pos = mode == 0, t_on_neg = mode == 1;
    const int nrb = (M + 15) / 16;
    const size_t cbase = ((size_t)mode * A.nbox + box) * M;
    // rows of W_2 for block rb: thread q < 16 K0 takes (kk, rr) = (q / 16, q % 16) for q = tid + 256 u
    const int K0 = K;                                   // = w_1, the columns of W_2
    double nx[16];
    auto fetch = [&](int rb) {
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int q = tid + 256 * u, kk = q >> 4, rr = q & 15;
            const bool ok = q < 16 * K0 && 16 * rb + rr < M;
            const double x = A.WTt[ok ? (size_t)kk * M + 16 * rb + rr : 0];
            nx[u] = ok ? x : 0.0;
        }
    };
    fetch(0);
    for (int rb = 0; rb < nrb; ++rb) {
        __syncthreads();                               // vectors staged; the previous block is done with cst
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int q = tid + 256 * u;
            if (q < 16 * NN_MAXW) cst[q] = nx[u];
        }
        __syncthreads();
        if (rb + 1 < nrb) fetch(rb + 1);
        d4 acc = d4{0.0, 0.0, 0.0, 0.0};
        double pb = 0.0, pe = 0.0;
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            const int c = 4 * wave + 16 * m + g;
            if (4 * wave + 16 * m >= Kc) break;
            const int k = sk[c];
            const double x = c < Kc ? cst[k * 16 + r] : 0.0;
            const bool pos = x >= 0.0;
            const double om = x * (pos ? cv[0][c] : cv[1][c]);
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(wv[m], om, acc, 0, 0, 0);
            if (pos ? t_on_pos : t_on_neg) pb = __builtin_fma(x, cv[2][c], pb);
            pb = __builtin_fma(om, cv[3][c], pb);
            pe = __builtin_fma(fabs(x), cv[4][c], pe);
        }
        if (wave > 0) {
#pragma unroll
            for (int q = 0; q < 4; ++q) spart[(wave - 1) * 256 + q * 64 + lane] = acc[q];
        }
        __syncthreads();
        if (wave == 0) {
            for (int sl = 1; sl < 4; ++sl) {
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[q] += spart[(sl - 1) * 256 + q * 64 + lane];
            }
            // accumulator element q: row 4 q + g... of the transposed tile: n = 4 q + g, row = r
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (16 * rb + r < M) A.C[(cbase + 16 * rb + r) * 16 + 4 * q + g] = acc[q];
        }
        __syncthreads();                               // partial tiles read
        spart[tid] = pb;
        spart[256 + tid] = pe;
        __syncthreads();
        if (tid < 16 && 16 * rb + tid < M) {
            double b_ = 0.0, e_ = 0.0;
            for (int w = 0; w < 4; ++w)
                for (int q = 0; q < 4; ++q) { b_ += spart[w * 64 + tid + 16 * q]; e_ += spart[256 + w * 64 + tid + 16 * q]; }
            const double bt = A.bt[16 * rb + tid];
            A.beta[cbase + 16 * rb + tid] = bt + b_;
            A.eps[cbase + 16 * rb + tid] = e_ + fabs(bt);
        }
    }
}

// ----------------------------------------------------------- concretize

struct ConcArgs {
    const double* L0;            // [mode][box][M][n0]
    const double* beta; const double* eps;   // [mode][box][M]
    const double* c; const double* rho;      // [box][n0]
    int M, n0, nbox;
    double* lo; double* hi;      // [box][W]
};

// mode 0 -> upper bound into hi, mode 1 -> lower bound into lo
__global__ void __launch_bounds__(256) nn_concretize_kernel(ConcArgs A) {
    const int box = blockIdx.x, r = threadIdx.x, mode = blockIdx.y;
    if (r >= A.M) return;
    const double* Lr = A.L0 + (((size_t)mode * A.nbox + box) * A.M + r) * A.n0;
    const double* c = A.c + (size_t)box * A.n0;
    const double* rho = A.rho + (size_t)box * A.n0;
    double lin = 0.0, mag = 0.0, ab = 0.0;
    // eight k at a time, every load of a group issued before its sums (same order of summation)
    int k = 0;
    for (; k + 8 <= A.n0; k += 8) {
        double lv[8], cv[8], rv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) { lv[u] = Lr[k + u]; cv[u] = c[k + u]; rv[u] = rho[k + u]; }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            lin = __builtin_fma(lv[u], cv[u], lin);
            mag = __builtin_fma(fabs(lv[u]), rv[u], mag);
            ab = __builtin_fma(fabs(lv[u]), fabs(cv[u]), ab);
        }
    }
    for (; k < A.n0; ++k) {
        lin = __builtin_fma(Lr[k], c[k], lin);
        mag = __builtin_fma(fabs(Lr[k]), rho[k], mag);
        ab = __builtin_fma(fabs(Lr[k]), fabs(c[k]), ab);
    }
    const size_t o = ((size_t)mode * A.nbox + box) * A.M + r;
    const double beta = A.beta[o];
    const double err = RT * (A.eps[o] + ab + mag + fabs(beta) + fabs(lin));
    if (mode == 0) A.hi[(size_t)box * NN_MAXW + r] = lin + mag + beta + err;
    else A.lo[(size_t)box * NN_MAXW + r] = lin - mag + beta - err;
}

// ---------------------------------------------------------------- thm 2

struct Thm2Args {
    const double* L0;            // [3][box][m][n0]: upper, lower, Jacobian
    const double* beta; const double* eps;   // [3][box][m]
    const double* alpha; const double* c; const double* rho;   // [box][n0]
    const double* g; const double* eg;        // [box][m]
    const uint32_t* flags;       // [box]
    const double* Juser;         // NULL, or the caller's J [unit][m][n0] (replaces mode 2)
    int m, n0, nbox;
    int64_t u0;
    double* r_lo; double* r_hi; double* c_bar; double* rho_bar; double pad;
    uint32_t* flags_out;
};

__global__ void __launch_bounds__(64) nn_thm2_kernel(Thm2Args A) {
    const int box = blockIdx.x, i = threadIdx.x;
    if (i >= A.m) return;
    const size_t sz = (size_t)A.nbox * A.m;
    const double* Lu = A.L0 + ((size_t)0 * sz + (size_t)box * A.m + i) * A.n0;
    const double* Ll = A.L0 + ((size_t)1 * sz + (size_t)box * A.m + i) * A.n0;
    const double* J = A.Juser ? A.Juser + ((size_t)(A.u0 + box) * A.m + i) * A.n0
                              : A.L0 + ((size_t)2 * sz + (size_t)box * A.m + i) * A.n0;
    const double* al = A.alpha + (size_t)box * A.n0;
    const double* c = A.c + (size_t)box * A.n0;
    const double* rho = A.rho + (size_t)box * A.n0;
    double hu = 0.0, hl = 0.0, mu_ = 0.0, ml = 0.0, ja = 0.0, ab = 0.0;
    for (int k = 0; k < A.n0; ++k) {
        const double du = Lu[k] - J[k], dl = Ll[k] - J[k];
        hu = __builtin_fma(du, c[k], hu);
        hl = __builtin_fma(dl, c[k], hl);
        mu_ = __builtin_fma(fabs(du), rho[k], mu_);
        ml = __builtin_fma(fabs(dl), rho[k], ml);
        ja = __builtin_fma(J[k], al[k], ja);
        ab += (fabs(du) + fabs(dl)) * fabs(c[k]) + fabs(J[k]) * fabs(al[k]);
    }
    const size_t ou = (size_t)box * A.m + i, ol = sz + ou;
    const double g = A.g[ou];
    const double bu = A.beta[ou], bl = A.beta[ol];
    const double base = ja - g;
    double hi = hu + mu_ + base + bu;
    double lo = hl - ml + base + bl;
    const double common = ab + mu_ + ml + fabs(ja) + fabs(g);
    hi += RT * (A.eps[ou] + common + fabs(bu) + fabs(hi)) + A.eg[ou];
    lo -= RT * (A.eps[ol] + common + fabs(bl) + fabs(lo)) + A.eg[ou];
    // 0 = r(a~) lies in every valid bound (for any J)
    hi = fmax(hi, 0.0);
    lo = fmin(lo, 0.0);
    uint32_t f = A.flags[box];
    // no unstable neuron: g is affine on the box and equal to its linearization
    // with the computed Jacobian, so that remainder is exactly 0
    if (!(f & NN_UNSTABLE) && !A.Juser) { lo = 0.0; hi = 0.0; }
    // a caller's J with a non-finite entry in this row: the whole unit is invalid
    if (A.Juser) {
        const double* Jb = A.Juser + (size_t)(A.u0 + box) * A.m * A.n0;
        bool bad = false;
        for (int q = 0; q < A.m * A.n0; ++q) bad |= !isfinite(Jb[q]);
        if (bad) f |= LEB_FLAG_BAD_INPUT;
    }
    if (f & LEB_FLAG_BAD_INPUT) { lo = -INFINITY; hi = INFINITY; }
    const int64_t o = (A.u0 + box) * A.m + i;
    A.r_lo[o] = lo;
    A.r_hi[o] = hi;
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
    if (A.flags_out && i == 0) A.flags_out[A.u0 + box] = f & ~NN_UNSTABLE;
}

// --------------------------------------------------------------- host

struct NNWorkspace {
    std::mutex mu;
    std::vector<void*> bufs;
    std::vector<size_t> sizes;
    WsFence fence;
};
static NNWorkspace g_nnws;

static int nn_ws(int slot, size_t bytes, double** out) {
    if ((int)g_nnws.bufs.size() <= slot) { g_nnws.bufs.resize(slot + 1, nullptr); g_nnws.sizes.resize(slot + 1, 0); }
    if (g_nnws.sizes[slot] < bytes) {
        if (g_nnws.bufs[slot]) (void)hipFree(g_nnws.bufs[slot]);
        g_nnws.bufs[slot] = nullptr;
        g_nnws.sizes[slot] = 0;
        if (getenv("LEB_TEST_FAIL_ALLOC")) return LEB_ENOMEM;
        if (hipMalloc(&g_nnws.bufs[slot], bytes) != hipSuccess) return LEB_ENOMEM;
        g_nnws.sizes[slot] = bytes;
    }
    *out = (double*)g_nnws.bufs[slot];
    return LEB_OK;
}

static int launch_chain(const ChainArgs& c, int nmode, int nact, hipStream_t st) {
    static bool attr = false;
    if (!attr) {
        if (hipFuncSetAttribute((const void*)nn_chain_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)CHAIN_STATE_BYTES) != hipSuccess ||
            hipFuncSetAttribute((const void*)nn_chain1_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)CHAIN_STATE_BYTES) != hipSuccess)
            return LEB_EDEVICE;
        attr = true;
    }
    if (c.k == 2 && c.w[0] == 16) {
        hipLaunchKernelGGL(nn_chain1_kernel, dim3(1, nmode, nact), dim3(256), CHAIN_STATE_BYTES, st, c);
        return hipGetLastError() == hipSuccess ? LEB_OK : LEB_EDEVICE;
    }
    const unsigned rbs = c.k == 2 ? 1u : (unsigned)((c.M + 15) / 16);
    hipLaunchKernelGGL(nn_chain_kernel, dim3(rbs, nmode, nact), dim3(256), CHAIN_STATE_BYTES, st, c);
    return hipGetLastError() == hipSuccess ? LEB_OK : LEB_EDEVICE;
}

}  // namespace leb

using namespace leb;

extern "C" int leb_mlp_create(int32_t n_layers, const int32_t* widths, const float* const* W,
                              const float* const* b, int32_t nx, int32_t residual, leb_mlp* out) {
    if (!out || !widths || !W || !b) return LEB_EINVAL;
    *out = nullptr;
    if (n_layers < 2 || n_layers > NN_MAXL) return LEB_ENOTSUP;
    for (int l = 0; l <= n_layers; ++l)
        if (widths[l] < 1) return LEB_EINVAL;
    for (int l = 0; l < n_layers; ++l) {
        if (widths[l] > NN_MAXW || widths[l] % 16 != 0) return LEB_ENOTSUP;
        if (!W[l] || !b[l]) return LEB_EINVAL;
    }
    if (widths[n_layers] > 64) return LEB_ENOTSUP;
    if (nx < 0 || nx > widths[0]) return LEB_EINVAL;
    if (residual && nx != widths[n_layers]) return LEB_EINVAL;
    leb_mlp_s* net = new leb_mlp_s();
    net->L = n_layers;
    for (int l = 0; l <= n_layers; ++l) net->w[l] = widths[l];
    net->nx = nx;
    net->nu = widths[0] - nx;
    net->residual = residual ? 1 : 0;
    for (int l = 0; l < n_layers; ++l) {
        const int in = widths[l], o = widths[l + 1];
        std::vector<double> w((size_t)in * o), wt((size_t)in * o), bb(o);
        for (int r = 0; r < o; ++r) {
            for (int k = 0; k < in; ++k) {
                const double x = (double)W[l][(size_t)r * in + k];
                if (!isfinite(x)) { leb_mlp_destroy(net); return LEB_EINVAL; }
                w[(size_t)r * in + k] = x;
                wt[(size_t)k * o + r] = x;
            }
            bb[r] = (double)b[l][r];
            if (!isfinite(bb[r])) { leb_mlp_destroy(net); return LEB_EINVAL; }
        }
        void *p1 = nullptr, *p2 = nullptr, *p3 = nullptr;
        if (getenv("LEB_TEST_FAIL_ALLOC") || hipMalloc(&p1, w.size() * 8) != hipSuccess ||
            hipMalloc(&p2, wt.size() * 8) != hipSuccess || hipMalloc(&p3, bb.size() * 8) != hipSuccess) {
            if (p1) (void)hipFree(p1);
            if (p2) (void)hipFree(p2);
            if (p3) (void)hipFree(p3);
            leb_mlp_destroy(net);
            return LEB_ENOMEM;
        }
        net->allocs.push_back(p1); net->allocs.push_back(p2); net->allocs.push_back(p3);
        if (hipMemcpy(p1, w.data(), w.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(p2, wt.data(), wt.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(p3, bb.data(), bb.size() * 8, hipMemcpyHostToDevice) != hipSuccess) {
            leb_mlp_destroy(net);
            return LEB_EDEVICE;
        }
        net->W[l] = (double*)p1; net->WT[l] = (double*)p2; net->b[l] = (double*)p3;
    }
    *out = net;
    return LEB_OK;
}

extern "C" int leb_mlp_destroy(leb_mlp net) {
    if (!net) return LEB_OK;
    for (void* p : net->allocs) (void)hipFree(p);
    delete net;
    return LEB_OK;
}

namespace leb {

void nn_dims(const leb_mlp_s* net, int* nx, int* nu, int* m) {
    *nx = net->nx;
    *nu = net->nu;
    *m = net->w[net->L];
}

// Sizes (bytes) of the 21 work buffers of the bound for chunks of CB boxes.
void nn_buffer_sizes(const leb_mlp_s* net, int CB, size_t sizes[NN_NBUF]) {
    const int L = net->L, n0 = net->w[0], m = net->w[L];
    const size_t per = (size_t)CB * NN_MAXW * 8;
    const size_t lam = (size_t)CB * 3 * NN_MAXW * n0 * 8;          // Lambda_0 of every row, mode and box
    const size_t v3 = (size_t)CB * 3 * NN_MAXW * 8;
    const size_t tab[NN_NBUF] = {(size_t)CB * n0 * 8, (size_t)CB * n0 * 8, (size_t)CB * n0 * 8, per * (L - 1),
                                 per * (L - 1), per * (L - 1), (size_t)CB * m * 8, (size_t)CB * m * 8,
                                 per * (L - 1), per * (L - 1), per * (L - 1), per * (L - 1), per * (L - 1),
                                 per * (L - 1), lam, 8, v3, v3, v3, v3, (size_t)CB * 8};
    for (int q = 0; q < NN_NBUF; ++q) sizes[q] = tab[q];
}

// The bound of `units` boxes in chunks of CB, with caller-provided work
// buffers (nn_buffer_sizes); only kernels are enqueued on st.
int nn_bound_run(const leb_mlp_s* net, int64_t units, const double* z, const double* v, const double* mu,
                 const double* sigma, const double* J, double* r_lo, double* r_hi, double* c_bar, double* rho_bar,
                 double pad, uint32_t* flags, int CB, double* const* buf, hipStream_t st) {
    const int L = net->L, n0 = net->w[0], m = net->w[L];
    int rc;
    double *alpha = buf[0], *c = buf[1], *rho = buf[2], *zhat = buf[3], *lo = buf[4], *hi = buf[5], *g = buf[6],
           *eg = buf[7], *s = buf[8], *t = buf[9], *a = buf[10], *D = buf[11], *e = buf[12], *amax = buf[13],
           *bufA = buf[14], *beta = buf[16], *eps = buf[17];
    uint32_t* fl = (uint32_t*)buf[20];
    auto layer = [&](double* base, int l) { return base + (size_t)l * CB * NN_MAXW; };   // hidden layer l+1

    for (int64_t u0 = 0; u0 < units; u0 += CB) {
        const int nb = (int)((units - u0) < CB ? (units - u0) : CB);
        PrepArgs pa;
        pa.z = z; pa.v = v; pa.mu = mu; pa.sigma = sigma; pa.u0 = u0; pa.nbox = CB;
        pa.L = L;
        for (int l = 0; l <= L; ++l) pa.w[l] = net->w[l];
        pa.nx = net->nx; pa.nu = net->nu;
        for (int l = 0; l < L; ++l) { pa.W[l] = net->W[l]; pa.WT[l] = net->WT[l]; pa.b[l] = net->b[l]; }
        pa.alpha = alpha; pa.c = c; pa.rho = rho; pa.zhat = zhat; pa.lo = lo; pa.hi = hi; pa.g = g; pa.eg = eg;
        pa.flags = fl;
        hipLaunchKernelGGL(nn_prep_kernel, dim3(nb), dim3(256), 0, st, pa);
        if (hipGetLastError() != hipSuccess) return LEB_EDEVICE;
        auto relax = [&](int l) -> int {     // hidden layer l+1 (0-based l)
            RelaxArgs ra;
            ra.lo = layer(lo, l); ra.hi = layer(hi, l);
            ra.amax_prev = l == 0 ? nullptr : layer(amax, l - 1);
            ra.c = c; ra.rho = rho;
            ra.WT = net->WT[l]; ra.b = net->b[l]; ra.zhat = layer(zhat, l);
            ra.in = net->w[l]; ra.out = net->w[l + 1]; ra.n0 = n0;
            ra.s = layer(s, l); ra.t = layer(t, l); ra.a = layer(a, l); ra.D = layer(D, l);
            ra.e = layer(e, l); ra.amax = layer(amax, l);
            ra.boxflags = fl;
            hipLaunchKernelGGL(nn_relax_kernel, dim3(nb), dim3(256), 0, st, ra);
            return hipGetLastError() == hipSuccess ? LEB_OK : LEB_EDEVICE;
        };
        if ((rc = relax(0))) return rc;
        // backward chain for target layer k (1-based, 2..L): modes 0 upper, 1 lower (, 2 Jacobian)
        auto chain = [&](int k, int nmode, double** lam_out, double** beta_out, double** eps_out) -> int {
            ChainArgs ca = {};
            ca.WTt = net->WT[k - 1]; ca.bt = net->b[k - 1];
            for (int l = 0; l < L; ++l) { ca.W[l] = net->W[l]; ca.b[l] = net->b[l]; }
            for (int l = 0; l <= L; ++l) ca.w[l] = net->w[l];
            ca.k = k; ca.M = net->w[k]; ca.nbox = CB;
            ca.s = s; ca.t = t; ca.a = a; ca.D = D; ca.e = e; ca.hi = hi;
            ca.lstride = (size_t)CB * NN_MAXW;
            ca.C = bufA; ca.beta = beta; ca.eps = eps;
            if ((rc = launch_chain(ca, nmode, nb, st))) return rc;
            *lam_out = bufA; *beta_out = beta; *eps_out = eps;
            return LEB_OK;
        };
        for (int k = 2; k <= L - 1; ++k) {
            double *L0, *bt, *ep;
            if ((rc = chain(k, 2, &L0, &bt, &ep))) return rc;
            ConcArgs ca;
            ca.L0 = L0; ca.beta = bt; ca.eps = ep; ca.c = c; ca.rho = rho;
            ca.M = net->w[k]; ca.n0 = n0; ca.nbox = CB;
            ca.lo = layer(lo, k - 1); ca.hi = layer(hi, k - 1);
            hipLaunchKernelGGL(nn_concretize_kernel, dim3(nb, 2), dim3(256), 0, st, ca);
            if (hipGetLastError() != hipSuccess) return LEB_EDEVICE;
            if ((rc = relax(k - 1))) return rc;
        }
        double *L0, *bt, *ep;
        // the Jacobian chain (mode 2) only when the caller gives no J
        if ((rc = chain(L, J ? 2 : 3, &L0, &bt, &ep))) return rc;
        Thm2Args ta;
        ta.L0 = L0; ta.beta = bt; ta.eps = ep; ta.alpha = alpha; ta.c = c; ta.rho = rho; ta.g = g; ta.eg = eg;
        ta.flags = fl; ta.Juser = J; ta.m = m; ta.n0 = n0; ta.nbox = CB; ta.u0 = u0;
        ta.r_lo = r_lo; ta.r_hi = r_hi; ta.c_bar = c_bar; ta.rho_bar = rho_bar; ta.pad = pad; ta.flags_out = flags;
        hipLaunchKernelGGL(nn_thm2_kernel, dim3(nb), dim3(64), 0, st, ta);
        if (hipGetLastError() != hipSuccess) return LEB_EDEVICE;
    }
    return LEB_OK;
}

}  // namespace leb

extern "C" int leb_nn_bound(leb_mlp net, int32_t batch, int32_t N, const double* z, const double* v, const double* mu,
                            const double* sigma, const double* J, double* r_lo, double* r_hi, double* c_bar,
                            double* rho_bar, double pad, uint32_t* flags, void* stream) {
    if (!net) return LEB_EINVAL;
    if (batch < 0 || N < 0 || !(pad >= 0.0) || !isfinite(pad)) return LEB_EINVAL;
    if ((c_bar == nullptr) != (rho_bar == nullptr)) return LEB_EINVAL;
    const int64_t units = (int64_t)batch * N;
    if (units == 0) return LEB_OK;
    if (!z || !sigma || !r_lo || !r_hi || (net->nu > 0 && !v) || (net->nx > 0 && !z)) return LEB_EINVAL;
    const void* ptrs[] = {z, v, mu, sigma, J, r_lo, r_hi, c_bar, rho_bar};
    for (const void* p : ptrs)
        if (p && !aligned8(p)) return LEB_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    const int L = net->L, n0 = net->w[0], m = net->w[L];
    std::lock_guard<std::mutex> lock(g_nnws.mu);
    const int CB = (int)(units < NN_CHUNK ? units : NN_CHUNK);
    size_t sizes[NN_NBUF];
    nn_buffer_sizes(net, CB, sizes);
    double* buf[NN_NBUF];
    int rc;
    for (int q = 0; q < NN_NBUF; ++q)
        if ((rc = nn_ws(q, sizes[q], &buf[q]))) return rc;
    if ((rc = g_nnws.fence.enter(st))) return rc;
    WsFenceScope leave{g_nnws.fence, st};
    return nn_bound_run(net, units, z, v, mu, sigma, J, r_lo, r_hi, c_bar, rho_bar, pad, flags, CB, buf, st);
}
