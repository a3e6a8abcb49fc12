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
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>

#include "ivl.hpp"
#include "leb.h"
#include "leb_internal.hpp"
#include "pbh_node.hpp"

namespace leb {

constexpr int PBH_BLOCK = 256;

struct ChainArgs {
    const double* z; const double* v; const double* mu; const double* sigma;
    double* r_lo; double* r_hi; double* c_bar; double* rho_bar; uint32_t* flags;
    SweepFold fold;         // fixed point: the previous sweep's fold (fold.prev == NULL: none)
    const PbhTile* tiles;   // optional: one tile (its own pointers, <= T units) per workgroup
    int64_t units;
    int U, T;
    double c;        // dt / m
    double kL;       // k_spring * rest_len
    double L0;
    double pad;
    int compact;     // 1: c_bar, rho_bar hold rows 3 and 4 of each node only, [unit][U][2]
};


__global__ void __launch_bounds__(PBH_BLOCK) pbh_chain_fwd(ChainArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int U = A.U, T = A.T;
    const int nx = 6 * U, nu = 2 * U, n = nx + nu;
    SpringOut* s_sp = reinterpret_cast<SpringOut*>(smem);                  // [T][U]
    uint32_t* s_flag = reinterpret_cast<uint32_t*>(s_sp + (size_t)T * U);   // [T]

    const int tid = threadIdx.x;
    TileRef t0;
    int64_t u0 = 0;
    if (A.tiles) {
        const PbhTile& pt = A.tiles[blockIdx.x];
        t0 = TileRef{pt.z, pt.v, pt.mu, pt.sigma, pt.r_lo, pt.r_hi, pt.c_bar, pt.rho_bar, pt.flags, pt.n};
    } else {
        u0 = (int64_t)blockIdx.x * T;
        const int64_t left = A.units - u0;
        t0.nloc = left < T ? (int)left : T;
        t0.Z = A.z + u0 * nx; t0.V = A.v + u0 * nu; t0.MU = A.mu ? A.mu + u0 * n : nullptr;
        t0.SG = A.sigma + u0 * n;
        t0.RLO = A.r_lo ? A.r_lo + u0 * nx : nullptr; t0.RHI = A.r_hi ? A.r_hi + u0 * nx : nullptr;
        const int64_t ro = A.compact ? 2 * U : nx;       // row length of c_bar, rho_bar
        t0.CB = A.c_bar ? A.c_bar + u0 * ro : nullptr; t0.RB = A.rho_bar ? A.rho_bar + u0 * ro : nullptr;
        t0.FL = A.flags ? A.flags + u0 : nullptr;
    }
    // fixed point: is any trajectory of this workgroup's units left open by the
    // previous sweep's containment test?  (Its T units of consecutive timesteps
    // span at most T <= PBH_BLOCK trajectories.)  A certified trajectory's tube is
    // frozen, so its residuals are not needed again.
    __shared__ uint32_t s_wopen[PBH_BLOCK / 64];
    const bool fold = A.fold.prev != nullptr;
    if (fold) {
        uint32_t my = 1u;
        if (A.fold.sweep > 0) {
            const int64_t N = A.units / A.fold.B;
            const int64_t b0 = u0 / N, nb = (u0 + t0.nloc - 1) / N - b0 + 1;
            my = tid < nb ? fp_is_open(A.fold.prev[b0 + tid]) : 0u;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) my |= __shfl_xor(my, off);
        if ((tid & 63) == 0) s_wopen[tid >> 6] = my;
    }
    for (int q = tid; q < T; q += PBH_BLOCK) s_flag[q] = 0u;
    const int lt = tid / U;
    const int i = tid - lt * U;
    NodeIn d0;
    node_load(t0, U, lt, i, d0);
    __syncthreads();      // s_flag cleared, s_wopen written
    if (fold) {
        uint32_t mine = 0u;
#pragma unroll
        for (int w = 0; w < PBH_BLOCK / 64; ++w) mine |= s_wopen[w];
        if (blockIdx.x == 0) {
            // the fold itself: state words of the previous sweep -> next, and the
            // number of trajectories still open, published to the device and the host
            __shared__ uint32_t s_gopen[PBH_BLOCK / 64];
            uint32_t c = 0;
            for (int b = tid; b < A.fold.B; b += PBH_BLOCK) {
                uint32_t w = 0u;
                if (A.fold.sweep > 0) {
                    const uint32_t st = A.fold.prev[b];
                    c += fp_is_open(st);
                    w = fp_fold_word(st, A.fold.sweep);
                }
                A.fold.next[b] = w;
            }
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
            if ((tid & 63) == 0) s_gopen[tid >> 6] = c;
            __syncthreads();
            if (tid == 0) {
                uint32_t open = (uint32_t)A.fold.B;
                if (A.fold.sweep > 0) {
                    open = 0;
#pragma unroll
                    for (int w = 0; w < PBH_BLOCK / 64; ++w) open += s_gopen[w];
                }
                A.fold.next[A.fold.B] = open;
                if (A.fold.sweep > 0 && A.fold.host_open)
                    __hip_atomic_store(&A.fold.host_open[A.fold.sweep % FP_SLOTS], open, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_SYSTEM);
            }
        }
        if (mine == 0u) return;       // every trajectory of this workgroup is certified
    }
    node_pass(A, t0, d0, lt, i, s_sp, s_flag);
}


size_t pbh_smem_bytes_T(int U, int T) {
    return (size_t)T * U * sizeof(SpringOut) + (size_t)T * sizeof(uint32_t) + 16;
}
size_t pbh_smem_bytes(int U) { return pbh_smem_bytes_T(U, PBH_BLOCK / U); }

int launch_pbh_chain(const leb_dynamics* dyn, int64_t units, const double* z, const double* v,
                     const double* mu, const double* sigma, double* r_lo, double* r_hi, double* c_bar,
                     double* rho_bar, double pad, uint32_t* flags, hipStream_t stream, const SweepFold* fold,
                     hipEvent_t ev0, hipEvent_t ev1, bool compact) {
    ChainArgs a;
    a.z = z; a.v = v; a.mu = mu; a.sigma = sigma;
    a.r_lo = r_lo; a.r_hi = r_hi; a.c_bar = c_bar; a.rho_bar = rho_bar; a.flags = flags;
    a.fold = fold ? *fold : SweepFold{nullptr, nullptr, nullptr, 0, 0};
    a.tiles = nullptr;
    a.units = units;
    a.U = dyn->n_units;
    a.T = PBH_BLOCK / a.U;
    a.c = dyn->dt / dyn->m;
    a.kL = dyn->k_spring * dyn->rest_len;
    a.L0 = dyn->rest_len;
    a.pad = pad;
    a.compact = compact ? 1 : 0;
    int64_t blocks = (units + a.T - 1) / a.T;
    if (blocks > 0x7fffffff) return LEB_EINVAL;
    if (ev0)        // timed: events at the kernel's start and end
        hipExtLaunchKernelGGL(pbh_chain_fwd, dim3((unsigned)blocks), dim3(PBH_BLOCK), pbh_smem_bytes(a.U), stream, ev0,
                              ev1, 0, a);
    else
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

// ------------------------------------------------------------ work queue
//
// Every analytic group of a batch in one persistent launch: a workgroup
// takes the next tile (group, tile) from a device counter until the tiles
// run out, and bounds it exactly as pbh_chain_fwd bounds a tile launch of
// that group (the same node passes, the group's U, T and constants), so the
// results equal the per-group launches bit for bit.  The counter must be 0
// when the launch starts (a one-thread reset kernel before it).
__global__ void pbh_queue_reset_kernel(int* counter) { *counter = 0; }

__global__ void __launch_bounds__(PBH_BLOCK) pbh_queue_kernel(PbhQueueArgs Q) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_item;
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0) s_item = atomicAdd(Q.counter, 1);
        __syncthreads();              // the item is visible; the previous tile's LDS use is over
        const int item = s_item;
        if (item >= Q.total) return;  // the same for every thread of the workgroup
        int g = 0;
        while (g + 1 < Q.n_groups && Q.groups[g + 1].first <= item) ++g;
        const PbhQueueGroup& G = Q.groups[g];
        ChainArgs A = {};
        A.fold = SweepFold{nullptr, nullptr, nullptr, 0, 0};
        A.U = G.U; A.T = G.T; A.c = G.c; A.kL = G.kL; A.L0 = G.L0; A.pad = 0.0; A.compact = 0;
        const int U = G.U, T = G.T;
        SpringOut* s_sp = reinterpret_cast<SpringOut*>(smem);                  // [T][U]
        uint32_t* s_flag = reinterpret_cast<uint32_t*>(s_sp + (size_t)T * U);   // [T]
        const PbhTile& pt = G.tiles[item - G.first];
        const TileRef t0{pt.z, pt.v, pt.mu, pt.sigma, pt.r_lo, pt.r_hi, pt.c_bar, pt.rho_bar, pt.flags, pt.n};
        for (int q = tid; q < T; q += PBH_BLOCK) s_flag[q] = 0u;
        const int lt = tid / U;
        const int i = tid - lt * U;
        NodeIn d0;
        node_load(t0, U, lt, i, d0);
        __syncthreads();              // s_flag cleared
        node_pass(A, t0, d0, lt, i, s_sp, s_flag);
        __syncthreads();              // every thread has read s_item and finished with the LDS
    }
}

int launch_pbh_queue(const PbhQueueArgs& q, size_t smem, int grid, hipStream_t stream) {
    if (q.total == 0) return LEB_OK;
    hipLaunchKernelGGL(pbh_queue_reset_kernel, dim3(1), dim3(1), 0, stream, q.counter);
    hipLaunchKernelGGL(pbh_queue_kernel, dim3((unsigned)grid), dim3(PBH_BLOCK), smem, stream, q);
    return hipGetLastError() == hipSuccess ? LEB_OK : LEB_EDEVICE;
}

int pbh_queue_grid(size_t smem, int total) {
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, pbh_queue_kernel, PBH_BLOCK, smem) != hipSuccess ||
        hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return -1;
    const int64_t g = (int64_t)std::max(per_cu, 1) * std::max(cus, 1);
    return (int)std::min<int64_t>(g, total);
}

}  // namespace leb
