// leb_internal.hpp -- launchers shared between the C-ABI layer and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "leb.h"

namespace leb {

// Workgroup barrier that orders LDS only: each wave's LDS accesses complete
// before it, its global loads and stores stay in flight (__syncthreads would
// drain them too).
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Per-trajectory fixed-point state word.
constexpr uint32_t FP_CERT = 1u;          // certified (frozen)
constexpr uint32_t FP_OPEN = 1u << 31;    // this sweep: F(C) not inside C
constexpr int FP_SLOTS = 4096;            // host-visible open counts, one per sweep (mod FP_SLOTS)

// The fold of fixed-point sweep t, done by the bound launch of sweep t + 1:
// every workgroup counts the trajectories left open by sweep t (and returns
// at once when there are none); workgroup 0 also writes the folded state
// words (certified at t, or open) and the count for sweep t + 1 and publishes
// the count to host memory.  sweep == 0: nothing to fold, every trajectory open.
struct SweepFold {
    const uint32_t* prev;   // [B] state words after sweep t's containment marks
    uint32_t* next;         // [B] folded words, [B] open count after sweep t
    uint32_t* host_open;    // host-mapped counts, slot t % FP_SLOTS (NULL: device only)
    int B;
    int sweep;              // t
};
// fold of state words: certified at sweep t unless marked open
__device__ __forceinline__ uint32_t fp_fold_word(uint32_t st, int sweep) {
    return (st & FP_CERT) ? st : ((st & FP_OPEN) ? 0u : (FP_CERT | ((uint32_t)sweep << 1)));
}
__device__ __forceinline__ uint32_t fp_is_open(uint32_t st) {
    return (!(st & FP_CERT) && (st & FP_OPEN)) ? 1u : 0u;
}

// one workgroup's share of a batched bound launch: up to T units of one problem
struct PbhTile {
    const double* z; const double* v; const double* mu; const double* sigma;
    double* r_lo; double* r_hi; double* c_bar; double* rho_bar; uint32_t* flags;
    int n;
    int pad_;
};
constexpr int PBH_BLOCK_LANES = 256;
// tiles: device array of n_tiles tiles, each of at most T units (T <= 256 / n_units)
int launch_pbh_tiles(const leb_dynamics* dyn, const PbhTile* tiles, int n_tiles, int T, hipStream_t stream);
// one analytic group of a batch in the work queue: its tiles are items first .. first + n_tiles - 1
struct PbhQueueGroup {
    const PbhTile* tiles;
    int first, n_tiles;
    int U, T;
    double c, kL, L0;
};
struct PbhQueueArgs {
    const PbhQueueGroup* groups;   // device, in item order
    int n_groups, total;
    int* counter;                  // device
};
int launch_pbh_queue(const PbhQueueArgs& q, size_t smem, int grid, hipStream_t stream);
int pbh_queue_grid(size_t smem, int total);
size_t pbh_smem_bytes_T(int U, int T);

int launch_pbh_chain(const leb_dynamics* dyn, int64_t units, const double* z, const double* v,
                     const double* mu, const double* sigma, double* r_lo, double* r_hi, double* c_bar,
                     double* rho_bar, double pad, uint32_t* flags, hipStream_t stream,
                     const SweepFold* fold = nullptr, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr,
                     bool compact = false);
size_t pbh_smem_bytes(int U);
size_t bwd_smem_bytes(int U);
int launch_tube_map(int B, int N, int U, const double* phi, const double* e, const double* cbar,
                    const double* rbar, double* mu, double* sigma, hipStream_t s,
                    double scale = 1.0, double shift = 0.0);
// the tube map of compact residuals c2, r2 [B][N][U][2] (rows 3 and 4 of each
// node; the four affine rows are (0, pad))
int launch_tube_map_compact(int B, int N, int U, const double* phi, const double* e, double pad, const double* c2,
                            const double* r2, double* mu, double* sigma, hipStream_t s, double scale = 1.0,
                            double shift = 0.0);
// tube of the residual zonotopes (0, pad) at every step (the disturbance-only tube)
// fixed-point arguments checked before any launch: options and e (LEB_EINVAL),
// the horizon the compact tube map supports (LEB_ENOTSUP)
constexpr int FP_MAX_N = 210;
int fp_check_args(const leb_fp_options* opt, const double* e, int N);
int launch_disturbance_tube(int B, int N, int U, const double* phi, const double* e, double pad, double* mu,
                            double* sigma, hipStream_t s);

// ReLU-MLP bound with caller-provided work buffers
constexpr int NN_NBUF = 21;
void nn_buffer_sizes(const leb_mlp_s* net, int CB, size_t sizes[NN_NBUF]);
int nn_bound_run(const leb_mlp_s* net, int64_t units, const double* z, const double* v, const double* mu,
                 const double* sigma, const double* J, double* r_lo, double* r_hi, double* c_bar, double* rho_bar,
                 double pad, uint32_t* flags, int CB, double* const* buf, hipStream_t st);
void nn_dims(const leb_mlp_s* net, int* nx, int* nu, int* m);

// one surrogate sweep over a chain tube (features -> BF16 MLP -> residual zonotope,
// all rows [unit][6U], or compact: rows 3 and 4 [unit][U][2]).  sg_period > 0: the
// tube is the same for every trajectory, sigma holds one trajectory [sg_period][8U]
// and unit u reads row u % sg_period
int surrogate_chain_sweep(leb_surrogate s, const double* z, const double* v, const double* mu, const double* sigma,
                          int nodes, int U, double L0, double pad, double* cbar, double* rbar, hipStream_t st,
                          bool compact = false, int sg_period = 0);

// argument checks shared by the entry points
bool aligned8(const void* p);
int check_chain_dynamics(const leb_dynamics* dyn);     // CHAIN or LINEAR
int check_dynamics(const leb_dynamics* dyn);           // any kind of leb_dyn_kind

// Device-side order of the calls that share a library-owned workspace.  The
// host mutex of the workspace orders the host side only; its kernels may
// still be queued when the next call, on another stream, starts.  Each call
// therefore makes its stream wait for the event that the previous call
// recorded after its last launch (enter), and records its own (leave).
// Both run under the workspace's mutex.
struct WsFence {
    hipEvent_t ev = nullptr;
    bool armed = false;
    int enter(hipStream_t s);
    int leave(hipStream_t s);
};
// leave() on scope exit, for calls with several return paths after their first launch
struct WsFenceScope {
    WsFence& f;
    hipStream_t s;
    ~WsFenceScope() { (void)f.leave(s); }
};

// closed-form test dynamics (LINEAR, QUADRATIC, SINCOS): one thread per unit
int launch_small_dyn(const leb_dynamics* dyn, int mode, int64_t units, const double* z, const double* v,
                     const double* mu, const double* sigma, double* r_lo, double* r_hi, double* c_bar,
                     double* rho_bar, double pad, uint32_t* flags, hipStream_t s);
// point Jacobians A [units][nx][nx], B [units][nx][nu] of chain dynamics at the nominal
int launch_chain_jacobians(const leb_dynamics* dyn, int64_t units, const double* z, const double* v, double* A,
                           double* B, hipStream_t s);

}  // namespace leb
