/*
 * leb.h -- C ABI of the MI355X linearization-error-bound (LEB) library.
 *
 * The library computes, for every timestep k of a nominal trajectory, a
 * componentwise interval [r_lo, r_hi] that contains the linearization
 * remainder
 *     r(x, u) = f(x, u) - f(z_k, v_k) - A_k (x - z_k) - B_k (u - v_k)
 * for every (x, u) in the tube box of that timestep (paper: Problem 1 and
 * eq. linear_error_def).  The tube box is the interval set
 *     ((z_k, v_k) + mu_k) (+) diag(sigma_k) E        (eq. zontope_combination_interval)
 * extended, when |mu_k| > sigma_k in some coordinate, to the hull with the
 * nominal point (Theorem 1 needs the nominal point inside the box).
 *
 * Conventions shared by every entry point:
 *   - Array arguments are DEVICE pointers (for example torch tensor
 *     data_ptr()) unless marked "host"; FP64 arrays are row-major and
 *     contiguous and must be 8-byte aligned.  The caller owns every buffer.
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *     Work is enqueued asynchronously on it; argument checks happen on the
 *     host before anything is enqueued.
 *   - A negative return value (leb_status) means nothing was enqueued.
 *     Data anomalies found on the device never abort a call and never
 *     yield a finite unsound number: the affected rows become
 *     [-inf, +inf] and a bit is set in the per-unit flags word.
 *   - A "unit" is one (trajectory, timestep) pair; units are laid out
 *     trajectory-major: unit = b * N + k.
 */
#ifndef LEB_H
#define LEB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LEB_OK = 0,
    LEB_EINVAL = -1,     /* bad argument (shape, null pointer, parameter range) */
    LEB_ENOMEM = -2,     /* device allocation failed */
    LEB_EDEVICE = -3,    /* HIP runtime error on launch */
    LEB_ENOTSUP = -4     /* dynamics kind or size not supported */
} leb_status;

/* per-unit flags (uint32, OR of): */
#define LEB_FLAG_UNBOUNDED       1u  /* an enclosure needed 1/x over x containing 0 (spring of zero length) */
#define LEB_FLAG_BAD_INPUT       2u  /* non-finite nominal/mu/sigma or negative sigma: all rows [-inf, inf] */
#define LEB_FLAG_HULL_EXTENDED   4u  /* |mu_i| > sigma_i: box extended to contain the nominal point */

typedef enum {
    LEB_DYN_LINEAR = 0,        /* affine dynamics: the remainder is identically 0 */
    LEB_DYN_PQUAD_CHAIN = 4    /* planar quadrotors (1 = a single one) joined by springs */
} leb_dyn_kind;

/* Analytic dynamics, forward-Euler discretised (dynamics appendix,
 * "Planar Quadrotor"):  x+ = x + dt * xdot, per node i
 *   xdot = [vx, vz, omega, -(u1+u2) sin(theta)/m + Fx_i/m,
 *           (u1+u2) cos(theta)/m - g + Fz_i/m, (u1-u2) arm/inertia],
 * with the spring force between nodes i and i+1
 *   F = k_spring (|d| - rest_len) d / |d|,  d = (rest_len + px_{i+1} - px_i, pz_{i+1} - pz_i)
 * acting +F on node i and -F on node i+1.  State per node
 * (px, pz, theta, vx, vz, omega), input per node (u1, u2); the augmented
 * vector is [all node states; all node inputs] and this order defines the
 * coordinate-wise path of Theorem 1. */
typedef struct {
    int32_t kind;       /* leb_dyn_kind */
    int32_t nx, nu;     /* LINEAR: any sizes; CHAIN: must equal 6*n_units, 2*n_units */
    int32_t n_units;    /* CHAIN: 1 .. 256 */
    double dt, m, g, arm, inertia, k_spring, rest_len;   /* CHAIN: dt > 0, m > 0, k_spring >= 0, rest_len >= 0 */
} leb_dynamics;

/*
 * leb_analytic_bound -- path-based Hessian bound (Theorem 1, eq.
 * path_based_hessian) for every unit:
 *   R_l = sum_{j<k} [H_l,kj](X^(j)) (Delta_j Delta_k) + 1/2 sum_k [H_l,kk](X^(k)) Delta_k^2
 * over prefix boxes X^(p) of the coordinate-wise path, and its zonotope
 * packaging (eq. zono_map) c_bar = (lo+hi)/2, rho_bar = (hi-lo)/2 + pad.
 *
 *   dyn      host pointer
 *   batch, N number of trajectories and timesteps (0 is allowed: no work)
 *   z        [batch][N][nx]   nominal states z_k (k in [N]; z_N is not an input)
 *   v        [batch][N][nu]   nominal inputs v_k (may be NULL when nu == 0)
 *   mu       [batch][N][nx+nu] tube centre offsets, NULL means 0
 *   sigma    [batch][N][nx+nu] tube radii (>= 0)
 *   r_lo, r_hi [batch][N][nx] outputs (FP64, outward-rounded)
 *   c_bar, rho_bar [batch][N][nx] optional outputs (NULL to skip); rho_bar
 *            includes the diagonal padding `pad` (>= 0) that keeps the
 *            zonotope generator right-invertible (section V.A)
 *   flags    [batch][N] optional per-unit flags (NULL to skip)
 * Returns LEB_OK or a negative leb_status.
 */
int leb_analytic_bound(const leb_dynamics* dyn, int32_t batch, int32_t N,
                       const double* z, const double* v, const double* mu, const double* sigma,
                       double* r_lo, double* r_hi, double* c_bar, double* rho_bar, double pad,
                       uint32_t* flags, void* stream);

/*
 * leb_backward -- adjoint of leb_analytic_bound: the gradient of
 *     L = sum_{unit, row} g_lo r_lo + g_hi r_hi
 * with respect to z, v, sigma (and mu) for the exact-arithmetic path-based
 * bound (rounding treated as the identity; at ties between candidate
 * endpoints the first in the order lo*lo, lo*hi, hi*lo, hi*hi is used).
 * The paper differentiates the bound to refine the nominal point
 * (Table II) and to penalise propagated error (eq.
 * linearization_error_cost_penalty).  Interval intermediates are
 * recomputed, not stored.
 *   g_lo, g_hi [batch][N][nx]     upstream adjoints of r_lo, r_hi
 *   gz [batch][N][nx], gv [batch][N][nu], gsigma [batch][N][nx+nu] outputs
 *   gmu [batch][N][nx+nu] output, may be NULL; must be NULL when mu is NULL
 * Rows whose bound is unbounded and units with invalid data contribute 0.
 * Chains up to 128 nodes (LEB_ENOTSUP beyond).  Deterministic: per-
 * coordinate sums are taken in a fixed order.
 */
int leb_backward(const leb_dynamics* dyn, int32_t batch, int32_t N, const double* z, const double* v,
                 const double* mu, const double* sigma, const double* g_lo, const double* g_hi,
                 double* gz, double* gv, double* gmu, double* gsigma, void* stream);

/*
 * leb_tube_map -- tube centre and width from the residual zonotopes
 * (eqs. tight_tube_center, tight_tube_width):
 *   mu_k    = sum_{j<k} Phi_{k,j} c_bar_j
 *   sigma_k = sum_{j<k} |Phi_{k,j}| (e + rho_bar_j) = sum_j ||Phi_{k,j} [E diag(rho_bar_j)]||_{1,r}
 * for chains of n_units nodes with a decentralised, lag-invariant closed
 * loop: phi [N-1][8][6] (device) is the per-node block for lag d = k-j
 * (rows 0..5: the node's state rows of the tube; rows 6..7: its input
 * rows; columns: the node's residual rows), shared by every node and
 * trajectory.  e (host, 6 values >= 0) is the per-node disturbance
 * magnitude |E| 1.  c_bar, rho_bar [batch][N][6*n_units]; mu, sigma
 * [batch][N][8*n_units] outputs.  sigma is rounded upward and also covers
 * the rounding of mu.
 */
int leb_tube_map(int32_t batch, int32_t N, int32_t n_units, const double* phi, const double* e,
                 const double* c_bar, const double* rho_bar, double* mu, double* sigma, void* stream);

typedef struct {
    double tol;            /* stop when max |change| / sigma <= tol (e.g. 1e-6) */
    int32_t max_sweeps;    /* cap on bound sweeps (plain LEB evaluations of all steps) */
    double pad;            /* zonotope radius padding (>= 0) */
    double inflate_rel;    /* candidate tube: sigma (1 + inflate_rel) + inflate_abs */
    double inflate_abs;
    int32_t warm;          /* 1: start from the (mu, sigma) passed in; 0: disturbance-only tube */
} leb_fp_options;

/*
 * leb_fixed_point_solve -- certified tube/LEB fixed point for chain
 * dynamics (the loop of section V: bound -> zonotope -> tube map, until
 * the tube stops changing; Theorem 3 gives containment of the reachable
 * set in the tube).  Jacobi sweeps bound every (trajectory, step) at once
 * with leb_analytic_bound's kernel, then apply leb_tube_map.  After the
 * change falls below tol, the tube is inflated and accepted only if
 * F(B) lies inside B for every trajectory (a post-fixed point of the
 * inclusion-isotone map F: this certifies it); otherwise iteration goes on.
 *   z, v    [batch][N][nx], [batch][N][nu] nominal trajectories
 *   phi, e  as leb_tube_map
 *   mu, sigma [batch][N][nx+nu] in/out: warm start in (opt->warm), certified tube out
 *   certified [batch] device uint32 out: 1 = certified, 0 = sweep cap reached
 *   sweeps_out host int32 out: number of bound sweeps, including the certifying one
 * Synchronises `stream` once per sweep (the convergence test reads one
 * value per trajectory).  Uses a library-owned, grow-only device workspace
 * (kept until process exit); calls from several host threads serialise.
 */
int leb_fixed_point_solve(const leb_dynamics* dyn, int32_t batch, int32_t N, const double* z,
                          const double* v, const double* phi, const double* e, const leb_fp_options* opt,
                          double* mu, double* sigma, uint32_t* certified, int32_t* sweeps_out, void* stream);

/* Human-readable text of a leb_status code (static storage). */
const char* leb_strerror(int code);

/* Library version string (static storage). */
const char* leb_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LEB_H */
