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
    LEB_ENOTSUP = -4,    /* dynamics kind or size not supported */
    LEB_ESCRATCH = -5    /* the problem does not fit the fixed scratch of a no-allocation entry point */
} leb_status;

/* per-unit flags (uint32, OR of): */
#define LEB_FLAG_UNBOUNDED       1u  /* an enclosure needed 1/x over x containing 0 (spring of zero length) */
#define LEB_FLAG_BAD_INPUT       2u  /* non-finite nominal/mu/sigma or negative sigma: all rows [-inf, inf] */
#define LEB_FLAG_HULL_EXTENDED   4u  /* |mu_i| > sigma_i: box extended to contain the nominal point */

typedef enum {
    LEB_DYN_LINEAR = 0,        /* affine dynamics: the remainder is identically 0 */
    LEB_DYN_QUADRATIC = 1,     /* f_l(a) = 1/2 a^T Q_l a + affine: constant Hessian Q_l */
    LEB_DYN_SINCOS = 2,        /* nx = 1: f = sin(a_1); nx = 2: f = (sin a_1 cos a_2, cos a_1 sin a_2); nu = 0 */
    LEB_DYN_PQUAD_CHAIN = 4,   /* planar quadrotors (1 = a single one) joined by springs */
    LEB_DYN_SATELLITE = 5,     /* satellite attitude (dynamics appendix): nx = 7, nu = 3 */
    LEB_DYN_QUAD3D = 6         /* 3-D quadrotor (dynamics appendix): nx = 12, nu = 4 */
} leb_dyn_kind;

/* Interval-Hessian forms of leb_interval_hessian_bound (section IV.A) */
#define LEB_IH_PATH     0   /* Theorem 1: entries over the prefix boxes of the coordinate-wise path */
#define LEB_IH_EXPAND   1   /* eq. expanded_interval_hessian: the same sum, every entry over the full box */
#define LEB_IH_CLASSIC  2   /* eq. interval_quadratic_form: 1/2 Delta^T ([H](X) Delta) */

/* Analytic dynamics, forward-Euler discretised (dynamics appendix,
 * "Planar Quadrotor"):  x+ = x + dt * xdot, per node i
 *   xdot = [vx, vz, omega, -(u1+u2) sin(theta)/m + Fx_i/m,
 *           (u1+u2) cos(theta)/m - g + Fz_i/m, (u1-u2) arm/inertia],
 * with the spring force between nodes i and i+1
 *   F = k_spring (|d| - rest_len) d / |d|,  d = (rest_len + px_{i+1} - px_i, pz_{i+1} - pz_i)
 * acting +F on node i and -F on node i+1.  State per node
 * (px, pz, theta, vx, vz, omega), input per node (u1, u2); the augmented
 * vector is [all node states; all node inputs] and this order defines the
 * coordinate-wise path of Theorem 1.
 *
 * SATELLITE: a = (q0, q1, q2, q3, w1, w2, w3, v1, v2, v3), x+ = x + dt xdot with
 *   qdot = zeta(w) q,  zeta(w) = 1/2 [[0,-w1,-w2,-w3],[w1,0,w3,-w2],[w2,-w3,0,w1],[w3,w2,-w1,0]],
 *   wdot = I^-1 (v - w x (I w)),  I = diag(J[0], J[1], J[2]).
 * QUAD3D: a = (px, py, pz, phi, theta, psi, vx, vy, vz, p, q, r, T, tau_phi,
 *   tau_theta, tau_psi), x+ = x + dt xdot with the Euler-angle kinematics
 *   (phidot = p + (q sin phi + r cos phi) tan theta, thetadot = q cos phi - r sin phi,
 *   psidot = (q sin phi + r cos phi) / cos theta), vdot = (T/m) R e_3 - g e_3 and the
 *   rigid-body rates (pdot = (Jy - Jz)/Jx q r + tau_phi/Jx, ...), J = (Jx, Jy, Jz).
 *   Rows whose Hessian involves 1/cos(theta) are unbounded (LEB_FLAG_UNBOUNDED) where
 *   the cos(theta) interval of the evaluation box is not positive. */
typedef struct {
    int32_t kind;       /* leb_dyn_kind */
    int32_t nx, nu;     /* LINEAR: any sizes; CHAIN: must equal 6*n_units, 2*n_units;
                           QUADRATIC: 1 <= nx + nu <= 64; SINCOS: nx in {1, 2}, nu = 0;
                           SATELLITE: 7, 3; QUAD3D: 12, 4 */
    int32_t n_units;    /* CHAIN: 1 .. 256 */
    double dt, m, g, arm, inertia, k_spring, rest_len;   /* CHAIN: dt > 0, m > 0, k_spring >= 0, rest_len >= 0;
                                                            SATELLITE: dt > 0; QUAD3D: dt > 0, m > 0 (g enters
                                                            no Hessian) */
    const double* coeffs;  /* QUADRATIC: DEVICE pointer to Q [nx][nx+nu][nx+nu] (row l holds Q_l; only the
                              entries k >= j are read, as the lower triangle of a symmetric matrix, and each
                              must be finite); NULL for every other kind */
    double J[3];        /* SATELLITE: inertia diagonal I_S; QUAD3D: (Jx, Jy, Jz); all > 0 */
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
 *   r_lo, r_hi [batch][N][nx] outputs (FP64, outward-rounded); may both be
 *            NULL when c_bar and rho_bar are given
 *   c_bar, rho_bar [batch][N][nx] optional outputs (NULL to skip); rho_bar
 *            includes the diagonal padding `pad` (>= 0) that keeps the
 *            zonotope generator right-invertible (section V.A)
 *   flags    [batch][N] optional per-unit flags (NULL to skip)
 *   A, B     optional outputs (NULL to skip; CHAIN dynamics only, LEB_EINVAL
 *            otherwise): the point Jacobians of the discretised dynamics at
 *            the nominal (eq. linearizations), A [batch][N][nx][nx] = df/dx,
 *            B [batch][N][nx][nu] = df/du, row-major, FP64 (round to nearest;
 *            they define the linearization, they are not enclosures).  Every
 *            entry is written.
 * Kinds: CHAIN (nodes in one workgroup, FP32 outward intervals, FP64
 * accumulation); LINEAR ([0, 0] for valid data); QUADRATIC and SINCOS,
 * closed-form test dynamics, SATELLITE and QUAD3D (one thread per unit, the
 * same arithmetic; QUADRATIC reads Q through dyn->coeffs).  Invalid data (non-finite nominal, mu or sigma, negative
 * sigma) gives [-inf, +inf] on every row of the unit and LEB_FLAG_BAD_INPUT
 * for every kind; z and sigma (and v when nu > 0) are required for every kind.
 * Returns LEB_OK or a negative leb_status.
 */
int leb_analytic_bound(const leb_dynamics* dyn, int32_t batch, int32_t N,
                       const double* z, const double* v, const double* mu, const double* sigma,
                       double* r_lo, double* r_hi, double* c_bar, double* rho_bar, double pad,
                       uint32_t* flags, double* A, double* B, void* stream);

/*
 * leb_interval_hessian_bound -- the three interval-Hessian enclosures the
 * paper compares (section IV.A; Corollary 1 orders them: for a box symmetric
 * about the nominal point PATH is inside EXPAND, which is inside CLASSIC):
 *   mode LEB_IH_PATH    Theorem 1 (the same bound as leb_analytic_bound)
 *   mode LEB_IH_EXPAND  eq. expanded_interval_hessian: sum_{j<k} [H_kj](X) (Delta_j Delta_k)
 *                       + 1/2 sum_k [H_kk](X) Delta_k^2
 *   mode LEB_IH_CLASSIC eq. interval_quadratic_form: 1/2 Delta^T v with v = [H](X) Delta
 *                       over the symmetric interval Hessian
 * for the kinds LINEAR, QUADRATIC, SINCOS, SATELLITE, QUAD3D (CHAIN:
 * LEB_ENOTSUP).  Arguments, layout, flags and invalid-data handling as in
 * leb_analytic_bound; r_lo, r_hi are required.  LEB_EINVAL for another mode.
 */
int leb_interval_hessian_bound(const leb_dynamics* dyn, int32_t mode, int32_t batch, int32_t N,
                               const double* z, const double* v, const double* mu, const double* sigma,
                               double* r_lo, double* r_hi, uint32_t* flags, void* stream);

/*
 * leb_sample_remainder -- the random-sampling under-approximation of the
 * remainder that the tightness study compares against (results section):
 * for every unit, the minimum and maximum over K points
 *     a_s = a~ + mu + t_s * sigma   (elementwise; t_s in [-1, 1]^(nx+nu), caller-drawn)
 * and the nominal point itself (r = 0) of
 *     r_l(a; a~) = f_l(a) - f_l(a~) - J_l(a~) (a - a~)      (eq. linear_error_def)
 * evaluated in FP64 (QUADRATIC: its exact form 1/2 d^T Q_l d).
 *   t              DEVICE [K][nx+nu], shared by every unit
 *   s_lo, s_hi     [batch][N][nx] outputs
 * Kinds QUADRATIC, SINCOS, SATELLITE, QUAD3D with nx + nu <= 16 (else
 * LEB_ENOTSUP).  One workgroup per unit; the result is an estimate from
 * inside, not a bound.
 */
int leb_sample_remainder(const leb_dynamics* dyn, int32_t batch, int32_t N, const double* z, const double* v,
                         const double* mu, const double* sigma, int32_t K, const double* t, double* s_lo,
                         double* s_hi, void* stream);

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
 * leb_pgd_nominal -- refinement of the nominal (linearization) point (the
 * nominal-point optimization of the results section, Table II): projected
 * gradient descent on the width
 *     W(a~) = sum_l (r_hi,l - r_lo,l)
 * of the path-based bound linearized at a~, searching a~ in a0 +/- radius sigma
 * (a0 = [z0; v0], the start; 0 <= radius <= 1).  The set the bound covers is
 *   fixed_box = 0: the travelling box a~ + mu0 +/- sigma (a fixed perturbation
 *     radius around the nominal point, the paper's setting): dW/da~ = dW/dz;
 *   fixed_box = 1: the fixed box (a0 + mu0) +/- sigma, passed as
 *     a~ + mu +/- sigma with mu = a0 + mu0 - a~: dW/da~ = dW/dz - dW/dmu
 *     (keep |mu0| + radius sigma <= sigma so that a~ stays inside the box),
 * derivatives from the adjoint of leb_backward.  Step s moves each coordinate
 * by lr radius sigma_i (1 - s / steps) against the sign of its derivative
 * (not at all where it is 0) and projects onto the search box; `steps` steps
 * take steps + 1 bound and `steps` adjoint evaluations.  CHAIN dynamics (as
 * leb_backward).
 *   z0, v0, sigma  [batch][N][nx], [batch][N][nu], [batch][N][nx+nu]
 *   mu0            [batch][N][nx+nu] or NULL (0): box centre offset
 *   z, v           outputs: the narrowest iterate seen (the start included)
 *   width [batch][N] output: its W; width0 [batch][N] optional: W(a0)
 * LEB_EINVAL for fixed_box not 0/1, radius outside [0, 1], lr not positive
 * and finite, steps < 0.  Uses a library-owned grow-only workspace, ordered
 * across streams like the other workspaces.
 */
int leb_pgd_nominal(const leb_dynamics* dyn, int32_t batch, int32_t N, const double* z0, const double* v0,
                    const double* mu0, const double* sigma, int32_t fixed_box, double radius, int32_t steps,
                    double lr, double* z, double* v, double* width, double* width0, void* stream);

/* Opaque ReLU MLP prepared for the device (weights converted to FP64 and
 * laid out for the kernels).  Owned by the library. */
typedef struct leb_mlp_s* leb_mlp;

/*
 * leb_mlp_create -- upload a ReLU MLP g: z_l = W_l a_{l-1} + b_l,
 * a_l = relu(z_l) (l < n_layers), g = z_{n_layers}.
 *   widths   host [n_layers + 1]: input width, hidden widths, output width.
 *            Every width but the output must be a multiple of 16 and at
 *            most 256; the output at most 64; 2 <= n_layers <= 8.
 *   W, b     host arrays of n_layers host pointers to FP32 [out][in] and
 *            [out] (the FP32 values are used exactly, widened to FP64).
 *   nx       the first nx inputs are the state, the rest the control
 *   residual 1: dynamics f(x, u) = x + g(x, u) (needs nx == output width);
 *            the remainder is then that of g.
 * Synchronous (copies to the device).  *out receives the handle.
 */
int leb_mlp_create(int32_t n_layers, const int32_t* widths, const float* const* W, const float* const* b,
                   int32_t nx, int32_t residual, leb_mlp* out);
int leb_mlp_destroy(leb_mlp net);

/*
 * leb_nn_bound -- remainder bound of ReLU-MLP dynamics (section IV.B): CROWN
 * affine bounds over the box (full CROWN for every hidden layer's
 * pre-activation bounds; adaptive lower slopes) and Theorem 2 with the
 * local Jacobian J = J_g(a~) (relu'(0) = 0).  All contractions in FP64 on
 * MFMA with a rounding allowance, so the bound is sound.
 *   z [batch][N][nx], v [batch][N][nu], mu (NULL = 0) and sigma
 *   [batch][N][nx+nu], outputs r_lo, r_hi (and optional c_bar, rho_bar)
 *   [batch][N][m], flags [batch][N] (optional), as leb_analytic_bound.
 *   J        [batch][N][m][nx+nu] (FP64) or NULL: the matrix of the
 *            linearization.  NULL: the network's Jacobian at the nominal,
 *            computed by the library.  Given: Theorem 2 with this J (it holds
 *            for any J), so the bound encloses g(a) - g(a~) - J (a - a~);
 *            a unit whose J has a non-finite entry gets [-inf, +inf] on every
 *            row and LEB_FLAG_BAD_INPUT.
 * Uses a library-owned grow-only workspace (about 800 MB at the largest
 * chunk of 4096 boxes of a 256-wide network).  Calls from several host threads serialise on the
 * host, and a call's kernels wait (on the device) for those of the previous
 * call that used the workspace, whatever its stream.
 */
int leb_nn_bound(leb_mlp net, int32_t batch, int32_t N, const double* z, const double* v, const double* mu,
                 const double* sigma, const double* J, double* r_lo, double* r_hi, double* c_bar, double* rho_bar,
                 double pad, uint32_t* flags, void* stream);

/*
 * leb_nn_backward -- adjoint of leb_nn_bound (the differentiable bound of
 * section IV.D, for the ReLU-MLP bound of section IV.B): the gradient of
 *     L = sum_{unit, row} g_lo r_lo + g_hi r_hi
 * with respect to z, v, sigma (and mu) for the exact-arithmetic bound with
 * J = J_g(a~) (rounding allowances are not differentiated; J a~ - g(a~)
 * contributes 0, J being constant between kinks).  The bound is piecewise
 * smooth; at ties the branch taken is: a CROWN coefficient of exactly 0 counts
 * as non-negative, sign(0) = 0 in d|x|, the clamp min(mu - sigma, 0) passes
 * the derivative only where mu - sigma < 0 and max(mu + sigma, 0) only where
 * mu + sigma > 0, and a neuron is unstable when lo < 0 < hi.
 *   z [batch][N][nx], v [batch][N][nu], mu (NULL = 0), sigma [batch][N][nx+nu]
 *   g_lo, g_hi [batch][N][m]       upstream adjoints of r_lo, r_hi
 *   gz, gv, gsigma                 outputs, shaped as z, v, sigma
 *   gmu [batch][N][nx+nu]          output, may be NULL; must be NULL when mu is NULL
 * Units with invalid data (non-finite input, sigma < 0) get a zero gradient.
 * Every pass is recomputed (nothing of leb_nn_bound is reused), in FP64 (on
 * MFMA for networks with at most three hidden layers, on the VALU beyond).
 * Deterministic: every sum is taken in a fixed order.  Uses a library-owned
 * grow-only workspace of up to about 8.6 GB (it holds the CROWN coefficients
 * of the passes of up to 4,096 boxes: 1.34 MB per box of a 16-256-256-256-12
 * network; deep, wide networks take fewer boxes at a time), ordered across
 * streams like the other workspaces.
 * LEB_EINVAL for null or misaligned pointers or gmu without mu.
 */
int leb_nn_backward(leb_mlp net, int32_t batch, int32_t N, const double* z, const double* v, const double* mu,
                    const double* sigma, const double* g_lo, const double* g_hi, double* gz, double* gv,
                    double* gmu, double* gsigma, void* stream);

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
 * the rounding of mu.  A residual that is not finite (c_bar or rho_bar) at
 * step j makes sigma +inf at every later step of that node.  Horizons up
 * to N = 83 (LEB_ENOTSUP beyond: a workgroup keeps the residuals of all
 * steps of its 16 nodes in LDS).
 */
int leb_tube_map(int32_t batch, int32_t N, int32_t n_units, const double* phi, const double* e,
                 const double* c_bar, const double* rho_bar, double* mu, double* sigma, void* stream);

/*
 * leb_zonotope_hull -- interval hull of zonotopes (eq. tight_tube_width):
 * for each row i of a zonotope {c + G xi : |xi|_inf <= 1} with generator
 * matrix G [rows][n_gen] (row-major) and centre c [rows],
 *     mu[i] = c[i],    sigma[i] = ||G_i||_1 = sum_j |G_ij|   (rounded upward).
 * rows >= 0, n_gen >= 0 (0: sigma = 0); c may be NULL (mu = 0).  A row with a
 * non-finite generator entry gets sigma = +inf.  One wave per row.
 */
int leb_zonotope_hull(int32_t rows, int32_t n_gen, const double* G, const double* c, double* mu, double* sigma,
                      void* stream);

typedef struct {
    double tol;            /* relative inflation per sweep (>= 0, e.g. 1e-6) */
    int32_t max_sweeps;    /* cap on bound sweeps (plain LEB evaluations of all steps), >= 1 */
    double pad;            /* zonotope radius padding (>= 0) */
    double inflate_abs;    /* absolute inflation per sweep (> 0); floor of the relative change */
    int32_t warm;          /* 1: start from the (mu, sigma) passed in; 0: disturbance-only tube */
    double conv_tol;       /* acceptance also needs convergence: the next iterate C' differs from C by at
                              most |sigma' - sigma| <= conv_tol sigma + 2 inflate_abs and
                              |mu' - mu| <= conv_tol sigma + inflate_abs, per entry (>= tol).  From the
                              cold start (below the fixed point) every certified iterate meets this with
                              conv_tol = tol; a warm start above the fixed point keeps sweeping until it does */
} leb_fp_options;

/*
 * leb_fixed_point_solve -- certified tube/LEB fixed point for chain
 * dynamics (the loop of section V, Nonlinear SLS Formulation: bound ->
 * zonotope -> tube map, until the change of the iterates falls below a
 * threshold; Theorem 3 gives containment of the reachable set in the
 * tube).  Each sweep bounds every (trajectory, step) at once with
 * leb_analytic_bound's kernel and applies leb_tube_map: C' = F(C).  A tube
 * C is certified when F(C) lies inside C for every step (a post-fixed
 * point of the inclusion-isotone map F, so the Theorem 3 induction goes
 * through).  Iteration: C <- F(C) (1 + tol) + inflate_abs on sigma
 * (mu <- mu_F), which converges, by causality of F, in at most N + 1 sweeps
 * to a tube about tol above the least fixed point.  Each trajectory is
 * accepted (frozen) at the first iterate C that is certified and converged
 * (opt->conv_tol): from the cold start or any warm start the accepted tube
 * lies within about conv_tol of the least fixed point's neighbourhood
 * reached by the cold start.
 *   z, v    [batch][N][nx], [batch][N][nu] nominal trajectories
 *   phi, e  as leb_tube_map
 *   mu, sigma [batch][N][nx+nu] in/out: warm start in (opt->warm), certified tube out
 *   certified [batch] device uint32 out: 1 = certified, 0 = sweep cap reached first
 *   sweeps_out host int32 out: number of bound sweeps, including the certifying one
 * The host reads one open-trajectory count per sweep from pinned memory
 * (published by the next sweep's bound launch) while one sweep stays in
 * flight; it never synchronises `stream`.  On return the certificate
 * flags and the tube are enqueued on `stream`.  Horizons up to N = 210
 * (LEB_ENOTSUP beyond).  Options, e and N are checked before any launch
 * (LEB_EINVAL, LEB_ENOTSUP).  Device pointers must be 8-byte aligned.
 * Uses a library-owned, grow-only device workspace (kept until process
 * exit).  Calls from several host threads serialise on the host, and a
 * call's kernels wait (on the device) for those of the previous call that
 * used the workspace, whatever its stream.
 */
int leb_fixed_point_solve(const leb_dynamics* dyn, int32_t batch, int32_t N, const double* z,
                          const double* v, const double* phi, const double* e, const leb_fp_options* opt,
                          double* mu, double* sigma, uint32_t* certified, int32_t* sweeps_out, void* stream);

/*
 * leb_fixed_point_solve_noalloc -- leb_fixed_point_solve for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): same arguments, same kernels and
 * bitwise the same mu, sigma and certified flags.  It calls no hipMalloc,
 * hipFree or other allocating routine and never reads back from the device:
 *   - its workspace is a library-owned static device array of 64 MiB, one
 *     per GPU, held until the process ends; a problem needs
 *     2 B N (16 n_units + 8 (nx + nu)) + 8 (B + 1) bytes (each part rounded up to
 *     256), and one that needs more returns LEB_ESCRATCH before any launch
 *     (256 x 40 x 224: 46 MB);
 *   - all opt->max_sweeps sweeps are enqueued (a sweep after every trajectory
 *     is accepted exits at once), so *sweeps_out = opt->max_sweeps, the
 *     sweeps enqueued; the certificate flags tell which trajectories were
 *     accepted within them.
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (other host threads, or other streams before the first call's kernels
 * finish) race and corrupt each other's results; the caller orders them.
 * The array keeps the last call's contents; nothing in it needs clearing
 * (the first sweep writes every state word it reads).
 */
int leb_fixed_point_solve_noalloc(const leb_dynamics* dyn, int32_t batch, int32_t N, const double* z,
                                  const double* v, const double* phi, const double* e, const leb_fp_options* opt,
                                  double* mu, double* sigma, uint32_t* certified, int32_t* sweeps_out, void* stream);

/*
 * Launch timing of the fixed-point sweeps (instrumentation, off by default).
 * leb_launch_timing(1) clears the record and starts timing; from then on
 * leb_fixed_point_solve (and leb_fixed_point_learned) launch each sweep's
 * bound kernel (kernel 0) and tube-map kernel (kernel 1) with a pair of HIP
 * events taken at the kernel's start and end, up to 256 launches each;
 * leb_launch_timing(0) stops.  leb_launch_times writes the durations in ms of kernel's recorded
 * launches, in launch order, to ms[0 .. min(count, cap)) (waiting for them)
 * and their number to *count.  A sweep enqueued after the certifying one
 * exits at once and is recorded too.
 */
int leb_launch_timing(int32_t enable);
int leb_launch_times(int32_t kernel, float* ms, int32_t cap, int32_t* count);

/*
 * Learned warm start (not a step of the paper: a surrogate network that
 * starts the section-V fixed point from a predicted tube; every accepted
 * tube is still certified by the plain bound).  A GELU MLP with widths [d_0, ..., d_L] (L <= 8, every width in
 * 1..256), FP32 master parameters and BF16 MFMA arithmetic with FP32
 * accumulation:
 *   a_0 = bf16(x); z_l = bf16(W_l) a_{l-1} + b_l; a_l = bf16(gelu(z_l));
 *   y = bf16(W_L) a_{L-1} + b_L,    gelu(z) = z Phi(z) (exact form).
 * Parameters are one flat FP32 array [W_1, b_1, ..., W_L, b_L], W_l row-major
 * [d_l][d_{l-1}].  The object owns its device parameters, Adam moments,
 * BF16 weight copies and a grow-only training workspace; calls on one
 * object must not overlap (they serialise on an internal lock where they
 * use the workspace).
 */
typedef struct leb_surrogate_s* leb_surrogate;

/* Uploads params_host (host, leb_surrogate_n_params values); Adam moments start at 0. */
int leb_surrogate_create(int32_t n_layers, const int32_t* widths, const float* params_host, leb_surrogate* out);
int leb_surrogate_destroy(leb_surrogate s);
/* Number of FP32 parameters (-1 for NULL). */
int64_t leb_surrogate_n_params(leb_surrogate s);
/* Synchronises the device and downloads the FP32 parameters to params_host. */
int leb_surrogate_params(leb_surrogate s, float* params_host);

/* Inference: y [batch][d_L] = net(x [batch][d_0]) (device FP32). */
int leb_mlp_fwd_bf16(leb_surrogate s, int32_t batch, const float* x, float* y, void* stream);

/* Gradient of sum(dy . net(x)) with respect to the parameters, written to
 * grads (device FP32, the parameter layout).  batch must be a multiple of 32. */
int leb_mlp_bwd_bf16(leb_surrogate s, int32_t batch, const float* x, const float* dy, float* grads, void* stream);

/* One Adam step (Kingma and Ba, Algorithm 1; step >= 1 is the bias-
 * correction index) with the given device gradient; refreshes the BF16
 * copies.  The moments and parameters are FP32; lr / (1 - beta1^step),
 * 1 / sqrt(1 - beta2^step) and 1 - beta are formed in FP64. */
int leb_adam_step(leb_surrogate s, const float* grads, int32_t step, double lr, double beta1, double beta2,
                  double eps, void* stream);

/* Forward, mean-squared error against t [batch][d_L], backward and Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8) in one call.  loss (device, 1 float,
 * may be NULL) receives the mean-squared error before the update.  batch
 * must be a multiple of 32. */
int leb_surrogate_train_step(leb_surrogate s, int32_t batch, const float* x, const float* t, int32_t step, double lr,
                             float* loss, void* stream);

/* Input and output widths of a surrogate (d_0 and d_L). */
int leb_surrogate_dims(leb_surrogate s, int32_t* d_in, int32_t* d_out);

/*
 * Chain surrogate: for node i of a chain at one timestep, the bound of its
 * two non-linear rows (vx_i+, vz_i+) is regressed on what the path-based
 * bound of those rows depends on (Theorem 1 over the prefix boxes of the
 * node's attitude block and of its two springs).  With
 * Delta_c = [min(mu_c - sigma_c, 0), max(mu_c + sigma_c, 0)] scaled by 20:
 *   x[0..11]  theta_i, (u1_i + u2_i) / 10, Delta of theta_i, u1_i, u2_i,
 *             px_i, pz_i (lo, hi each)
 *   x[12..18] right spring: present (1/0), separation (L0 + px_{i+1} - px_i,
 *             pz_{i+1} - pz_i), Delta of px_{i+1}, pz_{i+1}  (zeros if absent)
 *   x[19..25] left spring: the same for node i-1 (separation from i-1 to i)
 *   x[26..31] 0 (rows are 128 bytes)
 * Targets: log(max(hi, 1e-14)), log(max(-lo, 1e-14)) of the vx row, then of
 * the vz row.
 */
#define LEB_CHAIN_FEATURES 32
#define LEB_CHAIN_OUTPUTS 4

/* x [batch][N][n_units][32] (device FP32, 16-byte aligned) from the
 * nominal trajectory and the tube (mu may be NULL). */
int leb_chain_features(const leb_dynamics* dyn, int32_t batch, int32_t N, const double* z, const double* v,
                       const double* mu, const double* sigma, float* x, void* stream);
/* t [batch][N][n_units][4] (device FP32, 16-byte aligned) from a bound r_lo, r_hi [batch][N][nx]. */
int leb_chain_targets(const leb_dynamics* dyn, int32_t batch, int32_t N, const double* r_lo, const double* r_hi,
                      float* t, void* stream);

/*
 * leb_chain_surrogate_bound -- the surrogate's residual zonotope for a chain
 * tube (the learned counterpart of leb_analytic_bound's c_bar, rho_bar):
 * features, the BF16 MLP and the decoding hi = exp(min(y_hi, 0)),
 * lo = -exp(min(y_lo, 0)) run in one kernel; c_bar = (lo + hi) / 2 and
 * rho_bar = (hi - lo) / 2 + pad on the vx, vz rows, 0 and pad on the
 * affine rows.  A prediction that is not finite counts as a zero bound.
 * Not a certified bound: it only seeds the certified iteration.
 *   z, v, mu (NULL = 0), sigma as leb_analytic_bound; c_bar, rho_bar [batch][N][nx]
 */
int leb_chain_surrogate_bound(const leb_dynamics* dyn, int32_t batch, int32_t N, const double* z, const double* v,
                              const double* mu, const double* sigma, leb_surrogate net, double* c_bar,
                              double* rho_bar, double pad, void* stream);

/*
 * NN surrogate (the learned start's second family; not a step of the paper): for ReLU-MLP
 * dynamics with n = nx + nu network inputs and m outputs (leb_nn_bound),
 * one box of the network's input is described by 2n features
 *   x[0..n-1]    a~ = [z; v] (the nominal point)
 *   x[n..2n-1]   20 rho, rho = (hi - lo) / 2 of the displacement interval
 *                Delta = [fmin(mu - sigma, 0), fmax(mu + sigma, 0)] (mu NULL: 0;
 *                fmin/fmax ignore a NaN operand)
 * and its regression targets are, per output row r, log(max(hi_r, 1e-14))
 * (r < m) then log(max(-lo_r, 1e-14)) (the bound of Theorem 2 contains 0,
 * so lo <= 0 <= hi).  FP32 rounding of each feature is from the FP64 value;
 * the logarithm is FP32.
 */
#define LEB_NN_MAX_FEATURES 256

/* x [batch][N][2 (nx + nu)] (device FP32, 8-byte aligned) from z [batch][N][nx],
 * v [batch][N][nu], mu (NULL = 0) and sigma [batch][N][nx + nu] (device FP64).
 * LEB_EINVAL: nx < 1, nu < 0, 2 (nx + nu) > LEB_NN_MAX_FEATURES, null or
 * misaligned pointers. */
int leb_nn_features(int32_t nx, int32_t nu, int32_t batch, int32_t N, const double* z, const double* v,
                    const double* mu, const double* sigma, float* x, void* stream);
/* t [batch][N][2m] (device FP32, 8-byte aligned) from a bound r_lo, r_hi [batch][N][m]
 * (device FP64); 1 <= m, 2m <= LEB_NN_MAX_FEATURES. */
int leb_nn_targets(int32_t m, int32_t batch, int32_t N, const double* r_lo, const double* r_hi, float* t,
                   void* stream);
/*
 * leb_nn_surrogate_bound -- the surrogate's predicted bound of each box:
 * features, the BF16 MLP (widths [2 (nx + nu), ..., 2m]) and the decoding
 * hi = exp(min(y_r, 80)), lo = -exp(min(y_{m+r}, 80)); a prediction that is
 * not finite gives 0.  Not a certified bound.
 *   z, v, mu (NULL = 0), sigma as leb_nn_features; r_lo, r_hi [batch][N][m] (device FP64).
 * LEB_EINVAL also when the network's widths do not match.  Uses a library-
 * owned grow-only workspace (batch N (2n + 2m) floats); calls serialise on
 * the host, and calls enqueued on different streams must not overlap on the
 * device (they share the workspace).
 */
int leb_nn_surrogate_bound(leb_surrogate net, int32_t nx, int32_t nu, int32_t batch, int32_t N, const double* z,
                           const double* v, const double* mu, const double* sigma, double* r_lo, double* r_hi,
                           void* stream);

typedef struct {
    leb_surrogate net;     /* widths [32, ..., 4] */
    int32_t sweeps;        /* tube sweeps with surrogate bounds before certification (>= 0) */
    double margin;         /* relative inflation of the surrogate tube's sigma (>= 0) */
} leb_warm_start;

/*
 * leb_fixed_point_learned -- certified tube/LEB fixed point started from a
 * learned tube: from the disturbance-only tube, ws->sweeps tube sweeps use
 * the surrogate's predicted bounds (features -> BF16 MLP -> zonotope ->
 * tube map); sigma is then inflated to sigma (1 + margin) + opt->inflate_abs
 * and passed to leb_fixed_point_solve as a warm start.  Acceptance is
 * unchanged: every accepted tube satisfies F(C) inside C with the plain
 * bound, whatever the surrogate predicted, and has converged to within
 * opt->conv_tol like the cold start's.  Arguments as leb_fixed_point_solve
 * (opt->warm is ignored); sweeps_out counts the certified (plain-bound)
 * sweeps only; the options, e, ws and N are checked before the first
 * surrogate sweep is launched.  Uses a library-owned workspace, ordered on
 * the device across streams like leb_fixed_point_solve's.
 */
int leb_fixed_point_learned(const leb_dynamics* dyn, int32_t batch, int32_t N, const double* z, const double* v,
                            const double* phi, const double* e, const leb_fp_options* opt, const leb_warm_start* ws,
                            double* mu, double* sigma, uint32_t* certified, int32_t* sweeps_out, void* stream);

/*
 * Batching: many uneven problems (analytic chains of any node count, and
 * ReLU-MLP dynamics), each one trajectory of its own horizon N, bounded by
 * one graph launch.  leb_batch_create groups the problems by launch shape
 * (analytic: node count and dynamics constants; MLP: network), picks each
 * group's tile shape by timing candidates on the problems' own data (steps
 * per workgroup for the path-based bound; boxes per chunk for the MLP
 * bound), caches the choice in the text file tune_cache (key: GPU
 * architecture and group shape; NULL: no cache), and captures all launches
 * (analytic and MLP groups on two streams, joined) into a hipGraph.
 * leb_batch_submit replays it on `stream`: every problem's r_lo, r_hi are
 * recomputed from the current contents of its input buffers.
 * The problem buffers are the caller's and must stay allocated, at the same
 * addresses, for the life of the batch; they must hold valid data at
 * creation (the autotuner runs the bounds).  Results are identical to
 * leb_analytic_bound / leb_nn_bound on each problem.  Submits of one batch
 * must not overlap.
 */
typedef enum { LEB_PROBLEM_ANALYTIC = 0, LEB_PROBLEM_NN = 1 } leb_problem_type;
typedef struct {
    int32_t type;                  /* leb_problem_type */
    const leb_dynamics* dyn;       /* analytic: chain dynamics (copied at creation) */
    leb_mlp net;                   /* NN: network (must outlive the batch) */
    int32_t N;                     /* horizon: steps of this trajectory (>= 1) */
    const double* z;               /* [N][nx] */
    const double* v;               /* [N][nu] */
    const double* mu;              /* [N][nx+nu] or NULL */
    const double* sigma;           /* [N][nx+nu] */
    double* r_lo;                  /* [N][nx] out */
    double* r_hi;                  /* [N][nx] out */
} leb_problem;
typedef struct leb_batch_s* leb_batch;

int leb_batch_create(const leb_problem* probs, int32_t count, const char* tune_cache, leb_batch* out);
int leb_batch_submit(leb_batch b, void* stream);
/* Synchronises the device, then frees the graph and the batch's buffers. */
int leb_batch_destroy(leb_batch b);
/* One line per group: kind, shape, problems, steps, chosen tile and whether it came from the cache. */
int leb_batch_info(leb_batch b, char* buf, int32_t len);

/*
 * System-level-synthesis layer: one controller update of section V (the
 * linearization, the closed-loop responses Phi, and the tube with its LEBs).
 * Sizes: nx <= 32 states, 1 <= nu <= 16 inputs, nw <= 64 disturbance
 * columns (LEB_EINVAL beyond); batch <= 65535 trajectories.  All arrays are
 * device FP64, row-major, 8-byte aligned; the caller owns every buffer.
 *
 * leb_linearize -- eq. linearizations for CHAIN dynamics:
 *   A [batch][N][nx][nx] = df/dx, B [batch][N][nx][nu] = df/du at (z_k, v_k),
 *   and, when E is not NULL, E [batch][N][nx][nx + U] = E(z_k) for the
 *   disturbance model E(x) = [diag(e) | T(x)]: e (host, nx values >= 0) the
 *   constant per-state disturbance, T(x) the thrust-magnitude disturbance of
 *   every quadrotor (total thrust (u1 + u2) + thrust w_i, thrust >= 0 in
 *   newtons): column i holds thrust dt/m (-sin theta_i, cos theta_i) on node
 *   i's (vx, vz) rows (eqs. linearization_error_all, linearization_error_dist).
 *   Other kinds: LEB_ENOTSUP.  E needs nx <= 32 (LEB_ENOTSUP beyond).
 */
int leb_linearize(const leb_dynamics* dyn, int32_t batch, int32_t N, const double* z, const double* v,
                  const double* e, double thrust, double* A, double* B, double* E, void* stream);

/*
 * leb_sls_responses -- closed-loop responses of the reformulated SLS problem
 * (eq. fastsls_qp_reform) by the parallel Riccati recursions (appendix on
 * solving for Phi, eqs. backward_prop and forward_prop, with the start
 * Phi^x_{j+1,j} = I of eq. fastsls_qp_cost_reform_init), one workgroup per
 * (trajectory, disturbance time j):
 *   A [batch][N][nx][nx], B [batch][N][nx][nu]   the LTV pairs (A_k, B_k)
 *   qx [batch][N+1][N][nx], qu [batch][N][N][nu] diagonal weights Q^x_{k,j},
 *       Q^u_{k,j} (Q^{ux} = 0; box constraints make Q^T Q of eq.
 *       sls_cost_matrices_tau diagonal); qu > 0 and qx >= 0 make every
 *       Cholesky pivot positive, otherwise that (trajectory, j) gets NaN gains
 *   K [batch][N][N][nu][nx]     out: gains K_{k,j} for j < k < N
 *   phi [batch][N][N][nx+nu][nx] out: Phi_{k,j} = [Phi^x_{k,j}; Phi^u_{k,j}]
 *       for j < k < N (rows 0..nx-1 state, nx.. input responses)
 * Entries with k <= j of K and phi are not written.  FP64 round-to-nearest
 * (the responses define the controller; the tube map bounds their use).
 */
int leb_sls_responses(int32_t nx, int32_t nu, int32_t batch, int32_t N, const double* A, const double* B,
                      const double* qx, const double* qu, double* K, double* phi, void* stream);

/*
 * leb_sls_tube_map -- tube centre and width of time-varying responses (eqs.
 * tight_tube_center, tight_tube_width):
 *   mu_k    = sum_{j<k} Phi_{k,j} c_bar_j
 *   sigma_k = sum_{j<k} || Phi_{k,j} [E_j  diag(rho_bar_j)] ||_{1,r}
 *           = sum_{j<k} |Phi_{k,j} E_j| 1 + |Phi_{k,j}| rho_bar_j
 *   phi as leb_sls_responses (only j < k is read), E [batch][N][nx][nw]
 *   (NULL when nw = 0), c_bar, rho_bar [batch][N][nx]; mu, sigma
 *   [batch][N][nx+nu] outputs (mu_0 = sigma_0 = 0).  sigma is rounded upward
 *   and covers the rounding of mu.  A non-finite input at some j < k makes
 *   row k mu = 0, sigma = +inf.
 */
int leb_sls_tube_map(int32_t nx, int32_t nu, int32_t nw, int32_t batch, int32_t N, const double* phi,
                     const double* E, const double* c_bar, const double* rho_bar, double* mu, double* sigma,
                     void* stream);

/*
 * leb_sls_fixed_point -- the exact tube/LEB fixed point of one controller
 * update (section V loop; Theorem 3): the tube at step k depends on the
 * residual zonotopes of steps j < k only, so steps are taken in order:
 * tube row k (as leb_sls_tube_map), then the path-based bound (as
 * leb_analytic_bound) over the tube set (z_k, v_k) + mu_k +- sigma_k, plus
 * the disturbance error r_dist of eq. interval_r_dist when thrust > 0 (CHAIN
 * only: the last U columns of E are the thrust columns of leb_linearize's
 * model; r_dist encloses (E(x) - E_k) w over the tube's theta interval),
 * then c_bar = (lo + hi)/2, rho_bar = (hi - lo)/2 + pad.  The result is
 * C = F(C) for the upward-rounded map: no further sweep changes it.
 *   z, v [batch][N][nx], [batch][N][nu]; phi, E as leb_sls_tube_map
 *   mu, sigma [batch][N][nx+nu] out: the tube
 *   r_lo, r_hi [batch][N][nx] out (both NULL to skip): remainder enclosures
 *   certified [batch] out (may be NULL): 1 when every tube entry and residual
 *       is finite
 * Kinds CHAIN, SATELLITE, QUAD3D (LEB_ENOTSUP otherwise).  The disturbance
 * part of every tube entry (which does not depend on the bounds) is one launch
 * over all rows; chains whose per-trajectory data fits in 64 KB of LDS then
 * take the whole causal pass in one launch (one workgroup per trajectory),
 * everything else one row launch and one bound launch per step.  All on
 * `stream`, no host synchronisation.  Uses a library-owned, grow-only device
 * workspace; calls serialise on the host and their kernels on the device,
 * like leb_fixed_point_solve.
 */
int leb_sls_fixed_point(const leb_dynamics* dyn, int32_t batch, int32_t N, const double* z, const double* v,
                        const double* phi, int32_t nw, const double* E, double thrust, double pad, double* mu,
                        double* sigma, double* r_lo, double* r_hi, uint32_t* certified, void* stream);

/* Human-readable text of a leb_status code (static storage). */
const char* leb_strerror(int code);

/* Library version string (static storage). */
const char* leb_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LEB_H */
