"""Oracle of the system-level-synthesis layer around the bound -- TEST
INFRASTRUCTURE (only tests, the smoke check and the CPU baseline use it).

Closed-loop responses.  The reformulated SLS problem (eq. fastsls_qp_reform)
splits over the disturbance time j into finite-horizon LQR problems, solved by
the parallel Riccati recursions of the appendix on solving for Phi (eq.
backward_prop): for every j independently, backward over k = N-1 .. j+1 from
P_{N,j} = Q^x_{N,j} (the printed left-hand side of the terminal condition is
read as P),

    S_{k,j}  = Q^u_{k,j} + B_k^T P_{k+1,j} B_k          (G_{k,j} = S^-1)
    Bc_{k,j} = Q^{ux}_{k,j} + B_k^T P_{k+1,j} A_k       (Q^{ux} = 0: box constraints)
    K_{k,j}  = -S_{k,j}^-1 Bc_{k,j}
    P_{k,j}  = Q^x_{k,j} + A_k^T P_{k+1,j} A_k + K_{k,j}^T Bc_{k,j},

then forward (eq. forward_prop with the reformulated start of eq.
fastsls_qp_cost_reform_init): Phi^x_{j+1,j} = I, Phi^u_{k,j} = K_{k,j}
Phi^x_{k,j}, Phi^x_{k+1,j} = (A_k + B_k K_{k,j}) Phi^x_{k,j}.  The weights
Q_{k,j}^T Q_{k,j} of eq. sls_cost_matrices_tau are diagonal for box
constraints G_k = [I; -I] (diag(Q~, R~) plus the dual weights of both
faces), so they are given as diagonals qx [N+1][N][nx], qu [N][N][nu].

Tube.  eqs. tight_tube_center and tight_tube_width:
    mu_k    = sum_{j<k} Phi_{k,j} c_bar_j
    sigma_k = sum_{j<k} || Phi_{k,j} [E_j  diag(rho_bar_j)] ||_{1,r}
            = sum_{j<k} |Phi_{k,j} E_j| 1 + |Phi_{k,j}| rho_bar_j
with Phi_{k,j} = [Phi^x_{k,j}; Phi^u_{k,j}] and E_j = E(z_j).

State-dependent disturbance (eqs. linearization_error_dist and
interval_r_dist): r_dist_k = (E(x_k) - E_k) w_k lies in ([E](Omega^x_k) - E_k)
times the unit box, i.e. in +-s with s_i = sum_m mag([E]_im(Omega^x_k) - E_k,im).
The state-dependent model used here: a thrust-magnitude disturbance of every
planar quadrotor of a chain, total thrust (u1 + u2) + thrust w_i, which after
explicit Euler gives node i the column thrust dt/m (-sin theta_i, cos theta_i)
on its (vx, vz) rows.  The full disturbance matrix is E(x) = [diag(e) | E_T(x)]
(nw = nx + U); only those two entries of each thrust column depend on the
state, every other entry of E(x) is the nominal matrix's.

Fixed point: one sequential sweep over k is exact (the tube at k depends on
the bounds at j < k only); the bound at k is taken over the tube set
Omega_k = z_k + mu_k +- sigma_k (the oracle's path-based bound, section
IV.A), packaged as c_bar = (lo + hi)/2, rho_bar = (hi - lo)/2 + s + pad.
Plain FP64 (numpy).
"""
from __future__ import annotations

import numpy as np

from . import Dyn, icos, isin, leb as _leb


# ------------------------------------------------------------ responses

def riccati(A, B, qx, qu):
    """A [N][nx][nx], B [N][nx][nu] (one trajectory); qx [N+1][N][nx] and
    qu [N][N][nu] the diagonal weights.  Returns the gains K [N][N][nu][nx]
    and cost-to-go matrices P [N+1][N][nx][nx] (entries (k, j) with
    k > j; zero elsewhere)."""
    N, nx, _ = A.shape
    nu = B.shape[2]
    K = np.zeros((N, N, nu, nx))
    Ps = np.zeros((N + 1, N, nx, nx))
    for j in range(N):
        P = np.diag(qx[N, j]).astype(np.float64)
        Ps[N, j] = P
        for k in range(N - 1, j, -1):
            S = np.diag(qu[k, j]) + B[k].T @ P @ B[k]
            Bc = B[k].T @ P @ A[k]
            Kk = -np.linalg.solve(S, Bc)
            P = np.diag(qx[k, j]) + A[k].T @ P @ A[k] + Kk.T @ Bc
            K[k, j] = Kk
            Ps[k, j] = P
    return K, Ps


def responses(A, B, K):
    """Phi [N][N][nx+nu][nx]: Phi[k, j] = [Phi^x_{k,j}; Phi^u_{k,j}] for
    j < k < N (zero otherwise), and the terminal responses
    Phi^x_{N,j} [N][nx][nx]."""
    N, nx, _ = A.shape
    nu = B.shape[2]
    phi = np.zeros((N, N, nx + nu, nx))
    term = np.zeros((N, nx, nx))
    for j in range(N):
        X = np.eye(nx)
        for k in range(j + 1, N):
            Uk = K[k, j] @ X
            phi[k, j, :nx] = X
            phi[k, j, nx:] = Uk
            X = (A[k] + B[k] @ K[k, j]) @ X
        term[j] = X
    return phi, term


def reform_cost(A, B, K, qx, qu, j):
    """Cost of disturbance time j in eq. fastsls_qp_cost_reform (squared
    weighted Frobenius norms) of the responses that gains K (any gains)
    produce: k = j+1 .. N-1 plus the terminal term at N."""
    N, nx, _ = A.shape
    X = np.eye(nx)
    c = 0.0
    for k in range(j + 1, N):
        Uk = K[k, j] @ X
        c += float((qx[k, j][:, None] * X * X).sum() + (qu[k, j][:, None] * Uk * Uk).sum())
        X = A[k] @ X + B[k] @ Uk
    c += float((qx[N, j][:, None] * X * X).sum())
    return c


# ------------------------------------------------------------ tube

def tube_map(phi, E, cbar, rbar):
    """(mu, sigma) [N][n] of one trajectory from its responses phi
    [N][N][n][nx], disturbance matrices E [N][nx][nw] and residual
    zonotopes cbar, rbar [N][nx]."""
    N, _, n, nx = phi.shape
    mu = np.zeros((N, n))
    sg = np.zeros((N, n))
    for k in range(N):
        for j in range(k):
            P = phi[k, j]
            mu[k] += P @ cbar[j]
            sg[k] += np.abs(P @ E[j]).sum(1) + np.abs(P) @ rbar[j]
    return mu, sg


# ------------------------------------------------------------ disturbance

def disturbance_matrix(dyn: Dyn, z, e, thrust):
    """E(z) = [diag(e) | E_T(z)] [..., nx][nx + U] for chain dynamics: e [nx]
    constant per-state magnitudes, thrust >= 0 the thrust-magnitude
    disturbance of every node."""
    z = np.asarray(z, dtype=np.float64)
    U = dyn.nx // 6
    c = thrust * dyn.c.dt / dyn.c.m
    E = np.zeros(z.shape[:-1] + (dyn.nx, dyn.nx + U))
    E[..., np.arange(dyn.nx), np.arange(dyn.nx)] = e
    for i in range(U):
        th = z[..., 6 * i + 2]
        E[..., 6 * i + 3, dyn.nx + i] = -c * np.sin(th)
        E[..., 6 * i + 4, dyn.nx + i] = c * np.cos(th)
    return E


def r_dist(dyn: Dyn, Ek, z, mu, sigma, thrust):
    """Half-width s [nx] of the enclosure +-s of (E(x) - E_k) w over
    x in z + mu +- sigma (state part), |w|_inf <= 1 (eq. interval_r_dist);
    only the thrust columns depend on the state."""
    U = dyn.nx // 6
    c = thrust * dyn.c.dt / dyn.c.m
    s = np.zeros(dyn.nx)
    if thrust == 0.0:
        return s
    for i in range(U):
        t = 6 * i + 2
        lo, hi = z[t] + mu[t] - sigma[t], z[t] + mu[t] + sigma[t]
        sl, sh = isin(lo, hi)
        cl, ch = icos(lo, hi)
        col = dyn.nx + i
        # row vx: -c sin, row vz: c cos; mag([a, b] - e) = max(|a - e|, |b - e|)
        e_vx, e_vz = Ek[6 * i + 3, col], Ek[6 * i + 4, col]
        s[6 * i + 3] += max(abs(-c * sh - e_vx), abs(-c * sl - e_vx))
        s[6 * i + 4] += max(abs(c * cl - e_vz), abs(c * ch - e_vz))
    return s


# ------------------------------------------------------------ fixed point

def fixed_point(dyn: Dyn, z, v, phi, E, pad=0.0, thrust=0.0):
    """Exact tube/LEB fixed point of one trajectory (z [N][nx], v [N][nu],
    phi [N][N][n][nx], E [N][nx][nw] the disturbance matrices at the nominal)
    by one sequential sweep over k.  thrust > 0 adds r_dist of the thrust
    columns (the last U columns of E; chain dynamics).  Returns mu, sigma
    [N][n] and the remainder enclosure lo, hi [N][nx] (linearization part
    from the bound, disturbance part +-s added)."""
    N, nx = z.shape
    n = phi.shape[2]
    mu = np.zeros((N, n))
    sg = np.zeros((N, n))
    lo = np.zeros((N, nx))
    hi = np.zeros((N, nx))
    cb = np.zeros((N, nx))
    rb = np.zeros((N, nx))
    for k in range(N):
        for j in range(k):
            P = phi[k, j]
            mu[k] += P @ cb[j]
            sg[k] += np.abs(P @ E[j]).sum(1) + np.abs(P) @ rb[j]
        l_, h_, _ = _leb(dyn, z[k][None], v[k][None], sg[k][None], mu=mu[k][None])
        s = r_dist(dyn, E[k], z[k], mu[k], sg[k], thrust)
        lo[k], hi[k] = l_[0] - s, h_[0] + s
        cb[k] = 0.5 * (lo[k] + hi[k])
        rb[k] = 0.5 * (hi[k] - lo[k]) + pad
    return mu, sg, lo, hi
