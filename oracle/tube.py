"""Oracle tube map and tube/LEB fixed point -- TEST INFRASTRUCTURE.

Tube update (eqs. tight_tube_center, tight_tube_width):
    mu_k    = sum_{j<k} Phi_{k,j} c_bar_j
    sigma_k = sum_{j<k} || Phi_{k,j} E_bar_j ||_{1,r} = sum_{j<k} |Phi_{k,j}| (e + rho_bar_j)
with the residual zonotope E_bar_j = [E  diag(rho_bar_j)] (eq. zonotope_combination)
and e = |E| 1.  The LEB of step k is evaluated over the box
((z_k, v_k) + mu_k) +/- sigma_k (eq. zontope_combination_interval), and
(c_bar, rho_bar) are its zonotope centre and radius (eq. zono_map).

Phi is the decentralised, lag-invariant closed-loop response that the
generators provide: one [8 x 6] block per lag d = k - j >= 1, shared by
every node; rows 0..5 act on the node's state entries of the tube, rows
6..7 on its input entries, columns on the node's residual entries.

The exact fixed point is reached by one sequential sweep k = 0, 1, ...,
N-1: the tube at k depends on the bounds of steps j < k only (causality;
the base case mu_0 = sigma_0 = 0 is the known initial state, as in the
induction of the Theorem 3 proof).  Plain FP64.
"""
from __future__ import annotations

import numpy as np

from . import leb as _leb, Dyn


def _node_cols(U):
    """Index helpers: state rows of node i = 6i..6i+5, input rows = 6U+2i.."""
    st = np.arange(6)[None, :] + 6 * np.arange(U)[:, None]          # [U][6]
    inp = 6 * U + np.arange(2)[None, :] + 2 * np.arange(U)[:, None]  # [U][2]
    return st, inp


def tube_map(phi, e, cbar, rbar):
    """(mu, sigma) [B][N][n] from residual zonotopes cbar, rbar [B][N][nx]."""
    B, N, nx = cbar.shape
    U = nx // 6
    n = 8 * U
    st, inp = _node_cols(U)
    cb = cbar.reshape(B, N, U, 6)
    w = (e[None, None, None, :] + rbar.reshape(B, N, U, 6))
    A = np.abs(phi)
    mu = np.zeros((B, N, U, 8))
    sg = np.zeros((B, N, U, 8))
    for k in range(1, N):
        for j in range(k):
            P = phi[k - j - 1]
            mu[:, k] += np.einsum("rc,buc->bur", P, cb[:, j])
            sg[:, k] += np.einsum("rc,buc->bur", A[k - j - 1], w[:, j])
    out_mu = np.zeros((B, N, n))
    out_sg = np.zeros((B, N, n))
    out_mu[:, :, st.reshape(-1)] = mu[..., :6].reshape(B, N, -1)
    out_mu[:, :, inp.reshape(-1)] = mu[..., 6:].reshape(B, N, -1)
    out_sg[:, :, st.reshape(-1)] = sg[..., :6].reshape(B, N, -1)
    out_sg[:, :, inp.reshape(-1)] = sg[..., 6:].reshape(B, N, -1)
    return out_mu, out_sg


def zono(lo, hi, pad=0.0):
    """Zonotope centre and radius of [lo, hi] (eq. zono_map), radius padded."""
    return 0.5 * (lo + hi), 0.5 * (hi - lo) + pad


def fixed_point(dyn: Dyn, z, v, phi, e, pad=0.0, threads=0):
    """Exact tube/LEB fixed point by one sequential sweep over k.

    Returns (mu, sigma) [B][N][n], (lo, hi) [B][N][nx] of the final boxes."""
    B, N, nx = z.shape
    U = nx // 6
    n = 8 * U
    mu = np.zeros((B, N, n))
    sg = np.zeros((B, N, n))
    lo = np.zeros((B, N, nx))
    hi = np.zeros((B, N, nx))
    st, inp = _node_cols(U)
    rows = np.concatenate([st, inp], 1)          # [U][8] tube rows of node i
    A = np.abs(phi)
    cb = np.zeros((B, N, U, 6))
    w = np.zeros((B, N, U, 6))
    for k in range(N):
        if k > 0:
            m = np.zeros((B, U, 8))
            s = np.zeros((B, U, 8))
            for j in range(k):
                m += np.einsum("rc,buc->bur", phi[k - j - 1], cb[:, j])
                s += np.einsum("rc,buc->bur", A[k - j - 1], w[:, j])
            mu[:, k][:, rows.reshape(-1)] = m.reshape(B, -1)
            sg[:, k][:, rows.reshape(-1)] = s.reshape(B, -1)
        l_, h_, _ = _leb(dyn, z[:, k], v[:, k], sg[:, k], mu=mu[:, k], threads=threads)
        lo[:, k], hi[:, k] = l_, h_
        c, r = zono(l_, h_, pad)
        cb[:, k] = c.reshape(B, U, 6)
        w[:, k] = (e[None, None, :] + r.reshape(B, U, 6))
    return mu, sg, lo, hi


def contains(mu_in, sg_in, mu_out, sg_out):
    """Box (mu_out +/- sg_out) inside box (mu_in +/- sg_in), per trajectory."""
    ok = (mu_out - sg_out >= mu_in - sg_in) & (mu_out + sg_out <= mu_in + sg_in)
    return ok.reshape(ok.shape[0], -1).all(1)


def zonotope_hull(G, c=None):
    """Interval hull of the zonotopes {c + G xi : |xi|_inf <= 1}, row by row
    (eq. tight_tube_width): mu = c, sigma_i = sum_j |G_ij|, the row's
    maximum of |G_i xi| over the unit box.  G [rows][n_gen]; the sums are
    exact to the last bit (math.fsum), then rounded to nearest."""
    import math
    G = np.asarray(G, dtype=np.float64)
    sg = np.array([math.fsum(np.abs(row)) for row in G]) if G.shape[1] else np.zeros(G.shape[0])
    mu = np.zeros(G.shape[0]) if c is None else np.asarray(c, dtype=np.float64).copy()
    return mu, sg
