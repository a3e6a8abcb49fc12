"""Oracle gradient of the ReLU-MLP remainder bound -- TEST INFRASTRUCTURE.

The derivative of the Theorem 2 bound [r_lo, r_hi] of `oracle.nn.leb` (CROWN
relaxations with full CROWN passes for every hidden layer, section IV.B) with
respect to the nominal point a~, the radii sigma and the offset mu, as used
by the paper's differentiable bound implementation (section IV.D).  The
bound is piecewise smooth in these inputs; between kinks every branch choice
(stable/unstable neuron, the adaptive lower slope, the sign of each CROWN
coefficient, the sign inside |.|, the clamps of the displacement interval)
is fixed and the derivative is that of the selected branch.

Written in forward mode: every quantity of the bound is carried with its
tangent along one input direction, in the order the bound computes them
(box, first-layer bounds, one CROWN pass per later hidden layer, the output
pass, Theorem 2).  The gradient of L = sum g_hi r_hi + g_lo r_lo is the set
of directional derivatives along the unit directions.  Conventions at ties
(measure zero): sign(0) = 0 in d|x|, the clamp min(m - sigma, 0) passes the
derivative only where m - sigma < 0 and max(m + sigma, 0) only where
m + sigma > 0, a CROWN coefficient of exactly 0 counts as non-negative.

The Jacobian J = J_g(a~) is constant between kinks, so the terms J a~ - g(a~)
of Theorem 2 have derivative J - J = 0 along a~.

Pinned by central finite differences of `oracle.nn.leb` (itself pinned) in
tests/test_oracle_nn_grad.py.  Plain FP64 numpy.
"""
from __future__ import annotations

import numpy as np

from . import nn


def _relax_t(lo, dlo, hi, dhi):
    """Relaxation (s, t, a) of `nn.relaxation` and its tangent (ds, dt)."""
    s, t, a = nn.relaxation(lo, hi)
    ds = np.zeros_like(lo)
    dt = np.zeros_like(lo)
    unst = (lo < 0) & (hi > 0)
    den = hi - lo
    # s = u / (u - l): ds = (u dl - l du) / (u - l)^2;  t = -s l: dt = -l ds - s dl
    ds[unst] = (hi[unst] * dlo[unst] - lo[unst] * dhi[unst]) / den[unst] ** 2
    dt[unst] = -lo[unst] * ds[unst] - s[unst] * dlo[unst]
    return (s, t, a), (ds, dt)


def _crown_t(W, b, rel, drel, target_W, target_b, n_layers, upper):
    """`nn.crown` with tangents: returns (Lam, dLam, beta, dbeta) of the
    pass for the target target_W a_{n_layers} + target_b (weights fixed)."""
    Lam = np.array(target_W, dtype=np.float64)
    dLam = np.zeros_like(Lam)
    beta = np.array(target_b, dtype=np.float64)
    dbeta = np.zeros_like(beta)
    for k in range(n_layers, 0, -1):
        s, t, a = rel[k - 1]
        ds, dt = drel[k - 1]
        pos = Lam >= 0
        sel = pos if upper else ~pos          # where the upper line (s, t) is taken
        S = np.where(sel, s[..., None, :], a[..., None, :])
        dS = np.where(sel, ds[..., None, :], 0.0)
        beta = beta + np.sum(np.where(sel, Lam * t[..., None, :], 0.0), axis=-1)
        dbeta = dbeta + np.sum(np.where(sel, dLam * t[..., None, :] + Lam * dt[..., None, :], 0.0), axis=-1)
        Om = Lam * S
        dOm = dLam * S + Lam * dS
        beta = beta + Om @ b[k - 1]
        dbeta = dbeta + dOm @ b[k - 1]
        Lam = Om @ W[k - 1]
        dLam = dOm @ W[k - 1]
    return Lam, dLam, beta, dbeta


def _conc_t(Lam, dLam, beta, dbeta, c, dc, rho, drho, upper):
    """Tangent of Lam c +/- |Lam| rho + beta."""
    sg = 1.0 if upper else -1.0
    val = np.einsum("...mn,...n->...m", Lam, c) + sg * np.einsum("...mn,...n->...m", np.abs(Lam), rho) + beta
    d = (np.einsum("...mn,...n->...m", dLam, c) + np.einsum("...mn,...n->...m", Lam, dc)
         + sg * (np.einsum("...mn,...n->...m", np.sign(Lam) * dLam, rho)
                 + np.einsum("...mn,...n->...m", np.abs(Lam), drho))
         + dbeta)
    return val, d


def leb_jvp(W, b, alpha, sigma, mu, dalpha, dsigma, dmu):
    """Directional derivative of (r_lo, r_hi) of `nn.leb` (J = J_g(a~))
    along (dalpha, dsigma, dmu).  alpha, sigma, mu [n0] (mu may be None:
    zero, and then dmu must be zero).  Returns (r_lo, r_hi, dr_lo, dr_hi)."""
    W = [np.asarray(w, dtype=np.float64) for w in W]
    b = [np.asarray(x, dtype=np.float64) for x in b]
    alpha = np.asarray(alpha, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    m = np.zeros_like(alpha) if mu is None else np.asarray(mu, dtype=np.float64)
    L = len(W)
    # displacement interval [min(m - sigma, 0), max(m + sigma, 0)] and its box
    lo_d = np.minimum(m - sigma, 0.0)
    hi_d = np.maximum(m + sigma, 0.0)
    dlo_d = np.where(m - sigma < 0, dmu - dsigma, 0.0)
    dhi_d = np.where(m + sigma > 0, dmu + dsigma, 0.0)
    c = alpha + 0.5 * (lo_d + hi_d)
    rho = 0.5 * (hi_d - lo_d)
    dc = dalpha + 0.5 * (dlo_d + dhi_d)
    drho = 0.5 * (dhi_d - dlo_d)
    # first hidden layer: exact interval of W_1 a + b_1 over the box
    z1 = W[0] @ c + b[0]
    r1 = np.abs(W[0]) @ rho
    dz1 = W[0] @ dc
    dr1 = np.abs(W[0]) @ drho
    rel, drel = [], []
    r, dr = _relax_t(z1 - r1, dz1 - dr1, z1 + r1, dz1 + dr1)
    rel.append(r)
    drel.append(dr)
    # later hidden layers: one CROWN pass each (upper and lower)
    for k in range(2, L):
        Lu, dLu, bu, dbu = _crown_t(W, b, rel, drel, W[k - 1], b[k - 1], k - 1, True)
        Ll, dLl, bl, dbl = _crown_t(W, b, rel, drel, W[k - 1], b[k - 1], k - 1, False)
        hi, dhi = _conc_t(Lu, dLu, bu, dbu, c, dc, rho, drho, True)
        lo, dlo = _conc_t(Ll, dLl, bl, dbl, c, dc, rho, drho, False)
        r, dr = _relax_t(lo, dlo, hi, dhi)
        rel.append(r)
        drel.append(dr)
    # output pass and Theorem 2 with J = J_g(a~) (locally constant)
    zs = nn.forward(W, b, alpha)
    g = zs[-1]
    J = nn.jacobian(W, zs)
    Lu, dLu, bu, dbu = _crown_t(W, b, rel, drel, W[-1], b[-1], L - 1, True)
    Ll, dLl, bl, dbl = _crown_t(W, b, rel, drel, W[-1], b[-1], L - 1, False)
    r_hi, dr_hi = _conc_t(Lu - J, dLu, bu, dbu, c, dc, rho, drho, True)
    r_lo, dr_lo = _conc_t(Ll - J, dLl, bl, dbl, c, dc, rho, drho, False)
    Ja_g = J @ alpha - g
    return r_lo + Ja_g, r_hi + Ja_g, dr_lo, dr_hi


def leb_grad(W, b, alpha, sigma, mu, g_lo, g_hi):
    """Gradient of L = sum_m g_hi[m] r_hi[m] + g_lo[m] r_lo[m] for one box:
    returns (d alpha, d sigma, d mu) [n0] each (d mu all zero when mu is None),
    from one directional derivative per input coordinate."""
    alpha = np.asarray(alpha, dtype=np.float64)
    n0 = alpha.shape[-1]
    z = np.zeros(n0)
    out = []
    for which in range(3 if mu is not None else 2):
        gcol = np.zeros(n0)
        for i in range(n0):
            e = np.zeros(n0)
            e[i] = 1.0
            da, ds, dm = (e, z, z) if which == 0 else ((z, e, z) if which == 1 else (z, z, e))
            _, _, dlo, dhi = leb_jvp(W, b, alpha, sigma, mu, da, ds, dm)
            gcol[i] = np.dot(g_lo, dlo) + np.dot(g_hi, dhi)
        out.append(gcol)
    if mu is None:
        out.append(np.zeros(n0))
    return tuple(out)
