"""Oracle for neural-network dynamics -- TEST INFRASTRUCTURE.

Dynamics f(x, u) = x + g([x; u]) with a ReLU MLP g (z_l = W_l a_{l-1} + b_l,
a_l = relu(z_l), g = z_L).  The residual x is linear, so the remainder is
that of g.  Plain FP64 numpy, written from section IV.B:

* CROWN affine bounds W_lo a + b_lo <= g(a) <= W_hi a + b_hi over a box
  (Theorem "CROWN bounds", Zhang et al. 2018 Thm 3.2), by backward
  substitution through per-neuron ReLU relaxations:
    stable active (l >= 0): a = z; stable inactive (u <= 0): a = 0;
    unstable: upper line s z + t with s = u/(u-l), t = -s l; lower line
    a_slope z with a_slope = 1 if u >= -l else 0 (adaptive choice);
  a positive coefficient takes the upper line for an upper bound and the
  lower line for a lower bound (reversed for negative coefficients).
* Intermediate pre-activation bounds: the first layer exactly
  (W_1 c + b_1 -/+ |W_1| rho); every later hidden layer by a full CROWN
  pass of its own.
* Theorem 2 (eq. crown_remainder_interval): with J = J_g(a~),
    r_hi = max_X (W_hi - J) a + J a~ - g(a~) + b_hi,
    r_lo = min_X (W_lo - J) a + J a~ - g(a~) + b_lo,
  and, as a self-check, the centred form
    r_hi = (W_hi - J)(c - a~) + |W_hi - J| rho + kappa_hi,
  kappa_hi = sum over relaxed neurons of coefficient x (line(z^) - relu(z^)),
  each summand >= 0, so no cancellation.
* relu'(0) = 0 in J (any J is valid for Theorem 2).
Floating point: plain FP64 round-to-nearest (errors ~1e-13 relative, far
below the parity tolerance); the oracle defines the value, the GPU adds its
own rounding allowance.
"""
from __future__ import annotations

import numpy as np


def box_of(alpha, sigma, mu=None):
    """Centre and half-width of hull({a~} U [a~+mu-sigma, a~+mu+sigma])."""
    m = 0.0 if mu is None else mu
    dlo = np.minimum(m - sigma, 0.0)
    dhi = np.maximum(m + sigma, 0.0)
    return alpha + 0.5 * (dlo + dhi), 0.5 * (dhi - dlo)


def forward(W, b, a0):
    """Pre-activations z_1..z_L (z_L = g) at a0 [..., n0]."""
    zs = []
    a = a0
    for l, (Wl, bl) in enumerate(zip(W, b)):
        z = a @ Wl.T + bl
        zs.append(z)
        a = np.maximum(z, 0.0)
    return zs


def jacobian(W, zs):
    """J = W_L D_{L-1} ... D_1 W_1 with D = 1[z > 0] (relu'(0) = 0)."""
    J = np.broadcast_to(W[-1], zs[0].shape[:-1] + W[-1].shape).copy()
    for l in range(len(W) - 2, -1, -1):
        D = (zs[l] > 0).astype(np.float64)
        J = (J * D[..., None, :]) @ W[l]
    return J


def relaxation(lo, hi):
    """Per-neuron (s, t, a): upper line s z + t, lower line a z."""
    s = np.zeros_like(lo)
    t = np.zeros_like(lo)
    a = np.zeros_like(lo)
    act = lo >= 0
    s[act] = 1.0
    a[act] = 1.0
    unst = (lo < 0) & (hi > 0)
    s[unst] = hi[unst] / (hi[unst] - lo[unst])
    t[unst] = -s[unst] * lo[unst]
    a[unst] = (hi[unst] >= -lo[unst]).astype(np.float64)
    return s, t, a


def crown(W, b, rel, target_W, target_b, n_layers, upper):
    """Backward substitution for target_W z_{n_layers+1}-style targets.

    The target is target_W a_{n_layers} + target_b, where a_k = relu(z_k)
    for k = n_layers .. 1 use the relaxations rel[k-1] = (s, t, a).
    Returns (Lambda_0 [..., m, n0], beta [..., m], slack terms kept for
    the centred form: list of (Lambda_k, k))."""
    Lam = np.array(target_W, dtype=np.float64)
    beta = np.array(target_b, dtype=np.float64)
    kept = []
    for k in range(n_layers, 0, -1):
        s, t, a = rel[k - 1]
        pos = Lam >= 0
        if upper:
            S = np.where(pos, s[..., None, :], a[..., None, :])
            beta = beta + np.sum(np.where(pos, Lam * t[..., None, :], 0.0), axis=-1)
        else:
            S = np.where(pos, a[..., None, :], s[..., None, :])
            beta = beta + np.sum(np.where(pos, 0.0, Lam * t[..., None, :]), axis=-1)
        kept.append((Lam, k))
        Om = Lam * S
        beta = beta + Om @ b[k - 1]
        Lam = Om @ W[k - 1]
    return Lam, beta, kept


def concretize(Lam, beta, c, rho, upper):
    lin = np.einsum("...mn,...n->...m", Lam, c)
    mag = np.einsum("...mn,...n->...m", np.abs(Lam), rho)
    return lin + mag + beta if upper else lin - mag + beta


def layer_bounds(W, b, c, rho):
    """Pre-activation bounds (l_k, u_k) of the hidden layers k = 1..L-1."""
    L = len(W)
    z1 = c @ W[0].T + b[0]
    r1 = rho @ np.abs(W[0]).T
    bounds = [(z1 - r1, z1 + r1)]
    rel = [relaxation(*bounds[0])]
    for k in range(2, L):
        tw = np.broadcast_to(W[k - 1], c.shape[:-1] + W[k - 1].shape)
        tb = np.broadcast_to(b[k - 1], c.shape[:-1] + b[k - 1].shape)
        Lu, bu, _ = crown(W, b, rel, tw, tb, k - 1, True)
        Ll, bl, _ = crown(W, b, rel, tw, tb, k - 1, False)
        hi = concretize(Lu, bu, c, rho, True)
        lo = concretize(Ll, bl, c, rho, False)
        bounds.append((lo, hi))
        rel.append(relaxation(lo, hi))
    return bounds, rel


def leb(W, b, alpha, sigma, mu=None, centred=True, J=None):
    """Theorem 2 bound [r_lo, r_hi] per unit (alpha, sigma [..., n0]).

    J [..., m, n0]: the matrix of the linearization (None: the network's
    Jacobian at alpha).  Theorem 2 holds for any J: the bound then encloses
    g(a) - g(a~) - J (a - a~).
    Returns dict with r_lo, r_hi (direct form), c_lo, c_hi (centred form),
    J, g, Lambda_hi, Lambda_lo, beta_hi, beta_lo, unstable counts."""
    W = [np.asarray(w, dtype=np.float64) for w in W]
    b = [np.asarray(x, dtype=np.float64) for x in b]
    alpha = np.asarray(alpha, dtype=np.float64)
    c, rho = box_of(alpha, np.asarray(sigma, dtype=np.float64), mu)
    L = len(W)
    zs = forward(W, b, alpha)
    g = zs[-1]
    J = jacobian(W, zs) if J is None else np.asarray(J, dtype=np.float64)
    bounds, rel = layer_bounds(W, b, c, rho)
    tw = np.broadcast_to(W[-1], alpha.shape[:-1] + W[-1].shape)
    tb = np.broadcast_to(b[-1], alpha.shape[:-1] + b[-1].shape)
    Lu, bu, keep_u = crown(W, b, rel, tw, tb, L - 1, True)
    Ll, bl, keep_l = crown(W, b, rel, tw, tb, L - 1, False)
    Ja = np.einsum("...mn,...n->...m", J, alpha)
    Du, Dl = Lu - J, Ll - J
    r_hi = np.einsum("...mn,...n->...m", Du, c) + np.einsum("...mn,...n->...m", np.abs(Du), rho) + Ja - g + bu
    r_lo = np.einsum("...mn,...n->...m", Dl, c) - np.einsum("...mn,...n->...m", np.abs(Dl), rho) + Ja - g + bl
    out = {"r_lo": r_lo, "r_hi": r_hi, "J": J, "g": g, "Lambda_hi": Lu, "Lambda_lo": Ll, "beta_hi": bu,
           "beta_lo": bl, "bounds": bounds,
           "unstable": [int(((lo < 0) & (hi > 0)).sum()) for lo, hi in bounds]}
    if centred:
        dev = c - alpha
        kap_u = np.zeros_like(g)
        kap_l = np.zeros_like(g)
        for (Lam, k), (Laml, _) in zip(keep_u, keep_l):
            s, t, a = rel[k - 1]
            zh = zs[k - 1]
            rz = np.maximum(zh, 0.0)
            up_gap = (s * zh + t - rz)[..., None, :]      # >= 0
            lo_gap = (a * zh - rz)[..., None, :]          # <= 0
            kap_u += np.sum(np.where(Lam >= 0, Lam * up_gap, Lam * lo_gap), axis=-1)
            kap_l += np.sum(np.where(Laml >= 0, Laml * lo_gap, Laml * up_gap), axis=-1)
        out["c_hi"] = np.einsum("...mn,...n->...m", Du, dev) + np.einsum("...mn,...n->...m", np.abs(Du), rho) + kap_u
        out["c_lo"] = np.einsum("...mn,...n->...m", Dl, dev) - np.einsum("...mn,...n->...m", np.abs(Dl), rho) + kap_l
        out["kappa_hi"], out["kappa_lo"] = kap_u, kap_l
    return out


def remainder(W, b, alpha_nom, pts, J=None):
    """True remainder g(a) - g(a~) - J(a~)(a - a~) at points [..., S, n0]
    for nominals [..., n0], in FP64 (long double where numpy provides it is
    not needed: the allowance below bounds the FP64 error).  J [..., m, n0]
    replaces the network's Jacobian when given."""
    W = [np.asarray(w, dtype=np.float64) for w in W]
    b = [np.asarray(x, dtype=np.float64) for x in b]
    zs0 = forward(W, b, alpha_nom)
    J = jacobian(W, zs0) if J is None else np.asarray(J, dtype=np.float64)
    g0 = zs0[-1]
    zs = forward(W, b, pts)
    d = pts - alpha_nom[..., None, :]
    lin = np.einsum("...mn,...sn->...sm", J, d)
    r = zs[-1] - g0[..., None, :] - lin
    # FP64 error allowance: magnitude chain |W| |a| through the layers
    mag = np.abs(pts)
    mag0 = np.abs(alpha_nom)
    for Wl, bl in zip(W, b):
        mag = mag @ np.abs(Wl).T + np.abs(bl)
        mag0 = mag0 @ np.abs(Wl).T + np.abs(bl)
    eps = 1e-12 * (mag + mag0[..., None, :] + np.einsum("...mn,...sn->...sm", np.abs(J), np.abs(d)))
    return r, eps
