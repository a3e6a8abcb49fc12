"""What FP32 arithmetic would cost the CROWN bound -- TEST INFRASTRUCTURE.

The backward substitution of CROWN (section IV.B) forms
    Lambda_{j-1} = (Lambda_j . S_j) W_j
for every layer j, S_j the sign-selected relaxation slopes.  Computed on
FP32 matrix cores, the product is exact only up to rounding; the bound stays
sound for whatever matrix Lambda^_{j-1} comes out, once the error
    |Lambda^_{j-1} - (Lambda^_j . S_j) W_j| <= gamma_{K+1} |Lambda^_j . S_j| |W_j|
is paid for: in centred coordinates (a - a~) the error multiplies the
deviation of layer j-1's activations from their nominal values, bounded by
w_{j-1} (w_0 = rho + |c - a~|; a hidden layer's w from its pre-activation
bounds), so the bound widens by
    gamma_{K+1} |Lambda^_j . S_j| (|W_j| w_{j-1})     (per output row and mode).
gamma_n = n u / (1 - n u), u = 2^-24, K the length of the FP32 partial sums
(the chunks are added in FP64; the +1 is the rounding of the FP32 operand).

With Jacobian-deviation coefficients the FP64 Jacobian chain M (S = the
nominal masks D) is kept exactly and only Lambda - M goes through FP32, so
the operand is Lambda_j . S_j - M_j . D_j, which vanishes where the
relaxation equals the nominal mask (stable neurons).

This module computes that widening for the output chain (the intermediate
chains only add to it) and compares it with the bound's magnitude: the
evidence for the precision of the GPU's contractions.
"""
from __future__ import annotations

import numpy as np

from . import nn

U32 = 2.0 ** -24


def gamma(n):
    return n * U32 / (1.0 - n * U32)


def fp32_chunked_product(A, B, K):
    """A @ B with FP32 operands, FP32 partial sums over chunks of K terms of
    the contraction, chunks added in FP64 (what a K-deep FP32 MFMA chain with
    FP64 chunk accumulation computes, up to the order inside a chunk)."""
    A32 = np.asarray(A, dtype=np.float32)
    B32 = np.asarray(B, dtype=np.float32)
    n = A32.shape[-1]
    out = np.zeros(A32.shape[:-1] + (B32.shape[-1],), dtype=np.float64)
    for k0 in range(0, n, K):
        out += (A32[..., k0:k0 + K] @ B32[k0:k0 + K]).astype(np.float64)
    return out


def output_chain_widening(W, b, alpha, sigma, K, jac_dev=True, mu=None):
    """Widening (upper, lower) [..., m] of the Theorem 2 bound when the output
    chain's products are formed in FP32 chunks of K (see the module text)."""
    W = [np.asarray(w, dtype=np.float64) for w in W]
    b = [np.asarray(x, dtype=np.float64) for x in b]
    alpha = np.asarray(alpha, dtype=np.float64)
    c, rho = nn.box_of(alpha, np.asarray(sigma, dtype=np.float64), mu)
    L = len(W)
    zs = nn.forward(W, b, alpha)
    bounds, rel = nn.layer_bounds(W, b, c, rho)
    # deviation bounds of the activations feeding each layer
    w = [rho + np.abs(c - alpha)]
    for j in range(1, L):
        lo, hi = bounds[j - 1]
        zh = zs[j - 1]
        w.append(np.maximum(hi - zh, zh - lo))
    g = gamma(K + 1)
    out = []
    for upper in (True, False):
        Lam = np.broadcast_to(W[-1], alpha.shape[:-1] + W[-1].shape).copy()
        M = Lam.copy()
        wid = np.zeros(Lam.shape[:-1])
        for k in range(L - 1, 0, -1):
            s, _, a = rel[k - 1]
            D = (zs[k - 1] > 0).astype(np.float64)
            pos = Lam >= 0
            if upper:
                S = np.where(pos, s[..., None, :], a[..., None, :])
            else:
                S = np.where(pos, a[..., None, :], s[..., None, :])
            Om = Lam * S
            Md = M * D[..., None, :]
            X = Om - Md if jac_dev else Om
            v = np.einsum("ij,...j->...i", np.abs(W[k - 1]), w[k - 1])      # |W_k| w_{k-1}
            wid = wid + g * np.einsum("...mi,...i->...m", np.abs(X), v)
            Lam = Om @ W[k - 1]
            M = Md @ W[k - 1]
        out.append(wid)
    return out[0], out[1]


def study(W, b, alpha, sigma, Ks=(4, 16, 256)):
    """Ratio of the FP32 widening to the bound's magnitude max(|r_lo|, |r_hi|),
    per box (the largest over its rows), for each K, without and with
    Jacobian-deviation coefficients.  Returns {(K, jac_dev): ratios [boxes]}."""
    o = nn.leb(W, b, alpha, sigma)
    M = np.maximum(np.abs(o["r_lo"]), np.abs(o["r_hi"]))
    res = {}
    for K in Ks:
        for jd in (False, True):
            wu, wl = output_chain_widening(W, b, alpha, sigma, K, jac_dev=jd)
            ratio = np.maximum(wu, wl) / np.maximum(M, 1e-300)
            res[(K, jd)] = ratio.max(axis=-1)
    return res
