"""Oracle for the learned warm-start MLP -- TEST INFRASTRUCTURE.

Only tests/, the package's smoke check and bench.py's CPU baseline may
import this module; the product path never does.

The surrogate is a GELU MLP with widths [d0, h, h, h, d_out] (four affine
layers) trained with mixed precision: BF16 operands, FP32 accumulation,
FP32 master weights.  The steps below fix where values are rounded to
BF16, so the oracle (FP64 arithmetic between those points) defines what a
kernel computes up to its FP32 accumulation order:

forward, per sample x:
    a_0 = bf16(x)
    z_l = bf16(W_l) a_{l-1} + b_l,   h_l = gelu(z_l),   a_l = bf16(h_l)   (l < L)
    y   = bf16(W_L) a_{L-1} + b_L
mean-squared error over a batch of B samples and d_out outputs:
    loss = sum (y - t)^2 / (B d_out),   dy = 2 (y - t) / (B d_out)
backward:
    g_L = bf16(dy)
    dW_L = sum_b g_L a_{L-1}^T,   db_L = sum_b dy
    for l = L-1 .. 1:
        dz_l = (bf16(W_{l+1})^T g_{l+1}) * gelu'(z_l),   g_l = bf16(dz_l)
        dW_l = sum_b g_l a_{l-1}^T,   db_l = sum_b dz_l
Adam (Kingma and Ba, Algorithm 1) on the FP32 master parameters.

gelu(z) = z Phi(z) with the standard normal CDF Phi (the exact form),
gelu'(z) = Phi(z) + z phi(z).

bf16(v): v rounded to FP32 (nearest) and then to 8 significant bits
(nearest, ties to even): the conversion the kernels perform on their FP32
values.  With exact=True every bf16() is the identity, which makes the
network a smooth function for finite-difference pins.
"""
from __future__ import annotations

import math

import numpy as np

_SQRT2 = math.sqrt(2.0)
_INV_SQRT2PI = 1.0 / math.sqrt(2.0 * math.pi)


def bf16(v):
    """Round to BF16 (through FP32, nearest-even at both steps); FP64 out."""
    f = np.asarray(v, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    nan = np.isnan(f)
    r = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(nan, np.nan, out)


def _erf(x):
    from scipy.special import erf
    return erf(x)


def gelu(z):
    z = np.asarray(z, dtype=np.float64)
    return 0.5 * z * (1.0 + _erf(z / _SQRT2))


def gelu_grad(z):
    z = np.asarray(z, dtype=np.float64)
    return 0.5 * (1.0 + _erf(z / _SQRT2)) + z * np.exp(-0.5 * z * z) * _INV_SQRT2PI


def unpack(params, widths):
    """Flat FP32 parameter vector [W_1, b_1, ..., W_L, b_L] (W_l row-major
    [out][in]) -> lists of FP64 arrays."""
    p = np.asarray(params, dtype=np.float64)
    W, b, o = [], [], 0
    for i, j in zip(widths[:-1], widths[1:]):
        W.append(p[o:o + i * j].reshape(j, i))
        o += i * j
        b.append(p[o:o + j])
        o += j
    assert o == p.size
    return W, b


def pack(W, b):
    return np.concatenate([np.concatenate([w.reshape(-1), x]) for w, x in zip(W, b)])


def n_params(widths):
    return sum(i * j + j for i, j in zip(widths[:-1], widths[1:]))


def forward(params, widths, x, exact=False):
    """Returns y [B, d_out] and the saved (a_0..a_{L-1}, z_1..z_{L-1})."""
    r = (lambda v: np.asarray(v, dtype=np.float64)) if exact else bf16
    W, b = unpack(params, widths)
    a = [r(x)]
    zs = []
    L = len(W)
    for l in range(L - 1):
        z = a[-1] @ r(W[l]).T + b[l]
        zs.append(z)
        a.append(r(gelu(z)))
    y = a[-1] @ r(W[L - 1]).T + b[L - 1]
    return y, (a, zs)


def mse(y, t):
    B, d = y.shape
    diff = y - t
    return float((diff * diff).sum() / (B * d)), 2.0 * diff / (B * d)


def backward(params, widths, x, dy, exact=False):
    """Flat gradient (same layout as params) of sum(dy * y)."""
    r = (lambda v: np.asarray(v, dtype=np.float64)) if exact else bf16
    W, _ = unpack(params, widths)
    _, (a, zs) = forward(params, widths, x, exact)
    L = len(W)
    dW, db = [None] * L, [None] * L
    dz = np.asarray(dy, dtype=np.float64)
    g = r(dz)
    for l in range(L - 1, -1, -1):
        dW[l] = g.T @ a[l]
        db[l] = dz.sum(axis=0)
        if l > 0:
            dz = (g @ r(W[l])) * gelu_grad(zs[l - 1])
            g = r(dz)
    return pack(dW, db)


def adam(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step >= 1); returns new (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(rng, widths):
    """He-normal weights (gain sqrt(2/fan_in)), zero biases, FP32 values."""
    W, b = [], []
    for i, j in zip(widths[:-1], widths[1:]):
        W.append(rng.normal(0.0, math.sqrt(2.0 / i), (j, i)))
        b.append(np.zeros(j))
    return pack(W, b).astype(np.float32)
