"""Learned warm start: certified training samples and surrogate training.

Samples are bounds the method itself certifies: tubes around a certified
fixed point are scaled and shifted (host-side, seeded), the plain
path-based bound is evaluated on them by the library, and the library's
feature and target kernels turn the bounds into (input, target) pairs.
Training runs the library's BF16 MFMA forward/backward/Adam kernels.
"""
from __future__ import annotations

import math

import numpy as np

from . import (CHAIN_FEATURES, CHAIN_OUTPUTS, Dynamics, Surrogate, analytic_bound, chain_features,
               chain_targets)

CHAIN_WIDTHS = [CHAIN_FEATURES, 128, 128, 128, CHAIN_OUTPUTS]


def he_init(widths, seed):
    """He-normal weights, zero biases: flat FP32 [W_1, b_1, ...]."""
    rng = np.random.default_rng(seed)
    parts = []
    for i, j in zip(widths[:-1], widths[1:]):
        parts.append(rng.normal(0.0, math.sqrt(2.0 / i), i * j))
        parts.append(np.zeros(j))
    return np.concatenate(parts).astype(np.float32)


def chain_samples(dyn: Dynamics, z, v, mu_star, sigma_star, draws, seed, scale=(0.0, 1.5), jitter=0.25):
    """Certified-bound samples around the tubes (mu_star, sigma_star)
    (host float64 arrays [B][N][n]); z, v: float64 GPU tensors.

    Each draw scales sigma_star by lambda ~ U(scale) per (trajectory, step)
    and by 1 + U(-jitter, jitter) per entry, and mu_star by U(0.5, 1.5) per
    (trajectory, step).  Returns (X [S][26], T [S][4]) float32 GPU tensors,
    S = draws * B * N * n_units, in a seeded random order."""
    import torch
    rng = np.random.default_rng(seed)
    B, N, n = sigma_star.shape
    xs, ts = [], []
    for _ in range(draws):
        lam = rng.uniform(scale[0], scale[1], (B, N, 1))
        jit = 1.0 + rng.uniform(-jitter, jitter, (B, N, n))
        sg = sigma_star * lam * jit
        mu = mu_star * rng.uniform(0.5, 1.5, (B, N, 1))
        S = torch.from_numpy(sg).to(z.device)
        M = torch.from_numpy(mu).to(z.device)
        out = analytic_bound(dyn, z, v, S, M)
        xs.append(chain_features(dyn, z, v, S, M).reshape(-1, CHAIN_FEATURES))
        ts.append(chain_targets(dyn, out["r_lo"], out["r_hi"]).reshape(-1, CHAIN_OUTPUTS))
    X = torch.cat(xs)
    T = torch.cat(ts)
    perm = torch.from_numpy(rng.permutation(X.shape[0])).to(z.device)
    return X.index_select(0, perm).contiguous(), T.index_select(0, perm).contiguous()


def train(net: Surrogate, X, T, epochs, batch=1024, lr=2e-3, lr_final=1e-4, log_every=0):
    """Adam on mean-squared error over (X, T) (GPU float32), batches taken
    in order (the sample order is already random), cosine-decayed learning
    rate.  Returns the per-epoch mean training loss (host floats)."""
    import torch
    S = (X.shape[0] // batch) * batch
    steps_per_epoch = S // batch
    total = epochs * steps_per_epoch
    loss = torch.zeros(steps_per_epoch, dtype=torch.float32, device=X.device)
    hist = []
    step = 0
    for ep in range(epochs):
        for k in range(steps_per_epoch):
            frac = step / max(1, total - 1)
            cur = lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * frac))
            step += 1
            net.train_step(X[k * batch:(k + 1) * batch], T[k * batch:(k + 1) * batch], step, cur, loss[k:k + 1])
        hist.append(float(loss.mean().item()))
        if log_every and (ep + 1) % log_every == 0:
            print("epoch %d loss %.4g" % (ep + 1, hist[-1]), flush=True)
    return hist


def evaluate(net: Surrogate, X, T):
    """Mean-squared error and the quantiles of |prediction - target| in log
    space (= relative error of the predicted bound)."""
    import torch
    Y = net.forward(X)
    d = (Y - T).abs().reshape(-1)
    q = torch.quantile(d[: min(d.numel(), 1 << 24)].float(), torch.tensor([0.5, 0.9, 0.99], device=d.device))
    return {"mse": float(((Y - T) ** 2).mean().item()), "abs_log_err_q50_q90_q99": [float(x) for x in q.cpu()]}
