"""Learned warm start: certified training samples and surrogate training.

Samples are bounds the method itself certifies.  Chain family: tubes
around a certified fixed point are scaled and shifted (host-side, seeded)
and the plain path-based bound is evaluated on them.  NN family: boxes of
a ReLU-MLP's input (nominal point and radii drawn host-side, seeded) are
bounded by CROWN and Theorem 2.  The library's feature and target kernels
turn the bounds into (input, target) pairs, and training runs the
library's BF16 MFMA forward/backward/Adam kernels.
"""
from __future__ import annotations

import math

import numpy as np

from . import (CHAIN_FEATURES, CHAIN_OUTPUTS, MLP, Dynamics, Surrogate, analytic_bound, chain_features,
               chain_targets, nn_bound, nn_features, nn_targets, tube_map)

CHAIN_WIDTHS = [CHAIN_FEATURES, 128, 128, 128, CHAIN_OUTPUTS]


def nn_widths(mlp: MLP, hidden=128):
    """NN-family surrogate widths: 2 (nx + nu) features, three hidden
    layers, 2m log-bounds (32 -> 128 -> 128 -> 128 -> 24 for a 16-input,
    12-output network)."""
    return [2 * mlp.widths[0], hidden, hidden, hidden, 2 * mlp.m]


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


def chain_fp_samples(dyn: Dynamics, z, v, phi, e, mu_star, sigma_star, seed):
    """Fixed-point-target samples: the features of the disturbance-only tube
    (the cold start, the same for every trajectory) paired with the targets
    of the certified bound at the fixed point (mu_star, sigma_star), so that
    one surrogate sweep from the cold start predicts the fixed point's
    residuals instead of one step of the iteration.  z, v, phi: float64 GPU
    tensors; mu_star, sigma_star: GPU tensors [B][N][n].  Returns (X, T)
    float32 GPU tensors, B * N * n_units rows in a seeded random order."""
    import torch
    B, N = int(z.shape[0]), int(z.shape[1])
    zero = torch.zeros((B, N, dyn.nx), dtype=torch.float64, device=z.device)
    md, sd = tube_map(dyn.n_units, phi, e, zero, zero)
    X = chain_features(dyn, z, v, sd, md).reshape(-1, CHAIN_FEATURES)
    out = analytic_bound(dyn, z, v, sigma_star, mu_star)
    T = chain_targets(dyn, out["r_lo"], out["r_hi"]).reshape(-1, CHAIN_OUTPUTS)
    rng = np.random.default_rng(seed)
    perm = torch.from_numpy(rng.permutation(X.shape[0])).to(z.device)
    return X.index_select(0, perm).contiguous(), T.index_select(0, perm).contiguous()


def nn_samples(mlp: MLP, boxes, seed, nominal=(-1.0, 1.0), radii=(0.005, 0.05), chunk=4096, device="cuda:0"):
    """Certified-bound samples of ReLU-MLP dynamics: `boxes` boxes with the
    nominal input ~ U(nominal) and radii ~ U(radii) per input (drawn on the
    host, seeded), bounded by leb_nn_bound in chunks.  Returns (X [boxes][2n],
    T [boxes][2m]) float32 GPU tensors; the draws are independent, so the
    order is already random."""
    import torch
    rng = np.random.default_rng(seed)
    n, nx = mlp.widths[0], mlp.nx
    xs, ts = [], []
    done = 0
    while done < boxes:
        c = min(chunk, boxes - done)
        a = torch.from_numpy(rng.uniform(nominal[0], nominal[1], (c, 1, n))).to(device)
        sg = torch.from_numpy(rng.uniform(radii[0], radii[1], (c, 1, n))).to(device)
        z, v = a[..., :nx].contiguous(), a[..., nx:].contiguous()
        out = nn_bound(mlp, z, v, sg)
        xs.append(nn_features(z, v, sg).reshape(c, 2 * n))
        ts.append(nn_targets(out["r_lo"], out["r_hi"]).reshape(c, 2 * mlp.m))
        done += c
    return torch.cat(xs).contiguous(), torch.cat(ts).contiguous()


def save_samples(path, X, T):
    """Writes a sample set (X, T float32 tensors) to an .npz file (no
    pickled objects), so a surrogate can be retrained without bounding the
    samples again."""
    np.savez(path, X=X.detach().cpu().numpy().astype(np.float32), T=T.detach().cpu().numpy().astype(np.float32))


def load_samples(path, device="cuda:0"):
    """Reads a sample set written by save_samples (pickles refused)."""
    import torch
    with np.load(path, allow_pickle=False) as f:
        X, T = f["X"], f["T"]
    if X.ndim != 2 or T.ndim != 2 or X.shape[0] != T.shape[0] or X.dtype != np.float32 or T.dtype != np.float32:
        raise ValueError("%s: not a sample set" % path)
    return torch.from_numpy(X).to(device), torch.from_numpy(T).to(device)


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
