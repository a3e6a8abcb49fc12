"""Oracle refinement of the linearization point -- TEST INFRASTRUCTURE.

The nominal-point optimization of the results section (Table II):
projected gradient descent on the width W = sum_l (hi_l - lo_l) of the
path-based bound as a function of the nominal (linearization) point a~,
searched within a0 +/- radius sigma of the start a0.  Two readings of the
set the bound covers:
  * travelling box (the paper's setting: the perturbation radius is fixed,
    the set is centred on the nominal point): X = a~ + mu0 +/- sigma, so
    dW/da~ = (dW/dz, dW/dv) at fixed mu = mu0;
  * fixed box: X = (a0 + mu0) +/- sigma whatever a~ is; written
    a~ + mu +/- sigma with mu = a0 + mu0 - a~, so
    dW/da~ = (dW/dz, dW/dv) - dW/dmu.
The derivatives are the oracle's forward-mode gradient with upstream -1 on
lo and +1 on hi.  Step s moves each coordinate by
lr radius sigma_i (1 - s / steps) against the sign of its derivative and
clips to the search box; the narrowest iterate is kept.  Plain FP64.
"""
from __future__ import annotations

import numpy as np

from . import Dyn, leb, leb_grad


def width(dyn: Dyn, a, mu, sigma):
    """Width of the bound over the box a + mu +/- sigma linearized at a."""
    lo, hi, _ = leb(dyn, a[..., :dyn.nx], a[..., dyn.nx:], sigma, mu=mu)
    return (hi - lo).sum(-1)


def pgd_nominal(dyn: Dyn, z0, v0, sigma, mu0=None, radius=0.5, steps=20, lr=0.25, fixed_box=False):
    """Returns (a_best [..., n], w_best [...], w0 [...]) for units [..., n]."""
    a0 = np.concatenate([z0, v0], -1)
    m0 = np.zeros_like(a0) if mu0 is None else np.asarray(mu0, dtype=np.float64)
    box_mu = (lambda a: a0 + m0 - a) if fixed_box else (lambda a: m0)
    a = a0.copy()
    r = radius * sigma
    best_a, best_w, w0 = a0.copy(), None, None
    ones = np.ones(z0.shape)
    for s in range(steps + 1):
        w = width(dyn, a, box_mu(a), sigma)
        if w0 is None:
            w0 = w.copy()
            best_w = np.full_like(w, np.inf)
        better = w < best_w
        best_w = np.where(better, w, best_w)
        best_a = np.where(better[..., None], a, best_a)
        if s == steps:
            break
        g = leb_grad(dyn, a[..., :dyn.nx], a[..., dyn.nx:], sigma, -ones, ones, mu=box_mu(a))
        ga = np.concatenate([g["gz"], g["gv"]], -1)
        if fixed_box:
            ga = ga - g["gmu"]
        a = np.clip(a - lr * (1.0 - s / steps) * r * np.sign(ga), a0 - r, a0 + r)
    return best_a, best_w, w0
