"""Pins of the oracle's nominal-point refinement (oracle/pgd.py), for both
readings of the covered set (the box travelling with the nominal point, and
a fixed box): the search stays in its box, never returns a wider bound than
the start, leaves the start alone at radius 0, and its first sign step
lowers the width by what the gradient predicts (first order, small steps,
away from kinks).  On the travelling box it also beats random nominal points
drawn from the same search box at four bound evaluations per step, the
comparison of the paper's Table II."""
import numpy as np
import pytest

import workloads as W
from oracle import pgd


def _offcentre(b, seed, frac=0.5):
    """A start a0 off the box centre c: a0 = c + U(-frac, frac) sigma, mu0 = c - a0."""
    rng = np.random.default_rng(seed)
    c = np.concatenate([b.z, b.v], -1)
    off = rng.uniform(-frac, frac, c.shape) * b.sigma
    a0 = c + off
    nx = b.z.shape[-1]
    return a0[..., :nx], a0[..., nx:], -off


def _box_mu(fixed, a0, mu0, a):
    return a0 + mu0 - a if fixed else mu0


@pytest.mark.parametrize("fixed", [False, True])
def test_pgd_invariants(orc, fixed):
    b = W.planar_quad_cfg(N=8)
    d = orc.Dyn.like(b.dyn)
    if fixed:
        z0, v0, mu0 = _offcentre(b, 1)
    else:
        z0, v0, mu0 = b.z, b.v, np.zeros(b.sigma.shape)
    a, w, w0 = pgd.pgd_nominal(d, z0, v0, b.sigma, mu0=mu0, radius=0.5, steps=6, lr=0.3, fixed_box=fixed)
    a0 = np.concatenate([z0, v0], -1)
    assert (np.abs(a - a0) <= 0.5 * b.sigma * (1 + 1e-12)).all()
    assert (w <= w0).all() and (w < w0).mean() >= 0.75
    np.testing.assert_array_equal(pgd.width(d, a, _box_mu(fixed, a0, mu0, a), b.sigma), w)
    np.testing.assert_array_equal(pgd.width(d, a0, _box_mu(fixed, a0, mu0, a0), b.sigma), w0)
    a_, w_, w0_ = pgd.pgd_nominal(d, z0, v0, b.sigma, mu0=mu0, radius=0.0, steps=3, lr=0.3, fixed_box=fixed)
    assert np.array_equal(a_, a0) and np.array_equal(w_, w0_)


@pytest.mark.parametrize("fixed", [False, True])
def test_first_step_follows_the_gradient(orc, fixed):
    """W(a0 - h r sign(g)) - W(a0) = -h sum_i |g_i| r_i + O(h^2) at starts whose
    margin to every kink exceeds the step."""
    b = W.chain_batch(21, 1, 6, 3)
    d = orc.Dyn.like(b.dyn)
    if fixed:
        z0, v0, mu0 = _offcentre(b, 2)
    else:
        z0, v0, mu0 = b.z, b.v, np.zeros(b.sigma.shape)
    a0 = np.concatenate([z0, v0], -1)
    r = 0.5 * b.sigma
    ones = np.ones(b.z.shape)
    # the travelling box never moves mu, so its kinks in mu are not crossed
    g = orc.leb_grad(d, z0, v0, b.sigma, -ones, ones, mu=mu0 if fixed else None)
    ga = np.concatenate([g["gz"], g["gv"]], -1) - (g["gmu"] if fixed else 0.0)
    w0 = pgd.width(d, a0, mu0, b.sigma)
    ok = g["margin"] > 1e-3
    assert ok.sum() >= 3
    for h in (1e-5, 1e-6):
        a1 = a0 - h * r * np.sign(ga)
        pred = -h * (np.abs(ga) * r).sum(-1)
        dw = pgd.width(d, a1, _box_mu(fixed, a0, mu0, a1), b.sigma) - w0
        assert np.allclose(dw[ok], pred[ok], rtol=1e-3, atol=0), (h, dw[ok], pred[ok])


@pytest.mark.parametrize("case", ["planar_quad", "chain"])
def test_pgd_beats_sampling_on_the_travelling_box(orc, case):
    b = W.planar_quad_cfg(N=12) if case == "planar_quad" else W.chain_batch(7, 1, 8, 4)
    d = orc.Dyn.like(b.dyn)
    steps, radius = 10, 1.0
    a, w, w0 = pgd.pgd_nominal(d, b.z, b.v, b.sigma, radius=radius, steps=steps, lr=0.3)
    a0 = np.concatenate([b.z, b.v], -1)
    rng = np.random.default_rng(5)
    best = w0.copy()
    zero = np.zeros(a0.shape)
    for _ in range(4 * steps):
        best = np.minimum(best, pgd.width(d, a0 + rng.uniform(-radius, radius, a0.shape) * b.sigma, zero, b.sigma))
    assert (w <= best).all()
    assert (w < w0).all() and w.mean() <= 0.97 * w0.mean()
