"""Pins of the oracle's satellite and 3-D quadrotor dynamics (dynamics
appendix) and of its three interval-Hessian forms on them (section IV.A):
the hand gradients against central differences of the values, every
Hessian entry at a point against central differences of the gradients (and
every other entry against zero), the satellite's bounds against the exact
range of its bilinear remainder over the box vertices, Corollary 1's
ordering on the quadrotor, sampled soundness, and the unbounded rows where
cos(theta) may vanish."""
import itertools

import numpy as np
import pytest

import workloads as W


def _dyn(orc, name):
    return orc.Dyn.like(W.SATELLITE if name == "satellite" else W.QUAD3D)


def _points(name, seed, count):
    z, v = W.small_nominals(W.SATELLITE if name == "satellite" else W.QUAD3D, seed, count)
    return np.concatenate([z, v], 1)


@pytest.mark.parametrize("name", ["satellite", "quad3d"])
def test_gradient_matches_central_differences(orc, name):
    d = _dyn(orc, name)
    h = 1e-6
    for a in _points(name, 3, 4):
        for l in range(d.nx):
            _, g = orc.nonlin(d, l, a)
            for k in range(d.n):
                e = np.zeros(d.n)
                e[k] = h
                fd = (orc.nonlin(d, l, a + e)[0] - orc.nonlin(d, l, a - e)[0]) / (2 * h)
                assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(g[k])), (l, k, fd, g[k])


@pytest.mark.parametrize("name", ["satellite", "quad3d"])
def test_hessian_entries_match_differences_of_the_gradient(orc, name):
    """At a point box the entry enclosure is the Hessian value; every pair
    the dynamics does not couple is a structural zero (status 0)."""
    d = _dyn(orc, name)
    h = 1e-6
    for a in _points(name, 5, 3):
        for l in range(d.nx):
            for k in range(d.n):
                e = np.zeros(d.n)
                e[k] = h
                col = (orc.nonlin(d, l, a + e)[1] - orc.nonlin(d, l, a - e)[1]) / (2 * h)   # H[:, k]
                for j in range(k + 1):
                    st, lo, hi = orc.hess_entry(d, l, k, j, a, a)
                    fd = col[j]
                    if st == 0:
                        assert abs(fd) <= 1e-6, (l, k, j, fd)
                        continue
                    assert st == 1
                    assert hi - lo <= 1e-12 * max(1.0, abs(lo))
                    assert abs(0.5 * (lo + hi) - fd) <= 1e-6 * max(1.0, abs(fd)), (l, k, j, lo, fd)


def test_satellite_bounds_are_the_exact_remainder_range(orc):
    """The satellite's remainder is bilinear, each row a sum of products of
    distinct coordinates, so its range over a box is attained at vertices and
    is the interval sum of the products: all three forms give it (up to
    rounding) for boxes symmetric about the nominal."""
    d = _dyn(orc, "satellite")
    z, v = W.small_nominals(W.SATELLITE, 11, 3)
    rng = np.random.default_rng(0)
    sigma = rng.uniform(0.01, 0.3, (3, d.n))
    nom = np.concatenate([z, v], 1)
    verts = np.array(list(itertools.product((-1.0, 1.0), repeat=d.n)))
    for mode in ("path", "expand", "classic"):
        lo, hi, fl = orc.leb(d, z, v, sigma, mode=mode)
        assert (fl == 0).all()
        for u in range(3):
            pts = nom[u] + verts * sigma[u]
            r, eps = orc.remainder(d, nom[u:u + 1], pts, np.zeros(len(pts), dtype=np.int64))
            rlo, rhi = r.min(0), r.max(0)
            scale = np.maximum(np.abs(rlo), np.abs(rhi)) + 1e-300
            assert (np.abs(lo[u] - rlo) <= 1e-9 * scale).all(), (mode, lo[u], rlo)
            assert (np.abs(hi[u] - rhi) <= 1e-9 * scale).all(), (mode, hi[u], rhi)


@pytest.mark.parametrize("eps", [0.01, 0.1, 0.2])
def test_quad3d_corollary_1_ordering(orc, eps):
    """Symmetric boxes: PATH inside EXPAND inside CLASSIC, row by row, and
    strictly narrower on the attitude rows for most units."""
    d = _dyn(orc, "quad3d")
    b = W.small_batch(W.QUAD3D, 21, 40, eps)
    P = orc.leb(d, b.z, b.v, b.sigma, mode="path")
    E = orc.leb(d, b.z, b.v, b.sigma, mode="expand")
    C = orc.leb(d, b.z, b.v, b.sigma, mode="classic")
    tol = 1e-12
    for (l1, h1, _), (l2, h2, _) in ((P, E), (E, C)):
        s = np.maximum(np.abs(l2), np.abs(h2)) * tol
        assert (l1 >= l2 - s).all() and (h1 <= h2 + s).all()
    wp = (P[1] - P[0]).sum(-1)
    we = (E[1] - E[0]).sum(-1)
    wc = (C[1] - C[0]).sum(-1)
    assert (wp < we).mean() >= 0.9 and (we < wc).mean() >= 0.9


@pytest.mark.parametrize("eps", [0.01, 0.2])
def test_quad3d_sampled_soundness(orc, eps):
    d = _dyn(orc, "quad3d")
    b = W.small_batch(W.QUAD3D, 31, 24, eps)
    lo, hi, fl = orc.leb(d, b.z, b.v, b.sigma)
    assert (fl == 0).all()
    nom = np.concatenate([b.z, b.v], -1)[0]
    rng = np.random.default_rng(1)
    per = 2000
    blo, bhi = orc.box(nom, b.sigma[0])
    pts = W.sample_box_points(rng, blo, bhi, per).reshape(-1, d.n)
    uo = np.repeat(np.arange(nom.shape[0]), per)
    r, e = orc.remainder(d, nom, pts, uo)
    L = lo[0][uo]
    H = hi[0][uo]
    assert not ((r > H + e) | (r < L - e)).any()
    # and the bound is not vacuous: the samples reach a fair share of it
    wid = (H - L).reshape(nom.shape[0], per, d.nx)[:, 0].sum(-1)
    swid = (r.reshape(nom.shape[0], per, d.nx).max(1) - r.reshape(nom.shape[0], per, d.nx).min(1)).sum(-1)
    assert (swid >= 0.2 * wid).all()


def test_quad3d_unbounded_where_cos_theta_may_vanish(orc):
    d = _dyn(orc, "quad3d")
    b = W.small_batch(W.QUAD3D, 41, 2, 0.1)
    z = b.z.copy()
    z[0, 0, 4] = np.pi / 2 - 0.05            # the theta interval reaches past pi/2
    lo, hi, fl = orc.leb(d, z, b.v, b.sigma)
    assert fl[0, 0] & orc.FLAG_UNBOUNDED and not fl[0, 1] & orc.FLAG_UNBOUNDED
    assert np.isinf(lo[0, 0, [3, 5]]).all() and np.isinf(hi[0, 0, [3, 5]]).all()
    assert np.isfinite(lo[0, 0, [4, 6, 7, 8]]).all()
