"""Pins of the oracle gradient of the path-based bound: forward-mode dual
numbers against central finite differences (h = 1e-6) of the oracle bound
itself, at units whose selections are clear of every kink."""
import numpy as np
import pytest

import workloads as W

H = 1e-6


def _fd_check(orc, d, z, v, sg, mu, gl, gh, g, entries, tol=1e-6):
    def L(z_, v_, s_, m_):
        lo, hi, _ = orc.leb(d, z_, v_, s_, mu=m_)
        return float((gl * lo + gh * hi).sum())

    checked = 0
    for (name, key, idx) in entries:
        arrs = {"z": z, "v": v, "s": sg, "m": mu}
        a1 = {k: a.copy() for k, a in arrs.items()}
        a2 = {k: a.copy() for k, a in arrs.items()}
        a1[name][idx] += H
        a2[name][idx] -= H
        fd = (L(a1["z"], a1["v"], a1["s"], a1["m"]) - L(a2["z"], a2["v"], a2["s"], a2["m"])) / (2 * H)
        an = g[key][idx]
        scale = max(abs(an), 1e-3 * np.abs(g[key]).max(), 1e-12)
        assert abs(fd - an) <= tol * scale + 1e-10, (name, idx, fd, an)
        checked += 1
    return checked


@pytest.mark.parametrize("n_units,seed", [(1, 0), (3, 1), (4, 2)])
def test_gradient_matches_finite_differences(orc, n_units, seed):
    b = W.chain_batch(300 + seed, 1, 4, n_units)
    d = orc.Dyn.like(b.dyn)
    r = np.random.default_rng(seed)
    mu = r.uniform(-0.02, 0.02, b.sigma.shape)
    gl = r.normal(size=(1, 4, d.nx))
    gh = r.normal(size=(1, 4, d.nx))
    g = orc.leb_grad(d, b.z, b.v, b.sigma, gl, gh, mu=mu)
    ok_units = np.nonzero(g["margin"][0] > 1e-3)[0]
    assert len(ok_units) >= 2
    entries = []
    for t in ok_units[:3]:
        for c in range(d.nx):
            entries.append(("z", "gz", (0, t, c)))
        for c in range(d.nu):
            entries.append(("v", "gv", (0, t, c)))
        for c in range(d.n):
            entries.append(("s", "gsigma", (0, t, c)))
            entries.append(("m", "gmu", (0, t, c)))
    # restrict the FD to the units checked: other units' g must not matter
    assert _fd_check(orc, d, b.z, b.v, b.sigma, mu, gl, gh, g, entries) == len(entries)


def test_gradient_symmetric_boxes_sigma_and_nominal(orc):
    """mu = 0 (symmetric Delta): the bound is smooth in z, v and sigma even
    though product selections tie; check those directions."""
    b = W.planar_quad_cfg()
    d = orc.Dyn.like(b.dyn)
    r = np.random.default_rng(5)
    gl = r.normal(size=b.z.shape)
    gh = r.normal(size=b.z.shape)
    mu = np.zeros_like(b.sigma)
    g = orc.leb_grad(d, b.z, b.v, b.sigma, gl, gh, mu=mu)
    entries = []
    for t in range(0, b.N, 4):
        entries += [("z", "gz", (0, t, 2)), ("v", "gv", (0, t, 0)), ("v", "gv", (0, t, 1))]
        entries += [("s", "gsigma", (0, t, c)) for c in (2, 6, 7)]
    _fd_check(orc, d, b.z, b.v, b.sigma, mu, gl, gh, g, entries)
    # linear coordinates carry no gradient
    assert (g["gz"][..., [0, 1, 3, 4, 5]] == 0).all()
    assert (g["gsigma"][..., [0, 1, 3, 4, 5]] == 0).all()


def test_gradient_of_zero_upstream_is_zero(orc):
    b = W.chain_batch(7, 1, 3, 3)
    d = orc.Dyn.like(b.dyn)
    z0 = np.zeros((1, 3, d.nx))
    g = orc.leb_grad(d, b.z, b.v, b.sigma, z0, z0)
    assert all((g[k] == 0).all() for k in ("gz", "gv", "gsigma"))


def test_kink_margin_counts_only_slope_changes(orc):
    """The margin rule: a tie between candidate endpoints is a kink of L
    along a direction only when the tied candidates change at different
    rates along it.  On symmetric boxes (mu = 0) lo*lo and hi*hi of a
    displacement product tie exactly; along sigma, z and v they move at the
    same rate (no kink: the margin stays away from 0 and one-sided
    differences agree), along mu they move at opposite rates (a kink: the
    margin is 0 and the one-sided differences differ)."""
    b = W.planar_quad_cfg()
    d = orc.Dyn.like(b.dyn)
    r = np.random.default_rng(5)
    gl = r.normal(size=b.z.shape)
    gh = r.normal(size=b.z.shape)
    mu0 = np.zeros_like(b.sigma)
    smooth = orc.leb_grad(d, b.z, b.v, b.sigma, gl, gh)
    kinked = orc.leb_grad(d, b.z, b.v, b.sigma, gl, gh, mu=mu0)
    assert (smooth["margin"] > 1e-3).mean() >= 0.9
    assert (kinked["margin"] < 1e-12).all()

    def L(z_, v_, s_, m_):
        lo, hi, _ = orc.leb(d, z_, v_, s_, mu=m_)
        return float((gl * lo + gh * hi).sum())

    t = int(np.nonzero(smooth["margin"][0] > 1e-3)[0][0])
    base = L(b.z, b.v, b.sigma, mu0)

    def one_sided(name, c):
        arrs = {"z": b.z, "v": b.v, "s": b.sigma, "m": mu0}
        up = {k: a.copy() for k, a in arrs.items()}
        dn = {k: a.copy() for k, a in arrs.items()}
        up[name][0, t, c] += H
        dn[name][0, t, c] -= H
        return ((L(up["z"], up["v"], up["s"], up["m"]) - base) / H,
                (base - L(dn["z"], dn["v"], dn["s"], dn["m"])) / H)

    for name, c in (("s", 2), ("z", 2), ("v", 0)):
        right, left = one_sided(name, c)
        # smooth: the one-sided slopes differ only by the curvature term O(h)
        assert abs(right - left) <= 1e-4 * max(abs(right), 1e-9), (name, right, left)
    right, left = one_sided("m", 2)
    assert abs(right - left) > 1e-2 * max(abs(right), abs(left)), (right, left)
