"""Pins of the FP64 oracle's interval bounds (Theorem 1, Corollary 1 and
the expanded / classic forms of section IV.A) against facts that do not
come from the oracle itself: closed forms, brute-force ranges on grids,
finite-difference Hessians of the dynamics, sampled true remainders and
the invariants the theorems imply."""
import math

import numpy as np
import pytest

import workloads as W


def _rng(s):
    return np.random.default_rng(s)


# ----------------------------------------------------------------- basics

def test_linear_dynamics_zero(orc):
    """Affine dynamics have a zero Hessian, so the remainder is exactly 0."""
    d = orc.Dyn("linear", nx=3, nu=2)
    r = _rng(0)
    lo, hi, fl = orc.leb(d, r.normal(size=(7, 3)), r.normal(size=(7, 2)), r.uniform(0, 1, (7, 5)))
    assert (lo == 0).all() and (hi == 0).all() and (fl == 0).all()


def _quad_closed_form(Q, rho):
    """Symmetric box of radii rho: the bound is
    hi = sum_{j<k} |Q_kj| rho_j rho_k + 1/2 sum max(Q_kk,0) rho_k^2,
    lo = -sum_{j<k} |Q_kj| rho_j rho_k + 1/2 sum min(Q_kk,0) rho_k^2."""
    m, n, _ = Q.shape
    lo = np.zeros(m)
    hi = np.zeros(m)
    for l in range(m):
        for k in range(n):
            for j in range(k):
                t = abs(Q[l, k, j]) * rho[j] * rho[k]
                lo[l] -= t
                hi[l] += t
            hi[l] += 0.5 * max(Q[l, k, k], 0.0) * rho[k] ** 2
            lo[l] += 0.5 * min(Q[l, k, k], 0.0) * rho[k] ** 2
    return lo, hi


def _rand_sym(r, m, n):
    A = r.normal(size=(m, n, n))
    return 0.5 * (A + A.transpose(0, 2, 1))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_quadratic_closed_form(orc, seed):
    r = _rng(seed)
    nx, nu = 3, 2
    n = nx + nu
    Q = _rand_sym(r, nx, n)
    Q[:, 1, 0] = Q[:, 0, 1] = 0.0          # include structural zeros
    d = orc.Dyn("quadratic", nx=nx, nu=nu, Q=Q)
    for t in (1.0, 0.5, 3.0):
        rho = t * r.uniform(0.01, 1.0, n)
        z = r.normal(size=nx)
        v = r.normal(size=nu)
        lo, hi, _ = orc.leb(d, z[None], v[None], rho[None])
        elo, ehi = _quad_closed_form(Q, rho)
        np.testing.assert_allclose(lo[0], elo, rtol=1e-13, atol=0)
        np.testing.assert_allclose(hi[0], ehi, rtol=1e-13, atol=0)


def test_quadratic_t2_scaling_and_diagonal_tight(orc):
    r = _rng(5)
    n = 4
    Q = np.zeros((2, n, n))
    Q[0] = np.diag([1.5, -0.5, 2.0, 0.0])
    Q[1] = np.diag([-1.0, -2.0, 0.25, 3.0])
    d = orc.Dyn("quadratic", nx=2, nu=2, Q=Q)
    rho = r.uniform(0.1, 1.0, n)
    z, v = r.normal(size=(1, 2)), r.normal(size=(1, 2))
    lo1, hi1, _ = orc.leb(d, z, v, rho[None])
    lo2, hi2, _ = orc.leb(d, z, v, 2.0 * rho[None])
    np.testing.assert_allclose(lo2, 4.0 * lo1, rtol=1e-14)
    np.testing.assert_allclose(hi2, 4.0 * hi1, rtol=1e-14)
    # diagonal Q: the remainder 1/2 sum Q_kk d_k^2 attains both ends at box vertices / centre
    verts = np.array(np.meshgrid(*[[-1, 0, 1]] * n)).reshape(n, -1).T * rho
    rr = 0.5 * np.einsum("lk,sk->sl", np.stack([np.diag(Q[0]), np.diag(Q[1])]), verts ** 2)
    np.testing.assert_allclose(rr.max(0), hi1[0], rtol=1e-14)
    np.testing.assert_allclose(rr.min(0), lo1[0], rtol=1e-14)


def test_quadratic_off_centre_contains_brute_force(orc):
    """Boxes with mu != 0 (hull with the nominal point): every sampled
    remainder 1/2 d^T Q d lies in the bound."""
    r = _rng(7)
    nx, nu = 2, 1
    n = 3
    Q = _rand_sym(r, nx, n)
    d = orc.Dyn("quadratic", nx=nx, nu=nu, Q=Q)
    z, v = r.normal(size=(1, nx)), r.normal(size=(1, nu))
    sg = r.uniform(0.1, 0.5, (1, n))
    mu = r.uniform(-0.7, 0.7, (1, n))
    lo, hi, fl = orc.leb(d, z, v, sg, mu=mu)
    assert fl[0] & orc.FLAG_HULL
    dlo = np.minimum(mu - sg, 0)[0]
    dhi = np.maximum(mu + sg, 0)[0]
    g = np.array(np.meshgrid(*[np.linspace(dlo[i], dhi[i], 41) for i in range(n)])).reshape(n, -1).T
    rr = 0.5 * np.einsum("sk,lkj,sj->sl", g, Q, g)
    assert (rr.max(0) <= hi[0] + 1e-15).all() and (rr.min(0) >= lo[0] - 1e-15).all()


# ------------------------------------------------------------ sin / cos

def test_libm_sin_cos_within_one_ulp():
    """The oracle widens libm sin/cos by 4 ulps; check libm's error is below
    1 ulp on random arguments against 50-digit mpmath values."""
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 50
    r = _rng(11)
    xs = np.concatenate([r.uniform(-4, 4, 300), r.uniform(-1e-3, 1e-3, 50), r.uniform(-40, 40, 100)])
    for x in xs:
        for f, mf in ((math.sin, mpmath.sin), (math.cos, mpmath.cos)):
            y = f(float(x))
            ex = mf(mpmath.mpf(float(x)))
            ulp = math.ulp(y) if y != 0 else 5e-324
            assert abs(mpmath.mpf(y) - ex) <= ulp


@pytest.mark.parametrize("a,b", [(-0.3, 0.2), (1.2, 1.9), (1.5, 4.9), (-2.0, -1.0), (3.0, 3.3),
                                 (-7.0, 1.0), (0.0, 0.0), (6.0, 6.5), (-1.5707963, -1.5707962)])
def test_interval_sin_cos_contains_dense_grid(orc, a, b):
    xs = np.linspace(a, b, 20001)
    s = orc.isin(a, b)
    c = orc.icos(a, b)
    assert s[0] <= np.sin(xs).min() and s[1] >= np.sin(xs).max()
    assert c[0] <= np.cos(xs).min() and c[1] >= np.cos(xs).max()
    # tight: within a few ulps of the grid range plus grid resolution
    res = (b - a) / 20000
    assert s[1] - np.sin(xs).max() <= res + 1e-14 and np.sin(xs).min() - s[0] <= res + 1e-14
    assert c[1] - np.cos(xs).max() <= res + 1e-14 and np.cos(xs).min() - c[0] <= res + 1e-14


# ------------------------------------------------------------ 1-D, 2-D

@pytest.mark.parametrize("x0,rho", [(0.3, 0.2), (1.4, 0.5), (-2.0, 0.05), (0.0, 0.3)])
def test_sin1d_grid(orc, x0, rho):
    """f = sin(a): the grid range of r over [x0-rho, x0+rho] lies in R."""
    d = orc.Dyn("sin1d", nx=1)
    lo, hi, _ = orc.leb(d, np.array([[x0]]), np.zeros((1, 0)), np.array([[rho]]))
    a = np.linspace(x0 - rho, x0 + rho, 100001)
    r = np.sin(a) - np.sin(x0) - np.cos(x0) * (a - x0)
    eps = 1e-15
    assert r.max() <= hi[0, 0] + eps and r.min() >= lo[0, 0] - eps


def test_sin1d_tight_as_radius_shrinks(orc):
    """As rho -> 0 the single-term bound 1/2 (-sin X) [0, rho^2] approaches
    the true range (ratio of widths -> 1)."""
    d = orc.Dyn("sin1d", nx=1)
    x0 = 0.9
    ratios = []
    for rho in (0.2, 0.02, 0.002):
        lo, hi, _ = orc.leb(d, np.array([[x0]]), np.zeros((1, 0)), np.array([[rho]]))
        a = np.linspace(x0 - rho, x0 + rho, 20001)
        r = np.sin(a) - np.sin(x0) - np.cos(x0) * (a - x0)
        ratios.append((r.max() - r.min()) / (hi[0, 0] - lo[0, 0]))
    assert ratios[0] < ratios[1] < ratios[2] and ratios[2] > 0.99


def test_sincos2d_entries_exact_ranges(orc):
    """All entries of f1 = sin a1 cos a2, f2 = cos a1 sin a2 are single-use
    products, so each enclosure over its prefix set equals the exact range
    of the entry (checked on a 2001 x 2001 grid)."""
    d = orc.Dyn("sincos2d", nx=2)
    x = np.array([0.4, -1.1])
    rho = np.array([0.3, 0.25])
    lo_b, hi_b = x - rho, x + rho
    g1 = np.linspace(lo_b[0], hi_b[0], 2001)
    g2 = np.linspace(lo_b[1], hi_b[1], 2001)
    A1, A2 = np.meshgrid(g1, g2, indexing="ij")
    exact = {
        (0, 0, 0): (-np.sin(g1) * np.cos(x[1])),
        (0, 1, 0): (-np.cos(g1) * np.sin(x[1])),
        (0, 1, 1): (-np.sin(A1) * np.cos(A2)),
        (1, 0, 0): (-np.cos(g1) * np.sin(x[1])),
        (1, 1, 0): (-np.sin(g1) * np.cos(x[1])),
        (1, 1, 1): (-np.cos(A1) * np.sin(A2)),
    }
    for (l, k, j), vals in exact.items():
        p = j  # prefix: coordinates 0..j free
        blo = np.where(np.arange(2) <= p, lo_b, x)
        bhi = np.where(np.arange(2) <= p, hi_b, x)
        st, elo, ehi = orc.hess_entry(d, l, k, j, blo, bhi)
        assert st == 1
        res = 2e-3 * rho.max()
        assert elo <= vals.min() + 1e-14 and ehi >= vals.max() - 1e-14
        assert vals.min() - elo <= res and ehi - vals.max() <= res
    # remainder on the grid lies in R
    lo, hi, _ = orc.leb(d, x[None], np.zeros((1, 0)), rho[None])
    r1 = np.sin(A1) * np.cos(A2) - np.sin(x[0]) * np.cos(x[1]) - (
        np.cos(x[0]) * np.cos(x[1]) * (A1 - x[0]) - np.sin(x[0]) * np.sin(x[1]) * (A2 - x[1]))
    r2 = np.cos(A1) * np.sin(A2) - np.cos(x[0]) * np.sin(x[1]) - (
        -np.sin(x[0]) * np.sin(x[1]) * (A1 - x[0]) + np.cos(x[0]) * np.cos(x[1]) * (A2 - x[1]))
    assert r1.max() <= hi[0, 0] + 1e-14 and r1.min() >= lo[0, 0] - 1e-14
    assert r2.max() <= hi[0, 1] + 1e-14 and r2.min() >= lo[0, 1] - 1e-14


# ----------------------------------------------------------- planar quad

def test_planar_quad_entries_are_exact_ranges(orc):
    """cfg0 entries use Theta once: c s sin(Theta), -c s cos(Theta), -c cos,
    -c sin over the prefix set X^(theta) (u pinned).  Their enclosure equals
    the exact range (dense grid over Theta)."""
    b = W.planar_quad_cfg()
    d = orc.Dyn.like(b.dyn)
    c = b.dyn.dt / b.dyn.m
    for t in range(b.N):
        nom = np.concatenate([b.z[0, t], b.v[0, t]])
        blo, bhi = orc.box(nom, b.sigma[0, t])
        th = np.linspace(blo[2], bhi[2], 20001)
        s = nom[6] + nom[7]
        p = 2
        plo = np.where(np.arange(8) <= p, blo, nom)
        phi_ = np.where(np.arange(8) <= p, bhi, nom)
        cases = {(3, 2, 2): c * s * np.sin(th), (3, 6, 2): -c * np.cos(th), (3, 7, 2): -c * np.cos(th),
                 (4, 2, 2): -c * s * np.cos(th), (4, 6, 2): -c * np.sin(th), (4, 7, 2): -c * np.sin(th)}
        for (l, k, j), vals in cases.items():
            st, elo, ehi = orc.hess_entry(d, l, k, j, plo, phi_)
            assert st == 1
            res = 1e-4 * (bhi[2] - blo[2]) * c * max(s, 1) + 1e-15
            assert elo <= vals.min() + 1e-15 and ehi >= vals.max() - 1e-15
            assert vals.min() - elo <= res and ehi - vals.max() <= res
        # u-u entries and linear rows are structural zeros
        for (l, k, j) in ((3, 6, 6), (3, 7, 6), (0, 2, 2), (2, 6, 2), (5, 7, 6)):
            st, _, _ = orc.hess_entry(d, l, k, j, plo, phi_)
            assert st == 0


def _fd_hessian_row(orc, d, l, a, h=1e-5):
    n = d.n
    H = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = h
        _, gp = orc.nonlin(d, l, a + e)
        _, gm = orc.nonlin(d, l, a - e)
        H[:, k] = (gp - gm) / (2 * h)
    return 0.5 * (H + H.T)


@pytest.mark.parametrize("n_units", [1, 3])
def test_chain_point_hessian_matches_finite_differences(orc, n_units):
    """On a degenerate box (a point) every enclosure collapses to the point
    Hessian.  Compare every entry (including structural zeros) against
    central differences of the analytic gradient of the dynamics."""
    d = orc.Dyn.chain(n_units)
    b = W.chain_batch(13, 1, 3, n_units)
    for t in range(3):
        a = np.concatenate([b.z[0, t], b.v[0, t]])
        for l in range(d.nx):
            Hfd = _fd_hessian_row(orc, d, l, a)
            for k in range(d.n):
                for j in range(k + 1):
                    st, lo, hi = orc.hess_entry(d, l, k, j, a, a)
                    if st == 0:
                        assert abs(Hfd[k, j]) < 1e-7, (l, k, j, Hfd[k, j])
                    else:
                        assert st == 1
                        assert hi - lo <= 1e-12 * max(1, abs(hi))
                        assert abs(0.5 * (lo + hi) - Hfd[k, j]) < 1e-6 * max(1, abs(Hfd[k, j])), (l, k, j)


def test_chain_spring_entries_contain_grid_range(orc):
    """Each spring entry's enclosure over its prefix set contains the entry's
    values (finite-difference Hessian) on a coarse grid of the free position
    coordinates."""
    d = orc.Dyn.chain(3)
    b = W.chain_batch(21, 1, 1, 3, sigma_range=(0.05, 0.15))
    a = np.concatenate([b.z[0, 0], b.v[0, 0]])
    blo, bhi = orc.box(a, b.sigma[0, 0])
    l = 6 * 1 + 3          # vx of the middle node (both springs)
    pos = [0, 1, 6, 7, 12, 13]
    for k in pos:
        for j in pos:
            if j > k:
                continue
            plo = np.where(np.arange(d.n) <= j, blo, a)
            phi_ = np.where(np.arange(d.n) <= j, bhi, a)
            st, elo, ehi = orc.hess_entry(d, l, k, j, plo, phi_)
            if st == 0:
                continue
            free = [c for c in pos if c <= j]
            grids = np.array(np.meshgrid(*[np.linspace(plo[c], phi_[c], 4) for c in free])).reshape(len(free), -1).T
            for gpt in grids:
                p = a.copy()
                p[free] = gpt
                H = _fd_hessian_row(orc, d, l, p, h=1e-4)
                assert elo - 1e-6 <= H[k, j] <= ehi + 1e-6, (k, j)


# ------------------------------------------------------------ invariants

def _chain_inputs(seed=2, n_units=28, N=6):
    b = W.chain_batch(seed, 1, N, n_units)
    return b


def test_zero_radius_gives_exact_zero(orc):
    for b in (W.planar_quad_cfg(), _chain_inputs()):
        d = orc.Dyn.like(b.dyn)
        lo, hi, fl = orc.leb(d, b.z, b.v, np.zeros_like(b.sigma))
        assert (lo == 0).all() and (hi == 0).all() and (fl == 0).all()


def test_zero_in_bound_and_isotone(orc):
    """0 = r(a~) is in R; shrinking the box shrinks R (inclusion isotonicity)."""
    for b in (W.planar_quad_cfg(), _chain_inputs(3)):
        d = orc.Dyn.like(b.dyn)
        lo, hi, _ = orc.leb(d, b.z, b.v, b.sigma)
        assert (lo <= 0).all() and (hi >= 0).all()
        shrink = b.sigma * _rng(1).uniform(0.3, 1.0, b.sigma.shape)
        lo2, hi2, _ = orc.leb(d, b.z, b.v, shrink)
        assert (lo2 >= lo).all() and (hi2 <= hi).all()


def test_corollary1_path_expand_classic(orc):
    """Corollary 1: for symmetric Delta, R_path in R_expand in R_classic."""
    for b in (W.planar_quad_cfg(), _chain_inputs(4), W.chain_batch(5, 1, 4, 8)):
        d = orc.Dyn.like(b.dyn)
        lp, hp, _ = orc.leb(d, b.z, b.v, b.sigma, mode="path")
        le, he, _ = orc.leb(d, b.z, b.v, b.sigma, mode="expand")
        lc, hc, _ = orc.leb(d, b.z, b.v, b.sigma, mode="classic")
        # inclusions hold in exact arithmetic; allow the oracle's outward
        # rounding (a few ulps) where two forms coincide exactly
        tol = 1e-13 * np.maximum(np.abs(hc), np.abs(lc))
        assert (le <= lp + tol).all() and (hp <= he + tol).all()
        assert (lc <= le + tol).all() and (he <= hc + tol).all()
        # and strictly tighter somewhere (the path sets matter)
        assert ((hp < he) | (lp > le)).any()


def test_nominal_outside_box_is_hulled(orc):
    """|mu| > sigma: the box is extended to contain a~ and flagged."""
    b = W.planar_quad_cfg()
    d = orc.Dyn.like(b.dyn)
    mu = np.zeros_like(b.sigma)
    mu[..., 2] = 3.0 * b.sigma[..., 2]
    lo, hi, fl = orc.leb(d, b.z, b.v, b.sigma, mu=mu)
    assert (fl & orc.FLAG_HULL).all()
    assert (lo <= 0).all() and (hi >= 0).all()


def test_singular_spring_is_unbounded(orc):
    d = orc.Dyn.chain(2)
    b = W.chain_batch(8, 1, 1, 2)
    z = b.z.copy()
    z[0, 0, 6] = z[0, 0, 0] - d.c.rest_len        # node 1 on top of node 0
    z[0, 0, 7] = z[0, 0, 1]
    lo, hi, fl = orc.leb(d, z, b.v, b.sigma)
    assert fl[0, 0] & orc.FLAG_UNBOUNDED
    assert np.isneginf(lo[0, 0, 3]) and np.isposinf(hi[0, 0, 3])
    assert lo[0, 0, 0] == 0 and hi[0, 0, 0] == 0


def test_bad_input_flagged(orc):
    """Non-finite inputs and negative radii make every row of the unit
    [-inf, inf] with the BAD_INPUT flag; other units are unaffected."""
    b = W.planar_quad_cfg()
    d = orc.Dyn.like(b.dyn)
    z = b.z.copy()
    z[0, 3, 1] = np.nan
    sg = b.sigma.copy()
    sg[0, 5, 7] = -0.1
    lo, hi, fl = orc.leb(d, z, b.v, sg)
    for t in (3, 5):
        assert fl[0, t] & orc.FLAG_BAD_INPUT
        assert np.isneginf(lo[0, t]).all() and np.isposinf(hi[0, t]).all()
    assert np.isfinite(lo[0, 4]).all() and fl[0, 4] == 0


# ------------------------------------------------------------- sampling

def _violations(orc, d, z, v, sigma, lo, hi, per_box, seed, mu=None):
    nom = np.concatenate([z, v], -1).reshape(-1, d.n)
    sg = sigma.reshape(-1, d.n)
    blo, bhi = orc.box(nom, sg, None if mu is None else mu.reshape(-1, d.n))
    pts = W.sample_box_points(W.rng_for(seed), blo, bhi, per_box)
    U = nom.shape[0]
    r, eps = orc.remainder(d, nom, pts.reshape(-1, d.n), np.repeat(np.arange(U), per_box))
    r = r.reshape(U, per_box, d.nx)
    eps = eps.reshape(U, per_box, d.nx)
    L = lo.reshape(U, 1, d.nx)
    H = hi.reshape(U, 1, d.nx)
    return int(((r > H + eps) | (r < L - eps)).sum()), r


def test_sampled_soundness_planar_quad(orc):
    b = W.planar_quad_cfg()
    d = orc.Dyn.like(b.dyn)
    lo, hi, _ = orc.leb(d, b.z, b.v, b.sigma)
    nv, r = _violations(orc, d, b.z, b.v, b.sigma, lo, hi, 5000, 1_000_000)
    assert nv == 0
    # the bound is informative: sampled extremes reach a good part of it
    assert (r.max(1)[:, 3:5] / hi.reshape(-1, 6)[:, 3:5]).mean() > 0.3


def test_sampled_soundness_chain(orc):
    b = _chain_inputs(2, 28, 4)
    d = orc.Dyn.like(b.dyn)
    lo, hi, _ = orc.leb(d, b.z, b.v, b.sigma)
    nv, _ = _violations(orc, d, b.z, b.v, b.sigma, lo, hi, 2000, 1_000_002)
    assert nv == 0


def test_sampled_soundness_off_centre(orc):
    b = W.chain_batch(9, 1, 3, 4)
    d = orc.Dyn.like(b.dyn)
    mu = _rng(3).uniform(-0.06, 0.06, b.sigma.shape)
    lo, hi, _ = orc.leb(d, b.z, b.v, b.sigma, mu=mu)
    nv, _ = _violations(orc, d, b.z, b.v, b.sigma, lo, hi, 3000, 1_000_003, mu=mu)
    assert nv == 0


def test_expand_and_classic_closed_forms(orc):
    """The expanded (eq. expanded_interval_hessian) and classic (eq.
    interval_quadratic_form) enclosures written out by hand for a quadratic
    f = 1/2 a^T Q a with Q = [[a, b], [b, c]] on the symmetric box
    Delta = ([-s, s], [-t, t]):
      path = expand:  [-|b| s t + 1/2 min(a,0) s^2 + 1/2 min(c,0) t^2,
                        |b| s t + 1/2 max(a,0) s^2 + 1/2 max(c,0) t^2]
                      (point Hessian entries, so the prefix sets do not matter)
      classic:        v = [Q] Delta, then 1/2 Delta . v:
                      +-1/2 (|a| s^2 + 2 |b| s t + |c| t^2)
    and for a diagonal Q on one-sided boxes (mu = sigma, Delta = [0, 2 sigma]),
    where Delta x Delta = sq(Delta), all three are 1/2 Q_kk [0, 4 sigma_k^2]."""
    for (a, b, c) in ((2.0, 0.7, -1.5), (-0.3, -1.1, 0.4), (1.0, 0.0, 3.0)):
        Q = np.array([[[a, b], [b, c]]])
        d = orc.Dyn("quadratic", 1, 1, Q=Q)
        s, t = 0.3, 0.05
        z, v, sg = np.array([[0.4]]), np.array([[-0.2]]), np.array([[s, t]])
        hi_p = abs(b) * s * t + 0.5 * max(a, 0) * s * s + 0.5 * max(c, 0) * t * t
        lo_p = -abs(b) * s * t + 0.5 * min(a, 0) * s * s + 0.5 * min(c, 0) * t * t
        hc = 0.5 * (abs(a) * s * s + 2 * abs(b) * s * t + abs(c) * t * t)
        for mode, lo_w, hi_w in (("path", lo_p, hi_p), ("expand", lo_p, hi_p), ("classic", -hc, hc)):
            lo, hi, _ = orc.leb(d, z, v, sg, mode=mode)
            assert lo[0, 0] <= lo_w and hi[0, 0] >= hi_w, mode
            assert abs(lo[0, 0] - lo_w) <= 1e-14 and abs(hi[0, 0] - hi_w) <= 1e-14, (mode, lo, hi, lo_w, hi_w)
    rng = np.random.default_rng(2)
    n = 5
    Q = np.zeros((2, n, n))
    Q[0][np.diag_indices(n)] = rng.normal(size=n)
    Q[1][np.diag_indices(n)] = rng.normal(size=n)
    d = orc.Dyn("quadratic", 2, 3, Q=Q)
    sg = rng.uniform(0.01, 0.2, (4, n))
    z, v = rng.normal(size=(4, 2)), rng.normal(size=(4, 3))
    want_hi = 0.5 * (np.maximum(Q[:, range(n), range(n)], 0)[None] * 4 * sg[:, None, :] ** 2).sum(-1)
    want_lo = 0.5 * (np.minimum(Q[:, range(n), range(n)], 0)[None] * 4 * sg[:, None, :] ** 2).sum(-1)
    for mode in ("path", "expand", "classic"):
        lo, hi, _ = orc.leb(d, z, v, sg, mu=sg, mode=mode)
        np.testing.assert_allclose(hi, want_hi, rtol=1e-13, atol=0)
        np.testing.assert_allclose(lo, want_lo, rtol=1e-13, atol=0)
        assert (hi >= want_hi).all() and (lo <= want_lo).all()
