"""Pins of the NN-bound gradient oracle (forward-mode derivative of the CROWN
+ Theorem 2 bound): central finite differences of the bound oracle, a
one-neuron network done by hand, the mu/alpha identity inside the clamps,
and values equal to the bound oracle's."""
import numpy as np
import pytest

from oracle import nn, nn_grad


def _net(rng, widths, scale=1.0):
    Ws, bs = [], []
    for i, o in zip(widths[:-1], widths[1:]):
        Ws.append(rng.normal(0, scale * np.sqrt(2.0 / i), (o, i)))
        bs.append(rng.uniform(-0.3, 0.3, o))
    return Ws, bs


def _bound(Ws, bs, a, s, m):
    o = nn.leb(Ws, bs, a, s, m, centred=False)
    return o["r_lo"], o["r_hi"]


@pytest.mark.parametrize("widths,seed", [([4, 8, 3], 1), ([4, 8, 8, 3], 2), ([6, 16, 16, 16, 4], 3),
                                         ([5, 12, 10, 8, 6, 2], 4)])
def test_values_equal_bound_oracle(widths, seed):
    rng = np.random.default_rng(seed)
    Ws, bs = _net(rng, widths)
    n0 = widths[0]
    for _ in range(4):
        a = rng.normal(0, 1, n0)
        s = rng.uniform(0.05, 0.5, n0)
        m = rng.uniform(-0.3, 0.3, n0)
        lo, hi, _, _ = nn_grad.leb_jvp(Ws, bs, a, s, m, np.zeros(n0), np.zeros(n0), np.zeros(n0))
        lo_o, hi_o = _bound(Ws, bs, a, s, m)
        np.testing.assert_allclose(lo, lo_o, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(hi, hi_o, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("widths,seed", [([4, 8, 3], 11), ([4, 8, 8, 3], 12), ([6, 16, 16, 16, 4], 13),
                                         ([5, 12, 10, 8, 6, 2], 14)])
def test_directional_derivative_matches_central_differences(widths, seed):
    """Random points and directions (in a~, sigma and mu together); a point
    is used when two step sizes give the same difference quotient (no kink
    within the step), and most points must be usable."""
    rng = np.random.default_rng(seed)
    Ws, bs = _net(rng, widths)
    n0 = widths[0]
    used = 0
    unstable_seen = 0
    for _ in range(24):
        a = rng.normal(0, 1, n0)
        s = rng.uniform(0.05, 0.5, n0)
        m = rng.uniform(-0.6, 0.6, n0)
        da, ds, dm = rng.normal(0, 1, n0), rng.normal(0, 1, n0), rng.normal(0, 1, n0)
        _, _, dlo, dhi = nn_grad.leb_jvp(Ws, bs, a, s, m, da, ds, dm)
        unstable_seen += sum(nn.leb(Ws, bs, a, s, m, centred=False)["unstable"])

        def fd(h):
            lp, hp = _bound(Ws, bs, a + h * da, s + h * ds, m + h * dm)
            lm, hm = _bound(Ws, bs, a - h * da, s - h * ds, m - h * dm)
            return (lp - lm) / (2 * h), (hp - hm) / (2 * h)

        l1, h1 = fd(1e-6)
        l2, h2 = fd(5e-7)
        scale = 1.0 + np.abs(dlo).max() + np.abs(dhi).max()
        if max(np.abs(l1 - l2).max(), np.abs(h1 - h2).max()) > 1e-6 * scale:
            continue                      # a kink within the step
        used += 1
        assert np.abs(dlo - l2).max() <= 2e-6 * scale
        assert np.abs(dhi - h2).max() <= 2e-6 * scale
    assert used >= 16
    assert unstable_seen > 0


def test_gradient_matches_coordinate_differences():
    """leb_grad (one derivative per coordinate) against coordinate-wise
    central differences of L = g_lo . r_lo + g_hi . r_hi."""
    rng = np.random.default_rng(21)
    Ws, bs = _net(rng, [4, 10, 10, 3])
    a = rng.normal(0, 1, 4)
    s = rng.uniform(0.1, 0.4, 4)
    m = rng.uniform(-0.5, 0.5, 4)
    g_lo, g_hi = rng.normal(0, 1, 3), rng.normal(0, 1, 3)
    ga, gs, gm = nn_grad.leb_grad(Ws, bs, a, s, m, g_lo, g_hi)

    def L(a_, s_, m_):
        lo, hi = _bound(Ws, bs, a_, s_, m_)
        return g_lo @ lo + g_hi @ hi

    h = 1e-6
    for i in range(4):
        e = np.zeros(4)
        e[i] = h
        for got, args in ((ga, lambda x: (a + x, s, m)), (gs, lambda x: (a, s + x, m)), (gm, lambda x: (a, s, m + x))):
            ref = (L(*args(e)) - L(*args(-e))) / (2 * h)
            assert abs(got[i] - ref) <= 1e-5 * (1 + abs(ref))


def test_one_neuron_by_hand():
    """g(a) = w2 relu(w1 a + b1) + b2 with w2 > 0, scalar a, mu = 0 and an
    unstable neuron.  With z = w1 a + b1, w = |w1|: the upper line has
    s = 1/2 + z / (2 w sigma), t = w sigma / 2 - z^2 / (2 w sigma); the upper
    pass gives Lambda = w2 s w1, beta = w2 (t + s b1) + b2 (the line
    s (w1 a + b1) + t in a), and Theorem 2
    r_hi = Lambda a + |Lambda - J| sigma - g(a) + beta (J = w2 w1 [z > 0]).
    The lower pass takes the line a z with slope [z >= 0] = [z > 0] here,
    so Lambda_lo = J and r_lo = -w2 b1 [z > 0], constant."""
    w1, b1, w2, b2 = -1.3, 0.2, 0.7, 0.05
    Ws = [np.array([[w1]]), np.array([[w2]])]
    bs = [np.array([b1]), np.array([b2])]
    for a, sg in ((0.1, 0.5), (-0.3, 0.6), (0.4, 0.45)):
        z = w1 * a + b1
        w = abs(w1)
        assert abs(z) < w * sg                      # unstable
        s = 0.5 + z / (2 * w * sg)
        J = w2 * w1 * (z > 0)
        Lam = w2 * s * w1
        ds_dsg = -z / (2 * w * sg ** 2)
        dt_dsg = w / 2 + z ** 2 / (2 * w * sg ** 2)
        ds_da = w1 / (2 * w * sg)
        dt_da = -z * w1 / (w * sg)
        sgn = np.sign(Lam - J)
        dhi_dsg = (w2 * w1 * ds_dsg * a + sgn * w2 * w1 * ds_dsg * sg + abs(Lam - J) + w2 * dt_dsg
                   + w2 * b1 * ds_dsg)
        dhi_da = Lam + w2 * w1 * ds_da * a + sgn * w2 * w1 * ds_da * sg - J + w2 * dt_da + w2 * b1 * ds_da
        ga, gs, gm = nn_grad.leb_grad(Ws, bs, np.array([a]), np.array([sg]), None, np.array([0.0]), np.array([1.0]))
        assert abs(gs[0] - dhi_dsg) <= 1e-13 * (1 + abs(dhi_dsg))
        assert abs(ga[0] - dhi_da) <= 1e-13 * (1 + abs(dhi_da))
        assert gm[0] == 0.0
        ga, gs, _ = nn_grad.leb_grad(Ws, bs, np.array([a]), np.array([sg]), None, np.array([1.0]), np.array([0.0]))
        assert abs(ga[0]) <= 1e-15 and abs(gs[0]) <= 1e-15


def test_mu_acts_like_alpha_inside_the_clamps():
    """With |mu| < sigma the box is (a~ + mu) +/- sigma, and a~ enters the
    bound elsewhere only through J a~ - g(a~) (derivative 0): d/dmu = d/da~."""
    rng = np.random.default_rng(31)
    Ws, bs = _net(rng, [6, 16, 16, 4])
    a = rng.normal(0, 1, 6)
    s = rng.uniform(0.2, 0.5, 6)
    m = s * rng.uniform(-0.9, 0.9, 6)
    g_lo, g_hi = rng.normal(0, 1, 4), rng.normal(0, 1, 4)
    ga, gs, gm = nn_grad.leb_grad(Ws, bs, a, s, m, g_lo, g_hi)
    np.testing.assert_allclose(gm, ga, rtol=1e-12, atol=1e-13)
    assert np.abs(ga).max() > 0


def test_stable_box_has_zero_gradient():
    """A box so small that no neuron is unstable: the bound is [0, 0] up to
    rounding and does not move with a~ or sigma."""
    rng = np.random.default_rng(41)
    Ws, bs = _net(rng, [6, 16, 16, 4])
    a = rng.normal(0, 1, 6)
    s = np.full(6, 1e-9)
    assert sum(nn.leb(Ws, bs, a, s, centred=False)["unstable"]) == 0
    ga, gs, gm = nn_grad.leb_grad(Ws, bs, a, s, None, np.ones(4), np.ones(4))
    assert np.abs(ga).max() < 1e-12 and np.abs(gs).max() < 1e-12 and not gm.any()


def _fd_gap(Ws, bs, rng, n0, trials=6):
    """Largest |forward-mode - central difference| over a few kink-free points."""
    worst = 0.0
    for _ in range(trials):
        a = rng.normal(0, 1, n0)
        s = rng.uniform(0.1, 0.5, n0)
        m = rng.uniform(-0.3, 0.3, n0)
        da, ds, dm = rng.normal(0, 1, n0), rng.normal(0, 1, n0), rng.normal(0, 1, n0)
        _, _, dlo, dhi = nn_grad.leb_jvp(Ws, bs, a, s, m, da, ds, dm)
        h = 5e-7
        lp, hp = _bound(Ws, bs, a + h * da, s + h * ds, m + h * dm)
        lm, hm = _bound(Ws, bs, a - h * da, s - h * ds, m - h * dm)
        worst = max(worst, np.abs(dlo - (lp - lm) / (2 * h)).max(), np.abs(dhi - (hp - hm) / (2 * h)).max())
    return worst


@pytest.mark.parametrize("mistake", ["dt dropped", "ds sign", "drho dropped", "dc dropped"])
def test_pins_catch_planted_mistakes(monkeypatch, mistake):
    """A plausible slip in the tangent code (planted here, in the oracle, on
    the CPU) moves the derivative far outside the finite-difference pin."""
    rng_net = np.random.default_rng(51)
    Ws, bs = _net(rng_net, [6, 16, 16, 16, 4])
    assert _fd_gap(Ws, bs, np.random.default_rng(52), 6) < 1e-5
    relax, conc = nn_grad._relax_t, nn_grad._conc_t
    if mistake == "dt dropped":
        monkeypatch.setattr(nn_grad, "_relax_t", lambda *a: (relax(*a)[0], (relax(*a)[1][0], 0 * relax(*a)[1][1])))
    elif mistake == "ds sign":
        monkeypatch.setattr(nn_grad, "_relax_t", lambda *a: (relax(*a)[0], (-relax(*a)[1][0], relax(*a)[1][1])))
    elif mistake == "drho dropped":
        monkeypatch.setattr(nn_grad, "_conc_t",
                            lambda L, dL, b, db, c, dc, r, dr, up: conc(L, dL, b, db, c, dc, r, 0 * dr, up))
    else:
        monkeypatch.setattr(nn_grad, "_conc_t",
                            lambda L, dL, b, db, c, dc, r, dr, up: conc(L, dL, b, db, c, 0 * dc, r, dr, up))
    assert _fd_gap(Ws, bs, np.random.default_rng(52), 6) > 1e-3
