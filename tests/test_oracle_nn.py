"""Pins of the NN oracle (CROWN + Theorem 2): closed forms, LP relaxations
solved by scipy's HiGHS, activation-pattern enumeration on tiny MLPs,
agreement of the direct and centred forms, and sampled containment."""
import itertools

import numpy as np
import pytest

import workloads as W
from oracle import nn

linprog = pytest.importorskip("scipy.optimize").linprog


def _net(rng, widths, scale=1.0):
    Ws, bs = [], []
    for i, o in zip(widths[:-1], widths[1:]):
        Ws.append(rng.normal(0, scale * np.sqrt(2.0 / i), (o, i)))
        bs.append(rng.uniform(-0.3, 0.3, o))
    return Ws, bs


def test_stable_box_gives_zero():
    """With no unstable neuron the relaxations are exact: W_lo = W_hi = J,
    all gaps 0, so the centred bound is exactly [0, 0]."""
    b = W.nn_cfg()
    a = np.concatenate([b.z, b.v], -1)[0, :5]
    o = nn.leb(b.net.W, b.net.b, a, np.full((5, 16), 1e-9))
    assert o["unstable"] == [0, 0, 0]
    assert (o["c_hi"] == 0).all() and (o["c_lo"] == 0).all()
    assert np.abs(o["r_hi"]).max() < 1e-12 and np.abs(o["r_lo"]).max() < 1e-12


def _triangle_lp(Ws, bs, a0, c, rho, sign):
    """max (sign = +1) or min (sign = -1) of the 1-hidden-layer remainder
    over the box with the triangle relaxation of every unstable neuron."""
    W1, b1 = Ws[0], bs[0]
    w2, b2 = Ws[1][0], bs[1][0]
    n, h = W1.shape[1], W1.shape[0]
    zs = nn.forward([np.asarray(w) for w in Ws], [np.asarray(x) for x in bs], a0)
    J = nn.jacobian(Ws, zs)[0]
    lo = W1 @ c + b1 - np.abs(W1) @ rho
    hi = W1 @ c + b1 + np.abs(W1) @ rho
    # variables [alpha (n), act (h)]; objective sign * (w2 . act - J . alpha)
    cost = -sign * np.concatenate([-J, w2])
    A_ub, b_ub, A_eq, b_eq = [], [], [], []
    bounds = [(c[k] - rho[k], c[k] + rho[k]) for k in range(n)] + [(None, None)] * h
    for j in range(h):
        row = np.zeros(n + h)
        if lo[j] >= 0:                   # a = z
            row[:n] = -W1[j]; row[n + j] = 1.0
            A_eq.append(row); b_eq.append(b1[j])
        elif hi[j] <= 0:                 # a = 0
            row[n + j] = 1.0
            A_eq.append(row); b_eq.append(0.0)
        else:
            s = hi[j] / (hi[j] - lo[j]); t = -s * lo[j]
            r1 = np.zeros(n + h); r1[n + j] = -1.0                               # a >= 0
            A_ub.append(r1); b_ub.append(0.0)
            r2 = np.zeros(n + h); r2[:n] = W1[j]; r2[n + j] = -1.0                # a >= z
            A_ub.append(r2); b_ub.append(-b1[j])
            r3 = np.zeros(n + h); r3[:n] = -s * W1[j]; r3[n + j] = 1.0            # a <= s z + t
            A_ub.append(r3); b_ub.append(s * b1[j] + t)
    res = linprog(cost, A_ub=np.array(A_ub) if A_ub else None, b_ub=b_ub if b_ub else None,
                  A_eq=np.array(A_eq) if A_eq else None, b_eq=b_eq if b_eq else None, bounds=bounds,
                  method="highs")
    assert res.status == 0
    const = J @ a0 - zs[-1][0] + b2
    return sign * (-res.fun) + const


def test_single_neuron_upper_line_equals_lp():
    """One unstable neuron with a positive output weight: CROWN's upper
    bound uses the triangle's upper line, so it equals the LP optimum."""
    rng = np.random.default_rng(3)
    for trial in range(20):
        W1 = rng.normal(size=(1, 2))
        b1 = np.array([0.0])
        w2 = np.array([[abs(rng.normal()) + 0.1]])
        b2 = np.array([rng.normal()])
        a0 = rng.uniform(-0.2, 0.2, 2)
        sg = rng.uniform(0.3, 0.6, 2)
        o = nn.leb([W1, w2], [b1, b2], a0, sg)
        assert o["unstable"] == [1]
        c, rho = nn.box_of(a0, sg)
        lp = _triangle_lp([W1, w2], [b1, b2], a0, c, rho, +1)
        assert abs(o["r_hi"][0] - lp) <= 1e-9 * max(1, abs(lp))


def test_single_hidden_layer_dominates_lp_and_true_range():
    """CROWN is a feasible dual point of the triangle LP: r_hi >= LP max >=
    true max (and symmetrically for the minimum)."""
    rng = np.random.default_rng(4)
    for trial in range(10):
        Ws, bs = _net(rng, [3, 6, 1])
        a0 = rng.uniform(-0.5, 0.5, 3)
        sg = rng.uniform(0.2, 0.5, 3)
        o = nn.leb(Ws, bs, a0, sg)
        c, rho = nn.box_of(a0, sg)
        lp_max = _triangle_lp(Ws, bs, a0, c, rho, +1)
        lp_min = _triangle_lp(Ws, bs, a0, c, rho, -1)
        g = np.array(np.meshgrid(*[np.linspace(c[k] - rho[k], c[k] + rho[k], 25) for k in range(3)])).reshape(3, -1).T
        r, _ = nn.remainder(Ws, bs, a0, g)
        assert o["r_hi"][0] >= lp_max - 1e-9 and lp_max >= r.max() - 1e-9
        assert o["r_lo"][0] <= lp_min + 1e-9 and lp_min <= r.min() + 1e-9


def _exact_range_by_patterns(Ws, bs, a0, c, rho):
    """Exact min/max of the remainder over the box: on each activation
    region g is affine, so each region's extremum is an LP."""
    zs = nn.forward(Ws, bs, a0)
    J = nn.jacobian(Ws, zs)
    g0 = zs[-1]
    hidden = [w.shape[0] for w in Ws[:-1]]
    n = Ws[0].shape[1]
    best_hi = -np.inf * np.ones(Ws[-1].shape[0])
    best_lo = np.inf * np.ones(Ws[-1].shape[0])
    for pattern in itertools.product([0, 1], repeat=sum(hidden)):
        masks, k = [], 0
        for h in hidden:
            masks.append(np.array(pattern[k:k + h], dtype=np.float64))
            k += h
        # affine maps z_l = M_l a + m_l on the region
        M, m = np.eye(n), np.zeros(n)
        A_ub, b_ub = [], []
        for l, (Wl, bl) in enumerate(zip(Ws[:-1], bs[:-1])):
            Mz, mz = Wl @ M, Wl @ m + bl
            for j in range(Wl.shape[0]):
                if masks[l][j]:      # z >= 0
                    A_ub.append(-Mz[j]); b_ub.append(mz[j])
                else:                # z <= 0
                    A_ub.append(Mz[j]); b_ub.append(-mz[j])
            M, m = masks[l][:, None] * Mz, masks[l] * mz
        G, gc = Ws[-1] @ M, Ws[-1] @ m + bs[-1]
        bnd = [(c[q] - rho[q], c[q] + rho[q]) for q in range(n)]
        for o_ in range(G.shape[0]):
            coef = G[o_] - J[o_]
            const = gc[o_] - g0[o_] + J[o_] @ a0
            for sign in (+1, -1):
                res = linprog(-sign * coef, A_ub=np.array(A_ub), b_ub=np.array(b_ub), bounds=bnd, method="highs")
                if res.status == 2:          # infeasible region
                    break
                assert res.status == 0
                val = sign * (-res.fun) + const
                if sign > 0:
                    best_hi[o_] = max(best_hi[o_], val)
                else:
                    best_lo[o_] = min(best_lo[o_], val)
    return best_lo, best_hi


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_tiny_mlp_pattern_enumeration(seed):
    rng = np.random.default_rng(seed)
    Ws, bs = _net(rng, [2, 3, 3, 2])
    a0 = rng.uniform(-0.4, 0.4, 2)
    sg = rng.uniform(0.3, 0.7, 2)
    o = nn.leb(Ws, bs, a0, sg)
    c, rho = nn.box_of(a0, sg)
    elo, ehi = _exact_range_by_patterns(Ws, bs, a0, c, rho)
    assert (elo >= o["r_lo"] - 1e-9).all() and (ehi <= o["r_hi"] + 1e-9).all()
    assert sum(o["unstable"]) > 0


def test_direct_and_centred_forms_agree_and_contain_zero():
    b = W.nn_cfg()
    a = np.concatenate([b.z, b.v], -1)[:2, :8]
    o = nn.leb(b.net.W, b.net.b, a, b.sigma[:2, :8])
    M = np.maximum(np.abs(o["c_hi"]), np.abs(o["c_lo"]))
    assert (np.abs(o["r_hi"] - o["c_hi"]) <= 1e-12 * M + 1e-15).all()
    assert (np.abs(o["r_lo"] - o["c_lo"]) <= 1e-12 * M + 1e-15).all()
    assert (o["r_lo"] <= 0).all() and (o["r_hi"] >= 0).all()
    assert (o["kappa_hi"] >= 0).all() and (o["kappa_lo"] <= 0).all()


def test_sampled_containment_nn():
    b = W.nn_cfg()
    a = np.concatenate([b.z, b.v], -1)[:4, :10].reshape(-1, 16)
    sg = b.sigma[:4, :10].reshape(-1, 16)
    mu = np.random.default_rng(2).uniform(-0.01, 0.01, sg.shape)
    o = nn.leb(b.net.W, b.net.b, a, sg, mu=mu)
    c, rho = nn.box_of(a, sg, mu)
    pts = W.sample_box_points(W.rng_for(1_000_001), c - rho, c + rho, 3000)
    r, eps = nn.remainder(b.net.W, b.net.b, a, pts)
    assert ((r > o["r_hi"][:, None] + eps) | (r < o["r_lo"][:, None] - eps)).sum() == 0


def test_given_jacobian_equals_computed_and_encloses_its_remainder():
    """Theorem 2 holds for any J.  Passing the network's own Jacobian gives
    the default bound; a perturbed J gives a bound that contains 0 and every
    sampled remainder g(a) - g(a~) - J (a - a~), and whose centred form
    (independent of J's choice of split) agrees with the direct form."""
    rng = np.random.default_rng(11)
    Ws, bs = _net(rng, [6, 16, 16, 3])
    a0 = rng.uniform(-1, 1, (4, 6))
    sg = rng.uniform(0.05, 0.2, (4, 6))
    o = nn.leb(Ws, bs, a0, sg)
    o2 = nn.leb(Ws, bs, a0, sg, J=o["J"])
    assert np.array_equal(o["r_lo"], o2["r_lo"]) and np.array_equal(o["r_hi"], o2["r_hi"])
    Jp = o["J"] + rng.normal(0, 0.3, o["J"].shape)
    oj = nn.leb(Ws, bs, a0, sg, J=Jp)
    assert (oj["r_lo"] <= 0).all() and (oj["r_hi"] >= 0).all()
    M = np.maximum(np.abs(oj["r_hi"]), np.abs(oj["r_lo"]))
    assert np.allclose(oj["c_hi"], oj["r_hi"], rtol=0, atol=1e-12 * M.max())
    assert np.allclose(oj["c_lo"], oj["r_lo"], rtol=0, atol=1e-12 * M.max())
    lo, hi = a0 - sg, a0 + sg
    pts = W.sample_box_points(rng, lo, hi, 4000)
    r, eps = nn.remainder(Ws, bs, a0, pts, J=Jp)
    assert (r <= oj["r_hi"][:, None, :] + eps).all() and (r >= oj["r_lo"][:, None, :] - eps).all()
    # the perturbed J's bound is wider: the linear part it misses is J_true - J
    assert (oj["r_hi"] - oj["r_lo"] > o["r_hi"] - o["r_lo"]).all()


def test_given_jacobian_stable_box_closed_form():
    """On a box with no unstable neuron g is affine with slope J*, so the
    remainder with any J is (J* - J)(a - a~) exactly, whose range over the
    symmetric box is +-|J* - J| rho: Theorem 2 must give exactly that."""
    b = W.nn_cfg()
    a = np.concatenate([b.z, b.v], -1)[0, :3]
    sg = np.full((3, 16), 1e-7)
    o = nn.leb(b.net.W, b.net.b, a, sg)
    assert o["unstable"] == [0, 0, 0]
    rng = np.random.default_rng(3)
    Jp = o["J"] + rng.normal(0, 0.1, o["J"].shape)
    oj = nn.leb(b.net.W, b.net.b, a, sg, J=Jp)
    exp = np.einsum("bmn,n->bm", np.abs(o["J"] - Jp), np.full(16, 1e-7))
    assert np.allclose(oj["r_hi"], exp, rtol=1e-9, atol=1e-15)
    assert np.allclose(oj["r_lo"], -exp, rtol=1e-9, atol=1e-15)
