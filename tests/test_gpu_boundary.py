"""GPU parity of the boundary's smaller entry points against the oracle:
the closed-form dynamics kinds of leb_analytic_bound (linear with invalid
data, quadratic against its closed form, 1-D and 2-D sin/cos), the point
Jacobians (eq. linearizations), the zonotope hull (eq. tight_tube_width), the
caller-given J of leb_nn_bound (Theorem 2 with any J), and the device-side
ordering of calls that share a library workspace from two streams."""
import numpy as np
import pytest

import workloads as W
from parity import check_bounds

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2607_01203_amd as leb
    leb.lib()
    return torch.device("cuda:0")


def _t(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _bound(leb, dyn, z, v, s, dev, mu=None):
    import torch
    out = leb.analytic_bound(dyn, _t(z, dev), _t(v, dev), _t(s, dev), None if mu is None else _t(mu, dev),
                             zonotope=True)
    torch.cuda.synchronize()
    return {k: x.cpu().numpy() for k, x in out.items()}


def test_linear_kind_validates_data(gpu, orc):
    """Linear dynamics: [0, 0] for valid data; a non-finite nominal, mu or
    sigma, or a negative sigma, gives [-inf, inf] with BAD_INPUT on every row
    of that unit only; |mu| > sigma sets HULL_EXTENDED; flags as the oracle's."""
    import paper_2607_01203_amd as leb
    rng = np.random.default_rng(21)
    U, nx, nu = 40, 5, 2
    z = rng.normal(size=(U, nx))
    v = rng.normal(size=(U, nu))
    s = rng.uniform(0, 1, (U, nx + nu))
    mu = rng.uniform(-0.5, 0.5, (U, nx + nu)) * s
    z[3, 1] = np.nan
    v[7, 0] = np.inf
    s[11, 4] = -1e-3
    mu[15, 2] = np.nan
    s[19, 6] = np.inf
    mu[23, 0] = 2.0 * s[23, 0] + 0.1       # outside: hull
    print("case: linear kind, 40 units with invalid rows", flush=True)
    g = _bound(leb, leb.linear_dynamics(nx, nu), z[:, None], v[:, None], s[:, None], gpu, mu=mu[:, None])
    lo, hi, fl = orc.leb(orc.Dyn("linear", nx, nu), z, v, s, mu=mu)
    check_bounds(g["r_lo"][:, 0], g["r_hi"][:, 0], lo, hi, "linear")
    assert np.array_equal(g["flags"][:, 0], fl.astype(np.int32))
    bad = [3, 7, 11, 15, 19]
    assert (g["flags"][bad, 0] & leb.FLAG_BAD_INPUT).all()
    assert np.isinf(g["r_hi"][bad]).all() and np.isinf(g["r_lo"][bad]).all()
    ok = np.setdiff1d(np.arange(U), bad)
    assert (g["r_lo"][ok] == 0).all() and (g["r_hi"][ok] == 0).all()
    assert g["flags"][23, 0] & leb.FLAG_HULL_EXTENDED
    assert np.isinf(g["rho_bar"][bad]).all() and (g["rho_bar"][ok] == 0).all()


def _quad_Q(rng, nx, n):
    Q = rng.normal(size=(nx, n, n))
    return 0.5 * (Q + np.transpose(Q, (0, 2, 1)))


@pytest.mark.parametrize("nx,nu,units", [(3, 1, 70), (8, 4, 33), (48, 16, 9)])
def test_quadratic_kind_closed_form(gpu, orc, nx, nu, units):
    """Quadratic dynamics on symmetric boxes: the path-based bound equals
    hi_l = sum_{j<k} |Q_kj| rho_j rho_k + 1/2 sum_k max(Q_kk, 0) rho_k^2 and
    lo_l = -sum_{j<k} |Q_kj| rho_j rho_k + 1/2 sum_k min(Q_kk, 0) rho_k^2; the
    GPU contains it, lies within 1e-4 of it and matches the oracle.  n = 64 is
    the largest supported size; zero radii give exactly [0, 0]."""
    import torch
    import paper_2607_01203_amd as leb
    rng = np.random.default_rng(100 + nx)
    n = nx + nu
    Q = _quad_Q(rng, nx, n)
    Q[0, :, :] = 0.0                          # a row without curvature: exactly 0
    z = rng.uniform(-1, 1, (units, nx))
    v = rng.uniform(-1, 1, (units, nu))
    s = rng.uniform(0.0, 0.3, (units, n))
    s[2] = 0.0                                # a unit with a point box
    print("case: quadratic n=%d units=%d" % (n, units), flush=True)
    dyn = leb.quadratic_dynamics(_t(Q, gpu), nu=nu)
    g = _bound(leb, dyn, z[:, None], v[:, None], s[:, None], gpu)
    lo_o, hi_o, _ = orc.leb(orc.Dyn("quadratic", nx, nu, Q=Q), z, v, s)
    check_bounds(g["r_lo"][:, 0], g["r_hi"][:, 0], lo_o, hi_o, "quadratic")
    off = np.tril(np.abs(Q), -1)              # |Q_kj|, j < k
    dg = np.einsum("lkk->lk", Q)
    cross = np.einsum("lkj,uk,uj->ul", off, s, s)
    hi_c = cross + 0.5 * np.einsum("lk,uk->ul", np.maximum(dg, 0), s * s)
    lo_c = -cross + 0.5 * np.einsum("lk,uk->ul", np.minimum(dg, 0), s * s)
    check_bounds(g["r_lo"][:, 0], g["r_hi"][:, 0], lo_c, hi_c, "quadratic closed form")
    assert (g["r_hi"][:, 0] >= hi_c).all() and (g["r_lo"][:, 0] <= lo_c).all()
    assert (g["r_lo"][:, 0, 0] == 0).all() and (g["r_hi"][:, 0, 0] == 0).all()
    assert (g["r_lo"][2] == 0).all() and (g["r_hi"][2] == 0).all()
    del torch


def test_quadratic_kind_nonfinite_coefficient(gpu, orc):
    """A non-finite Q_l entry makes row l [-inf, inf] with UNBOUNDED; the
    other rows are unaffected."""
    import paper_2607_01203_amd as leb
    rng = np.random.default_rng(7)
    Q = _quad_Q(rng, 3, 4)
    Q[1, 2, 0] = np.nan
    z = rng.uniform(-1, 1, (5, 3))
    v = rng.uniform(-1, 1, (5, 1))
    s = rng.uniform(0.01, 0.2, (5, 4))
    g = _bound(leb, leb.quadratic_dynamics(_t(Q, gpu), nu=1), z[:, None], v[:, None], s[:, None], gpu)
    assert np.isinf(g["r_lo"][:, 0, 1]).all() and np.isinf(g["r_hi"][:, 0, 1]).all()
    assert (g["flags"][:, 0] & leb.FLAG_UNBOUNDED).all()
    Q2 = Q.copy()
    Q2[1] = 0.0
    lo_o, hi_o, _ = orc.leb(orc.Dyn("quadratic", 3, 1, Q=Q2), z, v, s)
    check_bounds(g["r_lo"][:, 0, [0, 2]], g["r_hi"][:, 0, [0, 2]], lo_o[:, [0, 2]], hi_o[:, [0, 2]], "other rows")


@pytest.mark.parametrize("wide", [False, True])
def test_sin1d_kind(gpu, orc, wide):
    """f = sin(a): the bound is 1/2 (-sin X) x [0, rho^2] on a symmetric box
    (closed form) and matches the oracle; wide boxes take the FP64 sin/cos
    path (|X| beyond the polynomial range) and may contain extrema."""
    import paper_2607_01203_amd as leb
    rng = np.random.default_rng(31 + wide)
    U = 400
    z = rng.uniform(-3.5, 3.5, (U, 1)) if wide else rng.uniform(-0.6, 0.6, (U, 1))
    s = rng.uniform(0.0, 1.5, (U, 1)) if wide else rng.uniform(0.0, 0.15, (U, 1))
    v = np.zeros((U, 0))
    print("case: sin1d wide=%d" % wide, flush=True)
    g = _bound(leb, leb.sincos_dynamics(1), z[:, None], v[:, None], s[:, None], gpu)
    lo_o, hi_o, _ = orc.leb(orc.Dyn("sin1d", 1, 0), z, v, s)
    check_bounds(g["r_lo"][:, 0], g["r_hi"][:, 0], lo_o, hi_o, "sin1d")
    X = np.stack([z[:, 0] - s[:, 0], z[:, 0] + s[:, 0]], 1)
    grid = np.linspace(0, 1, 2001)[None, :] * (X[:, 1:] - X[:, :1]) + X[:, :1]
    ms = -np.sin(grid)
    hmin, hmax = ms.min(1), ms.max(1)
    r2 = s[:, 0] ** 2
    # closed form on the grid: range of 1/2 h t over h in -sin X, t in [0, rho^2]
    hi_c = 0.5 * np.maximum(hmax, 0) * r2
    lo_c = 0.5 * np.minimum(hmin, 0) * r2
    M = np.maximum(np.abs(hi_c), np.abs(lo_c)) + 1e-300
    assert (g["r_hi"][:, 0, 0] >= hi_c - 1e-6 * M).all() and (g["r_lo"][:, 0, 0] <= lo_c + 1e-6 * M).all()


def test_sincos2d_kind(gpu, orc):
    """f = (sin a1 cos a2, cos a1 sin a2): parity with the oracle over
    symmetric and off-centre boxes, narrow (polynomial path) and wide; the
    bound contains the grid range of the true remainder."""
    import paper_2607_01203_amd as leb
    rng = np.random.default_rng(41)
    U = 300
    z = rng.uniform(-2.0, 2.0, (U, 2))
    z[: U // 2] *= 0.3
    s = rng.uniform(0.0, 0.4, (U, 2))
    mu = rng.uniform(-1.2, 1.2, (U, 2)) * s
    v = np.zeros((U, 0))
    print("case: sincos2d", flush=True)
    g = _bound(leb, leb.sincos_dynamics(2), z[:, None], v[:, None], s[:, None], gpu, mu=mu[:, None])
    d = orc.Dyn("sincos2d", 2, 0)
    lo_o, hi_o, fl = orc.leb(d, z, v, s, mu=mu)
    check_bounds(g["r_lo"][:, 0], g["r_hi"][:, 0], lo_o, hi_o, "sincos2d")
    assert np.array_equal(g["flags"][:, 0], fl.astype(np.int32))
    # containment of the true remainder on a 41 x 41 grid of each box
    blo, bhi = orc.box(z, s, mu)
    t = np.linspace(0, 1, 41)
    P = np.stack(np.meshgrid(t, t, indexing="ij"), -1).reshape(-1, 2)
    pts = blo[:, None, :] + P[None] * (bhi - blo)[:, None, :]
    unit_of = np.repeat(np.arange(U), P.shape[0])
    r, eps = orc.remainder(d, z, pts.reshape(-1, 2), unit_of)
    r = r.reshape(U, -1, 2)
    eps = eps.reshape(U, -1, 2)
    assert (r <= g["r_hi"][:, 0][:, None, :] + eps).all() and (r >= g["r_lo"][:, 0][:, None, :] - eps).all()


@pytest.mark.parametrize("n_units,batch,N", [(1, 2, 20), (4, 3, 7), (28, 1, 5)])
def test_chain_jacobians(gpu, orc, n_units, batch, N):
    """A = df/dx and B = df/du at the nominal (eq. linearizations) from the
    optional outputs of leb_analytic_bound, against the oracle's Jacobians;
    the bound outputs are those of a call without them."""
    import torch
    import paper_2607_01203_amd as leb
    b = W.chain_batch(300 + n_units, batch, N, n_units)
    dyn = leb.dynamics_like(b.dyn)
    print("case: jacobians U=%d B=%d N=%d" % (n_units, batch, N), flush=True)
    out = leb.analytic_bound(dyn, _t(b.z, gpu), _t(b.v, gpu), _t(b.sigma, gpu), jacobians=True)
    ref = leb.analytic_bound(dyn, _t(b.z, gpu), _t(b.v, gpu), _t(b.sigma, gpu))
    torch.cuda.synchronize()
    A_o, B_o = orc.jacobian(orc.Dyn.like(b.dyn), b.z, b.v)
    A_g, B_g = out["A"].cpu().numpy(), out["B"].cpu().numpy()
    sa = np.abs(A_o).max()
    assert np.abs(A_g - A_o).max() <= 1e-13 * sa
    assert np.abs(B_g - B_o).max() <= 1e-13 * np.abs(B_o).max()
    assert torch.equal(out["r_lo"], ref["r_lo"]) and torch.equal(out["r_hi"], ref["r_hi"])


def test_zonotope_hull(gpu):
    """sigma = sum_j |G_ij| rounded upward (never below the exact sum, within
    1e-12 of it), mu = c; rows of zeros, a non-finite entry (+inf), no
    generators, and a long row of 20,000 generators."""
    import torch
    import paper_2607_01203_amd as leb
    from oracle import tube
    rng = np.random.default_rng(9)
    for rows, ng in [(1000, 37), (5, 20000), (64, 1), (3, 0)]:
        G = rng.normal(size=(rows, ng)) * np.exp(rng.uniform(-20, 20, (rows, 1)))
        c = rng.normal(size=rows)
        if rows > 10:
            G[7] = 0.0
            G[9, 0] = np.inf
        print("case: hull rows=%d n_gen=%d" % (rows, ng), flush=True)
        mu, sg = leb.zonotope_hull(_t(G, gpu), _t(c, gpu))
        torch.cuda.synchronize()
        mu, sg = mu.cpu().numpy(), sg.cpu().numpy()
        mo, so = tube.zonotope_hull(G, c)
        assert np.array_equal(mu, mo)
        fin = np.isfinite(so)
        assert np.array_equal(sg[~fin], so[~fin])
        assert (sg[fin] >= so[fin]).all() and (sg[fin] <= so[fin] * (1 + 1e-12)).all()
        if rows > 10:
            assert sg[7] == 0.0 and sg[9] == np.inf
    mu, sg = leb.zonotope_hull(_t(np.ones((4, 3)), gpu))
    torch.cuda.synchronize()
    assert (mu.cpu().numpy() == 0).all() and (sg.cpu().numpy() >= 3.0).all()


def test_nn_bound_given_jacobian(gpu):
    """leb_nn_bound with the caller's J: with the network's own Jacobian it
    matches the computed-J bound; with a perturbed J it matches the oracle's
    Theorem 2 bound for that J and contains sampled remainders; a non-finite
    entry of one unit's J makes only that unit [-inf, inf] with BAD_INPUT."""
    import torch
    import paper_2607_01203_amd as leb
    from oracle import nn as onn
    b = W.nn_cfg(seed=1, batch=2, N=9)
    net = leb.MLP(b.net.W, b.net.b, nx=b.z.shape[-1])
    a = np.concatenate([b.z, b.v], -1)
    o = onn.leb(b.net.W, b.net.b, a, b.sigma)
    rng = np.random.default_rng(5)
    Jp = o["J"] + rng.normal(0, 0.05, o["J"].shape)
    print("case: nn bound with given J", flush=True)
    zt, vt, st = _t(b.z, gpu), _t(b.v, gpu), _t(b.sigma, gpu)
    g0 = leb.nn_bound(net, zt, vt, st)
    g1 = leb.nn_bound(net, zt, vt, st, J=_t(o["J"], gpu))
    g2 = leb.nn_bound(net, zt, vt, st, J=_t(Jp, gpu))
    Jbad = Jp.copy()
    Jbad[1, 3, 2, 5] = np.nan
    g3 = leb.nn_bound(net, zt, vt, st, J=_t(Jbad, gpu))
    torch.cuda.synchronize()
    c = lambda d: {k: x.cpu().numpy() for k, x in d.items()}
    g0, g1, g2, g3 = c(g0), c(g1), c(g2), c(g3)
    check_bounds(g1["r_lo"], g1["r_hi"], g0["r_lo"], g0["r_hi"], "own J")
    oj = onn.leb(b.net.W, b.net.b, a, b.sigma, J=Jp)
    check_bounds(g2["r_lo"], g2["r_hi"], oj["r_lo"], oj["r_hi"], "perturbed J")
    lo, hi = a - b.sigma, a + b.sigma
    pts = W.sample_box_points(rng, lo.reshape(-1, 16), hi.reshape(-1, 16), 2000)
    r, eps = onn.remainder(b.net.W, b.net.b, a.reshape(-1, 16), pts, J=Jp.reshape(-1, 12, 16))
    assert (r <= g2["r_hi"].reshape(-1, 1, 12) + eps).all() and (r >= g2["r_lo"].reshape(-1, 1, 12) - eps).all()
    assert g3["flags"][1, 3] & leb.FLAG_BAD_INPUT and np.isinf(g3["r_hi"][1, 3]).all()
    keep = np.ones((2, 9), bool)
    keep[1, 3] = False
    assert np.array_equal(g3["r_hi"][keep], g2["r_hi"][keep]) and np.array_equal(g3["r_lo"][keep], g2["r_lo"][keep])
    net.close()


def test_workspace_calls_on_two_streams(gpu):
    """Calls that share a library-owned workspace, enqueued back to back on
    two streams, give the results of the same calls run one at a time (the
    second call's kernels wait for the first's on the device)."""
    import torch
    import paper_2607_01203_amd as leb
    tp1 = W.fixed_point_cfg(seed=61, batch=64, N=24, n_units=8)
    tp2 = W.fixed_point_cfg(seed=62, batch=32, N=30, n_units=8)
    dyn = leb.dynamics_like(tp1.batch.dyn)
    args = [(_t(tp.batch.z, gpu), _t(tp.batch.v, gpu), _t(tp.phi, gpu), tp.e) for tp in (tp1, tp2)]
    torch.cuda.synchronize()
    ref = [leb.fixed_point_solve(dyn, *a) for a in args]
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    print("case: fixed point on two streams", flush=True)
    out = []
    for _ in range(2):
        with torch.cuda.stream(s1):
            r1 = leb.fixed_point_solve(dyn, *args[0], stream=s1)
        with torch.cuda.stream(s2):
            r2 = leb.fixed_point_solve(dyn, *args[1], stream=s2)
        out.append((r1, r2))
    torch.cuda.synchronize()
    for r1, r2 in out:
        for r, q in ((r1, ref[0]), (r2, ref[1])):
            assert torch.equal(r[0], q[0]) and torch.equal(r[1], q[1]) and torch.equal(r[2], q[2]) and r[3] == q[3]
    # the MLP bound's workspace
    b1 = W.nn_cfg(seed=1, batch=8, N=50)
    b2 = W.nn_cfg(seed=1, batch=4, N=20)
    net = leb.MLP(b1.net.W, b1.net.b, nx=b1.z.shape[-1])
    t1 = [_t(x, gpu) for x in (b1.z, b1.v, b1.sigma)]
    t2 = [_t(x, gpu) for x in (b2.z, b2.v, b2.sigma)]
    torch.cuda.synchronize()
    q1, q2 = leb.nn_bound(net, *t1), leb.nn_bound(net, *t2)
    torch.cuda.synchronize()
    print("case: MLP bound on two streams", flush=True)
    with torch.cuda.stream(s1):
        p1 = leb.nn_bound(net, *t1, stream=s1)
    with torch.cuda.stream(s2):
        p2 = leb.nn_bound(net, *t2, stream=s2)
    torch.cuda.synchronize()
    for p, q in ((p1, q1), (p2, q2)):
        assert torch.equal(p["r_lo"], q["r_lo"]) and torch.equal(p["r_hi"], q["r_hi"])
    net.close()
