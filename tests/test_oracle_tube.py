"""Pins of the oracle tube map and tube/LEB fixed point (eqs.
tight_tube_center, tight_tube_width; causality of the tube recursion;
containment certificate mirroring the Theorem 3 induction)."""
import numpy as np
import pytest

import workloads as W


@pytest.fixture(scope="module")
def small():
    return W.fixed_point_cfg(seed=41, batch=3, N=9, n_units=4)


def _dense_phi(tp, k, j, U):
    """Dense Phi_{k,j} ([n] x [nx]) from the per-node block, for lag k-j."""
    n, nx = 8 * U, 6 * U
    P = np.zeros((n, nx))
    blk = tp.phi[k - j - 1]
    for i in range(U):
        P[6 * i:6 * i + 6, 6 * i:6 * i + 6] = blk[:6]
        P[nx + 2 * i:nx + 2 * i + 2, 6 * i:6 * i + 6] = blk[6:]
    return P


def test_phi_satisfies_response_recursion(small):
    """Phi^x_{j+1,j} = I and Phi^x_{k+1,j} = A Phi^x_{k,j} + B Phi^u_{k,j}
    (SLS closed-loop propagation) with Phi^u = K Phi^x."""
    tp = small
    dyn = tp.batch.dyn
    A, Bm, K = W.hover_lqr(dyn)
    np.testing.assert_allclose(tp.phi[0, :6], np.eye(6), atol=0)
    for d in range(1, tp.phi.shape[0]):
        np.testing.assert_allclose(tp.phi[d, :6], A @ tp.phi[d - 1, :6] + Bm @ tp.phi[d - 1, 6:], atol=1e-12)
        np.testing.assert_allclose(tp.phi[d, 6:], K @ tp.phi[d, :6], atol=1e-12)
    assert np.abs(np.linalg.eigvals(A + Bm @ K)).max() < 1.0


def test_tube_map_against_dense_definition(orc, small):
    """Block tube map == sum_j Phi_{k,j} c_j and row-wise l1 norms of
    Phi_{k,j} [E diag(rho_j)] built densely."""
    from oracle import tube
    tp = small
    B, N, nx = tp.batch.z.shape
    U = nx // 6
    r = np.random.default_rng(0)
    cb = r.normal(size=(B, N, nx)) * 1e-3
    rb = r.uniform(0, 1e-3, (B, N, nx))
    mu, sg = tube.tube_map(tp.phi, tp.e, cb, rb)
    E = np.diag(np.tile(tp.e, U))
    for b in range(B):
        for k in range(N):
            m = np.zeros(8 * U)
            s = np.zeros(8 * U)
            for j in range(k):
                P = _dense_phi(tp, k, j, U)
                m += P @ cb[b, j]
                Ebar = np.concatenate([E, np.diag(rb[b, j])], 1)
                s += np.abs(P @ Ebar).sum(1)          # || Phi E_bar ||_{1,r}
            np.testing.assert_allclose(mu[b, k], m, rtol=1e-12, atol=1e-15)
            np.testing.assert_allclose(sg[b, k], s, rtol=1e-12, atol=1e-15)


def test_tube_centre_follows_closed_loop_recursion(orc, small):
    """mu^x_{k+1} = A_cl mu^x_k + c_k and mu^u_k = K mu^x_k per node."""
    from oracle import tube
    tp = small
    B, N, nx = tp.batch.z.shape
    U = nx // 6
    cb = np.random.default_rng(1).normal(size=(B, N, nx))
    mu, _ = tube.tube_map(tp.phi, tp.e, cb, np.zeros_like(cb))
    for i in range(U):
        mx = mu[:, :, 6 * i:6 * i + 6]
        mu_u = mu[:, :, nx + 2 * i:nx + 2 * i + 2]
        for k in range(N - 1):
            np.testing.assert_allclose(mx[:, k + 1], mx[:, k] @ tp.A_cl.T + cb[:, k, 6 * i:6 * i + 6], atol=1e-12)
        np.testing.assert_allclose(mu_u, mx @ tp.K.T, atol=1e-12)


def test_sequential_sweep_is_fixed_point_and_jacobi_reaches_it(orc, small):
    from oracle import tube
    tp = small
    b = tp.batch
    d = orc.Dyn.like(b.dyn)
    mu, sg, lo, hi = tube.fixed_point(d, b.z, b.v, tp.phi, tp.e)
    # F(B*) = B*
    cb, rb = tube.zono(lo, hi)
    mu2, sg2 = tube.tube_map(tp.phi, tp.e, cb, rb)
    np.testing.assert_allclose(mu2, mu, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(sg2, sg, rtol=1e-12, atol=1e-15)
    # LEBs matter: the fixed point is larger than the disturbance-only tube
    _, sg0 = tube.tube_map(tp.phi, tp.e, np.zeros_like(cb), np.zeros_like(rb))
    assert (sg >= sg0 - 1e-15).all() and (sg > sg0 * (1 + 1e-6)).any()
    # Jacobi from the cold start (LEB = 0) reaches it after at most N sweeps
    m, s = np.zeros_like(mu), np.zeros_like(sg)
    N = b.z.shape[1]
    for it in range(N + 1):
        l_, h_, _ = orc.leb(d, b.z, b.v, s, mu=m)
        c_, r_ = tube.zono(l_, h_)
        m, s = tube.tube_map(tp.phi, tp.e, c_, r_)
    np.testing.assert_allclose(s, sg, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(m, mu, rtol=1e-12, atol=1e-15)


def test_fixed_point_is_certified(orc, small):
    """The sequential sweep yields F(B) = B exactly (same arithmetic in the
    same order), so the containment certificate F(B) inside B holds."""
    from oracle import tube
    tp = small
    b = tp.batch
    d = orc.Dyn.like(b.dyn)
    mu, sg, _, _ = tube.fixed_point(d, b.z, b.v, tp.phi, tp.e)
    l_, h_, _ = orc.leb(d, b.z, b.v, sg, mu=mu)
    c_, r_ = tube.zono(l_, h_)
    m2, s2 = tube.tube_map(tp.phi, tp.e, c_, r_)
    assert np.array_equal(m2, mu) and np.array_equal(s2, sg)
    assert tube.contains(mu, sg, m2, s2).all()


def test_uniform_inflation_fails_when_bounds_dominate(orc):
    """Where the bound grows faster than linearly in the radius and exceeds
    the disturbance, F(lambda B*) is not inside lambda B* for lambda > 1:
    a uniform inflation of the fixed point does not certify it."""
    from oracle import tube
    tp = W.fixed_point_cfg(seed=4, batch=4, N=40)
    b = tp.batch
    d = orc.Dyn.like(b.dyn)
    mu, sg, lo, hi = tube.fixed_point(d, b.z, b.v, tp.phi, tp.e)
    rho = 0.5 * (hi - lo)
    assert (rho.reshape(-1, 6) > tp.e[None, :] + 1e-12).any()
    sgi = sg * (1 + 1e-4)
    l_, h_, _ = orc.leb(d, b.z, b.v, sgi, mu=mu)
    c_, r_ = tube.zono(l_, h_)
    m2, s2 = tube.tube_map(tp.phi, tp.e, c_, r_)
    assert not tube.contains(mu, sgi, m2, s2).all()
    # a shrunken tube is not certified
    sgs = sg * 0.9
    l_, h_, _ = orc.leb(d, b.z, b.v, sgs, mu=mu)
    c_, r_ = tube.zono(l_, h_)
    m3, s3 = tube.tube_map(tp.phi, tp.e, c_, r_)
    assert not tube.contains(mu, sgs, m3, s3).any()


def test_zonotope_hull_is_vertex_maximum():
    """The hull radius of a zonotope row is max over the generator box of
    |G_i xi|, attained at a vertex: brute force over all 2^n vertices."""
    import itertools
    from oracle import tube
    rng = np.random.default_rng(5)
    G = rng.normal(size=(7, 9)) * rng.uniform(0, 2, (7, 1))
    G[3, :] = 0.0
    c = rng.normal(size=7)
    mu, sg = tube.zonotope_hull(G, c)
    V = np.array(list(itertools.product([-1.0, 1.0], repeat=9)))
    vals = V @ G.T                                  # [2^9][7]
    assert np.array_equal(mu, c)
    assert np.allclose(sg, np.abs(vals).max(0), rtol=1e-15, atol=0)
    assert sg[3] == 0.0
    # the tube width of the tube map is this hull of Phi_kj [E diag(rho_bar_j)]
    E = np.diag(rng.uniform(0, 1, 9))
    rb = rng.uniform(0, 1, 9)
    P = rng.normal(size=(5, 9))
    _, s1 = tube.zonotope_hull(np.concatenate([P @ E, P @ np.diag(rb)], 1))
    assert np.allclose(s1, np.abs(P) @ (np.diag(E) + rb), rtol=1e-14)
