"""Pins of the oracle's system-level-synthesis layer (oracle/sls.py):

* the Riccati gains and responses (appendix on solving for Phi, eqs.
  backward_prop and forward_prop) against the reformulated problem (eq.
  fastsls_qp_reform) solved directly as a batch least-squares problem per
  disturbance time and column, against the discrete algebraic Riccati
  equation for a long time-invariant horizon, and against the system-level
  constraint (eq. fastsls_qp_err_dyn) with the start Phi^x_{j+1,j} = I;
* the tube map (eqs. tight_tube_center, tight_tube_width) against the vertex
  extremes of the zonotope it encloses;
* the disturbance error enclosure (eq. interval_r_dist) against sampled and
  extreme states;
* the whole fixed point against Theorem 3: closed-loop rollouts of the true
  nonlinear system with a state-dependent disturbance under the SLS
  controller stay inside the tube.
"""
import itertools

import numpy as np
import pytest
import scipy.linalg

import workloads as W


@pytest.fixture(scope="module")
def sls(orc):
    from oracle import sls
    return sls


def _ls_responses(A, B, qx, qu, j, i):
    """Minimise the cost of eq. fastsls_qp_cost_reform for disturbance time j
    and column i (start x_{j+1} = e_i) over the inputs u_{j+1..N-1} by
    linear least squares on the stacked affine state map."""
    N, nx, _ = A.shape
    nu = B.shape[2]
    m = N - j - 1
    # x_k = c_k + G_k U, U = [u_{j+1}; ...; u_{N-1}]
    c = np.zeros(nx)
    c[i] = 1.0
    G = np.zeros((nx, m * nu))
    rows, rhs = [], []
    for t, k in enumerate(range(j + 1, N)):
        sq = np.sqrt(qx[k, j])[:, None]
        rows.append(sq * G)
        rhs.append(-(sq[:, 0] * c))
        Su = np.zeros((nu, m * nu))
        Su[:, t * nu:(t + 1) * nu] = np.eye(nu)
        rows.append(np.sqrt(qu[k, j])[:, None] * Su)
        rhs.append(np.zeros(nu))
        c = A[k] @ c
        G = A[k] @ G + B[k] @ Su
    sq = np.sqrt(qx[N, j])[:, None]
    rows.append(sq * G)
    rhs.append(-(sq[:, 0] * c))
    M = np.concatenate(rows, 0)
    U = np.linalg.lstsq(M, np.concatenate(rhs), rcond=None)[0]
    xs, us = [], []
    c = np.zeros(nx)
    c[i] = 1.0
    x = c
    for t, k in enumerate(range(j + 1, N)):
        u = U[t * nu:(t + 1) * nu]
        xs.append(x)
        us.append(u)
        x = A[k] @ x + B[k] @ u
    return np.array(xs), np.array(us), x


@pytest.mark.parametrize("nx,nu,N", [(3, 2, 6), (4, 1, 7), (6, 2, 5)])
def test_riccati_responses_solve_the_reformulated_problem(sls, nx, nu, N):
    A, B, qx, qu = W.random_ltv(11 + nx, 1, N, nx, nu, scale=0.3)
    A, B, qx, qu = A[0], B[0], qx[0], qu[0]
    K, _ = sls.riccati(A, B, qx, qu)
    phi, term = sls.responses(A, B, K)
    for j in range(N):
        for i in range(nx):
            xs, us, xN = _ls_responses(A, B, qx, qu, j, i)
            for t, k in enumerate(range(j + 1, N)):
                assert np.allclose(phi[k, j, :nx, i], xs[t], rtol=1e-9, atol=1e-9)
                assert np.allclose(phi[k, j, nx:, i], us[t], rtol=1e-9, atol=1e-9)
            assert np.allclose(term[j][:, i], xN, rtol=1e-9, atol=1e-9)
        for k in range(j + 1):
            assert (phi[k, j] == 0).all()


def test_optimal_cost_is_trace_of_cost_to_go_and_minimal(sls):
    """The reformulated cost of the Riccati responses equals trace P_{j+1,j}
    (the start is I), and random gain perturbations only increase it."""
    A, B, qx, qu = W.random_ltv(3, 1, 8, 4, 2, scale=0.3)
    A, B, qx, qu = A[0], B[0], qx[0], qu[0]
    K, P = sls.riccati(A, B, qx, qu)
    rng = np.random.default_rng(0)
    for j in range(7):
        c0 = sls.reform_cost(A, B, K, qx, qu, j)
        assert abs(c0 - np.trace(P[j + 1, j])) <= 1e-10 * c0
        for _ in range(5):
            Kp = K + 1e-3 * rng.normal(size=K.shape)
            assert sls.reform_cost(A, B, Kp, qx, qu, j) >= c0 - 1e-12 * c0


def test_long_horizon_gain_is_the_dare_gain(sls):
    """Time-invariant pair, constant weights: far from the end the gain of
    every disturbance time is the infinite-horizon LQR gain."""
    dyn = W.ChainDynamics(n_units=1)
    A0, B0, Kd = W.hover_lqr(dyn)
    N = 300
    A = np.repeat(A0[None], N, 0)
    B = np.repeat(B0[None], N, 0)
    qx = np.broadcast_to(np.asarray(W.HOVER_Q), (N + 1, N, 6)).copy()
    qu = np.full((N, N, 2), W.HOVER_R)
    K, _ = sls.riccati(A, B, qx, qu)
    P = scipy.linalg.solve_discrete_are(A0, B0, np.diag(W.HOVER_Q), W.HOVER_R * np.eye(2))
    Kare = -np.linalg.solve(W.HOVER_R * np.eye(2) + B0.T @ P @ B0, B0.T @ P @ A0)
    assert np.allclose(Kd, Kare)
    for j in (0, 5, 40):
        assert np.abs(K[j + 1, j] - Kare).max() <= 1e-8 * np.abs(Kare).max()


def test_responses_satisfy_the_system_level_constraint(sls):
    A, B, qx, qu = W.random_ltv(5, 1, 9, 5, 3, scale=0.4)
    A, B, qx, qu = A[0], B[0], qx[0], qu[0]
    K, _ = sls.riccati(A, B, qx, qu)
    phi, term = sls.responses(A, B, K)
    nx = 5
    for j in range(9):
        if j + 1 < 9:
            assert (phi[j + 1, j, :nx] == np.eye(nx)).all()
        for k in range(j + 1, 9):
            nxt = term[j] if k == 8 else phi[k + 1, j, :nx]
            assert np.allclose(nxt, A[k] @ phi[k, j, :nx] + B[k] @ phi[k, j, nx:], rtol=1e-12, atol=1e-12)


def test_tube_map_is_the_zonotope_vertex_extreme(sls):
    """mu_k +- sigma_k are the extremes over the vertices of
    sum_j Phi_{k,j} (c_bar_j + [E_j diag(rho_bar_j)] xi_j)."""
    rng = np.random.default_rng(4)
    N, nx, nu, nw = 4, 2, 1, 1
    phi = rng.normal(size=(N, N, nx + nu, nx))
    for k in range(N):
        phi[k, k:] = 0.0
    E = rng.normal(size=(N, nx, nw))
    cb = rng.normal(size=(N, nx))
    rb = rng.uniform(0.0, 1.0, (N, nx))
    mu, sg = sls.tube_map(phi, E, cb, rb)
    for k in range(N):
        gens = [np.concatenate([phi[k, j] @ E[j], phi[k, j] * rb[j]], 1) for j in range(k)]
        c = sum((phi[k, j] @ cb[j] for j in range(k)), np.zeros(nx + nu))
        if not gens:
            assert (mu[k] == 0).all() and (sg[k] == 0).all()
            continue
        Gm = np.concatenate(gens, 1)
        verts = np.array(list(itertools.product((-1.0, 1.0), repeat=Gm.shape[1])))
        pts = c[None] + verts @ Gm.T
        assert np.allclose(mu[k] + sg[k], pts.max(0), rtol=1e-12, atol=1e-12)
        assert np.allclose(mu[k] - sg[k], pts.min(0), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("perturb", [0.0, 1e-3])
def test_r_dist_encloses_and_reaches_the_disturbance_error(orc, sls, perturb):
    """|(E(x) - E_k) w| over x in the tube box and |w| <= 1 stays within s
    and reaches it at the theta extremes (the endpoints or the critical
    point of the cosine)."""
    dyn = orc.Dyn.chain(2)
    rng = np.random.default_rng(6)
    e = np.tile([0.0, 0.0, 0.0, 0.02, 0.02, 0.0], 2)
    for trial in range(40):
        z = rng.uniform(-0.5, 0.5, 12)
        mu = rng.uniform(-0.05, 0.05, 12)
        sg = rng.uniform(0.0, 0.4, 12)
        Ek = sls.disturbance_matrix(dyn, z, e, 0.3)
        for i in range(2):                  # a nominal matrix not taken at the box's centre
            Ek[6 * i + 3:6 * i + 5, 12 + i] += perturb * rng.normal(size=2)
        s = sls.r_dist(dyn, Ek, z, mu, sg, 0.3)
        ths = []
        for i in range(2):
            t = 6 * i + 2
            lo, hi = z[t] + mu[t] - sg[t], z[t] + mu[t] + sg[t]
            cand = np.concatenate([[lo, hi], rng.uniform(lo, hi, 200), [0.0] if lo <= 0.0 <= hi else []])
            ths.append(cand)
        best = np.zeros(12)
        for th0 in ths[0]:
            for th1 in ths[1][:20]:
                x = z + mu
                x[2], x[8] = th0, th1
                D = np.abs(sls.disturbance_matrix(dyn, x, e, 0.3) - Ek).sum(1)   # w at the best vertex
                best = np.maximum(best, D)
        assert (best <= s + 1e-15).all(), (trial, best - s)
        rows = [3, 4]
        assert np.allclose(best[rows], s[rows], rtol=1e-9, atol=1e-15)
    assert (sls.r_dist(dyn, Ek, z, mu, sg, 0.0) == 0).all()


def _rollout(orc, dyn, z0, v):
    z = [np.asarray(z0, dtype=np.float64)]
    for k in range(v.shape[0]):
        z.append(orc.step(dyn, z[-1][None], v[k][None])[0])
    return np.array(z)


@pytest.mark.parametrize("n_units,thrust", [(1, 0.5), (2, 0.3)])
def test_theorem_3_closed_loop_rollouts_stay_in_the_tube(orc, sls, n_units, thrust):
    """Dynamically consistent nominal (z_{k+1} = f(z_k, v_k)), Riccati
    responses from its Jacobians, the fixed-point tube with the thrust
    disturbance; the true system x+ = f(x, u) + E(x) w under the SLS
    controller u_k = v_k + sum_j Phi^u_{k,j} d_j (d_j the realised total
    disturbance) stays in z_k + mu_k +- sigma_k for every sampled w."""
    dyn = orc.Dyn.chain(n_units)
    nx, nu = dyn.nx, dyn.nu
    N = 14
    rng = np.random.default_rng(10 + n_units)
    z0 = np.zeros(nx)
    for i in range(n_units):
        z0[6 * i] = 0.2 * i
        z0[6 * i + 2] = 0.1
    hover = 0.5 * 1.0 * 9.81
    t = np.arange(N)
    v = np.empty((N, nu))
    for i in range(n_units):
        v[:, 2 * i] = hover + 0.4 * np.sin(0.5 * t + i)
        v[:, 2 * i + 1] = hover + 0.4 * np.cos(0.3 * t)
    z = _rollout(orc, dyn, z0, v)
    A, B = orc.jacobian(dyn, z[:N], v)
    qx = np.broadcast_to(np.tile(np.asarray(W.HOVER_Q), n_units), (N + 1, N, nx)).copy()
    qu = np.full((N, N, nu), W.HOVER_R)
    K, _ = sls.riccati(A, B, qx, qu)
    phi, _ = sls.responses(A, B, K)
    e = np.tile([0.0, 0.0, 0.0, 0.02, 0.02, 0.0], n_units)
    E = sls.disturbance_matrix(dyn, z[:N], e, thrust)
    mu, sg, lo, hi = sls.fixed_point(dyn, z[:N], v, phi, E, pad=0.0, thrust=thrust)
    assert np.isfinite(sg).all()
    nw = E.shape[2]
    worst = 0.0
    for trial in range(150):
        if trial % 3 == 0:
            w = rng.uniform(-1.0, 1.0, (N, nw))
        else:
            w = rng.choice([-1.0, 1.0], (N, nw))
        x = z0.copy()
        d = np.zeros((N, nx))
        for k in range(N):
            du = sum((phi[k, j, nx:] @ d[j] for j in range(k)), np.zeros(nu))
            u = v[k] + du
            dev = np.concatenate([x - z[k], du])
            tol = 1e-10 * (1.0 + np.abs(mu[k]) + sg[k])
            assert (np.abs(dev - mu[k]) <= sg[k] + tol).all(), (trial, k, dev - mu[k], sg[k])
            worst = max(worst, float((np.abs(dev - mu[k]) / np.maximum(sg[k], 1e-300))[sg[k] > 0].max(initial=0)))
            Ex = sls.disturbance_matrix(dyn, x, e, thrust)
            xn = orc.step(dyn, x[None], u[None])[0] + Ex @ w[k]
            d[k] = (xn - z[k + 1]) - A[k] @ (x - z[k]) - B[k] @ du
            # the realised disturbance lies in its zonotope
            rad = np.abs(E[k]).sum(1) + 0.5 * (hi[k] - lo[k])
            assert (np.abs(d[k] - 0.5 * (lo[k] + hi[k])) <= rad + 1e-12).all(), (trial, k)
            x = xn
    assert worst > 0.3          # the rollouts use a fair share of the tube


def test_fixed_point_reproduces_itself(orc, sls):
    """The tube is the tube map of its own residual zonotopes, and each
    step's bound is the bound over its own tube set."""
    p = W.sls_cfg(seed=7, batch=1, N=10, n_units=2)
    dyn = orc.Dyn.like(p.dyn)
    A, B = orc.jacobian(dyn, p.z[0], p.v[0])
    K, _ = sls.riccati(A, B, p.qx[0], p.qu[0])
    phi, _ = sls.responses(A, B, K)
    E = sls.disturbance_matrix(dyn, p.z[0], p.e, p.thrust)
    mu, sg, lo, hi = sls.fixed_point(dyn, p.z[0], p.v[0], phi, E, pad=1e-6, thrust=p.thrust)
    mu2, sg2 = sls.tube_map(phi, E, 0.5 * (lo + hi), 0.5 * (hi - lo) + 1e-6)
    assert np.allclose(mu2, mu, rtol=1e-13, atol=1e-15) and np.allclose(sg2, sg, rtol=1e-13, atol=1e-15)
    l_, h_, _ = orc.leb(dyn, p.z[0], p.v[0], sg, mu=mu)
    s = np.array([sls.r_dist(dyn, E[k], p.z[0, k], mu[k], sg[k], p.thrust) for k in range(10)])
    assert np.array_equal(l_ - s, lo) and np.array_equal(h_ + s, hi)
