"""GPU system-level-synthesis layer against the FP64 oracle: the Riccati
responses (appendix on solving for Phi), the time-varying tube map (eqs.
tight_tube_center, tight_tube_width), the linearization with the
state-dependent disturbance matrix (eqs. linearizations,
linearization_error_dist), and the exact tube/LEB fixed point of one
controller update with r_dist (eq. interval_r_dist).

Tolerances: responses and gains are FP64 on both sides in different
operation orders, so they agree to 1e-9 of the largest entry of each block.
Tube and bounds follow the library-wide parity bar: within 1e-4 of the
oracle's magnitude and never narrower by more than 1e-6 of it, with an
absolute floor of 1e-12 for entries that are zero in exact arithmetic (the
disturbance error at a zero-width tube is rounding on both sides)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

FLOOR = 1e-12


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2607_01203_amd as leb
    leb.lib()
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def sls(orc):
    from oracle import sls
    return sls


def _t(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _np(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _close_interval(lo_g, hi_g, lo_o, hi_o, where):
    M = np.maximum(np.abs(lo_o), np.abs(hi_o))
    tol = 1e-4 * M + FLOOR
    e = max((np.abs(lo_g - lo_o) - tol).max(), (np.abs(hi_g - hi_o) - tol).max())
    worst = max((np.abs(lo_g - lo_o) / (M + FLOOR)).max(), (np.abs(hi_g - hi_o) / (M + FLOOR)).max())
    assert e <= 0, "%s: relative error %.3e" % (where, worst)
    assert (lo_g <= lo_o + 1e-6 * M + FLOOR).all() and (hi_g >= hi_o - 1e-6 * M - FLOOR).all(), \
        "%s: narrower" % where


def _close_tube(mu_g, sg_g, mu_o, sg_o, where):
    assert np.isfinite(sg_g).all(), where
    scale = np.abs(mu_o) + sg_o
    ok_mu = np.abs(mu_g - mu_o) <= 1e-4 * scale + FLOOR
    ok_sg = np.abs(sg_g - sg_o) <= 1e-4 * scale + FLOOR
    e_mu = (np.abs(mu_g - mu_o) / (scale + FLOOR)).max()
    e_sg = (np.abs(sg_g - sg_o) / (scale + FLOOR)).max()
    assert ok_mu.all() and ok_sg.all(), "%s: mu %.3e sigma %.3e" % (where, e_mu, e_sg)
    assert (sg_g >= sg_o - 1e-6 * scale - FLOOR).all(), "%s: sigma narrower" % where


@pytest.mark.parametrize("nx,nu,N,batch", [(6, 2, 23, 3), (12, 4, 17, 2), (30, 10, 9, 2), (7, 3, 1, 2), (3, 1, 2, 2),
                                            (16, 4, 11, 2), (9, 1, 6, 2), (16, 5, 5, 1)])
def test_responses_parity(gpu, sls, nx, nu, N, batch):
    """Both kernels: FP64 MFMA tiles for 8 < nx <= 16 with nu <= 4, the
    LDS/VALU workgroup otherwise."""
    import paper_2607_01203_amd as leb
    A, B, qx, qu = W.random_ltv(100 + nx, batch, N, nx, nu, scale=0.2)
    print("case: responses nx=%d nu=%d N=%d batch=%d" % (nx, nu, N, batch), flush=True)
    K, phi = leb.sls_responses(_t(A, gpu), _t(B, gpu), _t(qx, gpu), _t(qu, gpu))
    K, phi = _np(K), _np(phi)
    for b in range(batch):
        Ko, _ = sls.riccati(A[b], B[b], qx[b], qu[b])
        Po, _ = sls.responses(A[b], B[b], Ko)
        for k in range(N):
            for j in range(N):
                if k <= j:
                    assert (phi[b, k, j] == 0).all() and (K[b, k, j] == 0).all()
                    continue
                s = max(np.abs(Po[k, j]).max(), 1e-300)
                assert np.abs(phi[b, k, j] - Po[k, j]).max() <= 1e-9 * s, (b, k, j)
                sk = max(np.abs(Ko[k, j]).max(), 1e-300)
                assert np.abs(K[b, k, j] - Ko[k, j]).max() <= 1e-9 * sk, (b, k, j)


def test_responses_long_horizon_reaches_the_dare_gain(gpu):
    """Time-invariant hover pair, constant weights, N = 150: the gain of the
    first disturbance time is the infinite-horizon LQR gain (scipy)."""
    import paper_2607_01203_amd as leb
    dyn = W.ChainDynamics(n_units=1)
    A0, B0, Kare = W.hover_lqr(dyn)
    N = 150
    A = np.broadcast_to(A0, (1, N, 6, 6)).copy()
    B = np.broadcast_to(B0, (1, N, 6, 2)).copy()
    qx = np.broadcast_to(np.asarray(W.HOVER_Q), (1, N + 1, N, 6)).copy()
    qu = np.full((1, N, N, 2), W.HOVER_R)
    print("case: responses DARE limit", flush=True)
    K, phi = leb.sls_responses(_t(A, gpu), _t(B, gpu), _t(qx, gpu), _t(qu, gpu))
    K = _np(K)
    assert np.abs(K[0, 1, 0] - Kare).max() <= 1e-8 * np.abs(Kare).max()


def _random_phi(rng, batch, N, n, nx):
    phi = rng.normal(size=(batch, N, N, n, nx)) * 0.5
    for k in range(N):
        phi[:, k, k:] = 0.0
    return phi


@pytest.mark.parametrize("nx,nu,nw,N,batch", [(6, 2, 7, 40, 3), (12, 4, 14, 19, 2), (30, 10, 0, 11, 2),
                                              (32, 16, 64, 5, 1), (2, 1, 1, 1, 2)])
def test_tube_map_parity(gpu, sls, nx, nu, nw, N, batch):
    import paper_2607_01203_amd as leb
    rng = np.random.default_rng(nx + nw)
    n = nx + nu
    phi = _random_phi(rng, batch, N, n, nx)
    E = rng.normal(size=(batch, N, nx, max(nw, 1)))[..., :nw] * 0.1
    cb = rng.normal(size=(batch, N, nx)) * 0.01
    rb = rng.uniform(0.0, 0.02, (batch, N, nx))
    print("case: tube map nx=%d nu=%d nw=%d N=%d" % (nx, nu, nw, N), flush=True)
    mu, sg = leb.sls_tube_map(_t(phi, gpu), _t(E, gpu) if nw else None, _t(cb, gpu), _t(rb, gpu))
    mu, sg = _np(mu), _np(sg)
    for b in range(batch):
        mo, so = sls.tube_map(phi[b], E[b] if nw else np.zeros((N, nx, 0)), cb[b], rb[b])
        scale = np.abs(mo) + so + 1e-300
        assert (np.abs(mu[b] - mo) <= 1e-12 * scale).all()
        assert (sg[b] >= so).all() and (sg[b] <= so + 1e-11 * scale).all()
    assert (mu[:, 0] == 0).all() and (sg[:, 0] == 0).all()


def test_tube_map_non_finite_residual(gpu):
    import paper_2607_01203_amd as leb
    rng = np.random.default_rng(3)
    N, nx, nu, nw = 9, 6, 2, 7
    phi = _random_phi(rng, 2, N, nx + nu, nx)
    E = rng.normal(size=(2, N, nx, nw))
    cb = rng.normal(size=(2, N, nx))
    rb = rng.uniform(0.0, 1.0, (2, N, nx))
    cb[0, 3, 2] = np.nan
    rb[1, 5, 0] = np.inf
    mu, sg = leb.sls_tube_map(_t(phi, gpu), _t(E, gpu), _t(cb, gpu), _t(rb, gpu))
    mu, sg = _np(mu), _np(sg)
    assert np.isfinite(sg[0, :4]).all() and np.isinf(sg[0, 4:]).all() and (mu[0, 4:] == 0).all()
    assert np.isfinite(sg[1, :6]).all() and np.isinf(sg[1, 6:]).all()


@pytest.mark.parametrize("n_units", [1, 2, 5])
def test_linearize_parity(gpu, orc, sls, n_units):
    import paper_2607_01203_amd as leb
    p = W.sls_cfg(seed=20 + n_units, batch=3, N=13, n_units=n_units)
    dyn = leb.dynamics_like(p.dyn)
    d = orc.Dyn.like(p.dyn)
    print("case: linearize U=%d" % n_units, flush=True)
    A, B, E = leb.linearize(dyn, _t(p.z, gpu), _t(p.v, gpu), p.e, p.thrust)
    A, B, E = _np(A), _np(B), _np(E)
    Ao, Bo = orc.jacobian(d, p.z, p.v)
    Eo = sls.disturbance_matrix(d, p.z, p.e, p.thrust)
    assert np.allclose(A, Ao, rtol=1e-14, atol=1e-15) and np.allclose(B, Bo, rtol=1e-14, atol=1e-15)
    assert np.allclose(E, Eo, rtol=1e-14, atol=1e-17)


def _oracle_update(orc, sls, p, b, pad):
    d = orc.Dyn.like(p.dyn)
    A, B = orc.jacobian(d, p.z[b], p.v[b])
    K, _ = sls.riccati(A, B, p.qx[b], p.qu[b])
    phi, _ = sls.responses(A, B, K)
    E = sls.disturbance_matrix(d, p.z[b], p.e, p.thrust)
    return sls.fixed_point(d, p.z[b], p.v[b], phi, E, pad=pad, thrust=p.thrust)


@pytest.mark.parametrize("n_units,thrust,N", [(1, 0.2, 40), (1, 0.0, 23), (2, 0.3, 17), (5, 0.2, 7)])
def test_sls_update_parity(gpu, orc, sls, n_units, thrust, N):
    """linearize -> responses -> fixed point on the GPU against the oracle's
    own chain (its Jacobians, Riccati responses and sequential fixed point)."""
    import paper_2607_01203_amd as leb
    p = W.sls_cfg(seed=30 + n_units, batch=3, N=N, n_units=n_units, thrust=thrust)
    dyn = leb.dynamics_like(p.dyn)
    print("case: sls update U=%d thrust=%g N=%d" % (n_units, thrust, N), flush=True)
    out = leb.sls_update(dyn, _t(p.z, gpu), _t(p.v, gpu), _t(p.qx, gpu), _t(p.qu, gpu), p.e, p.thrust, pad=1e-6)
    mu, sg, lo, hi, cert = (_np(out[k]) for k in ("mu", "sigma", "r_lo", "r_hi", "certified"))
    assert (cert == 1).all()
    for b in range(p.batch):
        mo, so, loo, hio = _oracle_update(orc, sls, p, b, 1e-6)
        _close_tube(mu[b], sg[b], mo, so, "tube U=%d b=%d" % (n_units, b))
        _close_interval(lo[b], hi[b], loo, hio, "bounds U=%d b=%d" % (n_units, b))


def test_sls_update_per_step_launches_until_the_tube_blows_up(gpu, orc, sls):
    """Five quadrotors at N = 60 do not fit the one-launch pass's LDS and take
    the per-step launches.  On these random nominals the tube grows into a
    spring singularity (the oracle's tube stops being finite near step 40):
    parity while the tube is moderate (every radius <= 1; closer to the
    singularity the bound's sensitivity amplifies the last-bit differences
    of the two sides), finite on both sides up to the same step, every later
    tube entry +inf, no certificate."""
    import paper_2607_01203_amd as leb
    p = W.sls_cfg(seed=35, batch=3, N=60, n_units=5, thrust=0.2)
    dyn = leb.dynamics_like(p.dyn)
    print("case: sls update U=5 N=60 per-step launches", flush=True)
    out = leb.sls_update(dyn, _t(p.z, gpu), _t(p.v, gpu), _t(p.qx, gpu), _t(p.qu, gpu), p.e, p.thrust, pad=1e-6)
    mu, sg, lo, hi, cert = (_np(out[k]) for k in ("mu", "sigma", "r_lo", "r_hi", "certified"))
    assert (cert == 0).all()
    for b in range(p.batch):
        with np.errstate(invalid="ignore", over="ignore"):
            mo, so, loo, hio = _oracle_update(orc, sls, p, b, 1e-6)
        fin_t = np.isfinite(so).all(1) & np.isfinite(mo).all(1)
        fin_r = np.isfinite(loo).all(1) & np.isfinite(hio).all(1)
        kt = int(np.argmin(fin_t)) if not fin_t.all() else p.N
        kr = int(np.argmin(fin_r)) if not fin_r.all() else p.N
        assert 10 < kt < p.N and kr < kt
        big = np.nanmax(np.where(np.isfinite(so), so, np.inf), 1) > 1.0
        km = int(np.argmax(big)) if big.any() else kt
        assert km > 10
        _close_tube(mu[b, :km], sg[b, :km], mo[:km], so[:km], "U=5 tube b=%d" % b)
        _close_interval(lo[b, :km], hi[b, :km], loo[:km], hio[:km], "U=5 bounds b=%d" % b)
        assert np.isfinite(sg[b, :kt]).all() and np.isfinite(lo[b, :kr]).all() and np.isfinite(hi[b, :kr]).all()
        assert np.isinf(sg[b, kt:]).all() and (mu[b, kt:] == 0).all()
        assert (~np.isfinite(lo[b, kr]) | ~np.isfinite(hi[b, kr])).any()


def test_sls_fixed_point_is_its_own_image(gpu):
    """The returned tube is C = F(C): the path-based bound over the returned
    tube (leb_analytic_bound) reproduces the returned bounds exactly (no
    disturbance error), and the tube map of the returned residual zonotopes
    reproduces the tube."""
    import torch
    import paper_2607_01203_amd as leb
    p = W.sls_cfg(seed=41, batch=4, N=21, n_units=2, thrust=0.0)
    dyn = leb.dynamics_like(p.dyn)
    z, v = _t(p.z, gpu), _t(p.v, gpu)
    out = leb.sls_update(dyn, z, v, _t(p.qx, gpu), _t(p.qu, gpu), p.e, 0.0, pad=0.0)
    r = leb.analytic_bound(dyn, z, v, out["sigma"], out["mu"])
    assert torch.equal(r["r_lo"], out["r_lo"]) and torch.equal(r["r_hi"], out["r_hi"])
    cb = 0.5 * (out["r_lo"] + out["r_hi"])
    rb = torch.maximum(out["r_hi"] - cb, cb - out["r_lo"])
    mu2, sg2 = leb.sls_tube_map(out["phi"], out["E"], cb, rb)
    # the library rounds rho_bar upward (by 2^-52 relative and 2^-1000), this check does not
    scale = out["mu"].abs() + out["sigma"]
    assert ((mu2 - out["mu"]).abs() <= 1e-12 * scale + 1e-290).all()
    assert ((sg2 - out["sigma"]).abs() <= 1e-12 * scale + 1e-290).all()


def test_sls_fixed_point_small_dynamics(gpu, orc, sls):
    """Satellite dynamics, responses of random time-varying pairs, constant E."""
    import paper_2607_01203_amd as leb
    N, batch = 12, 2
    z, v = W.small_nominals(W.SATELLITE, 5, batch * N)
    z, v = z.reshape(batch, N, 7), v.reshape(batch, N, 3)
    A, B, qx, qu = W.random_ltv(6, batch, N, 7, 3, scale=0.1)
    E = np.broadcast_to(1e-2 * np.eye(7), (batch, N, 7, 7)).copy()
    dyn = leb.dynamics_like(W.SATELLITE)
    print("case: sls fixed point satellite", flush=True)
    _, phi = leb.sls_responses(_t(A, gpu), _t(B, gpu), _t(qx, gpu), _t(qu, gpu))
    mu, sg, lo, hi, cert = leb.sls_fixed_point(dyn, _t(z, gpu), _t(v, gpu), phi, _t(E, gpu), 0.0, 1e-6)
    mu, sg, lo, hi, cert = _np(mu), _np(sg), _np(lo), _np(hi), _np(cert)
    d = orc.Dyn.like(W.SATELLITE)
    assert (cert == 1).all()
    for b in range(batch):
        K, _ = sls.riccati(A[b], B[b], qx[b], qu[b])
        po, _ = sls.responses(A[b], B[b], K)
        mo, so, loo, hio = sls.fixed_point(d, z[b], v[b], po, E[b], pad=1e-6)
        _close_tube(mu[b], sg[b], mo, so, "satellite tube b=%d" % b)
        _close_interval(lo[b], hi[b], loo, hio, "satellite bounds b=%d" % b)


def test_sls_update_full_size_sampled(gpu, orc, sls):
    """The bench workload (256 planar-quadrotor trajectories, N = 40, thrust
    disturbance) in one call: every trajectory certified and finite; four
    sampled trajectories against the oracle."""
    import paper_2607_01203_amd as leb
    p = W.sls_cfg()
    dyn = leb.dynamics_like(p.dyn)
    print("case: sls update full size", flush=True)
    out = leb.sls_update(dyn, _t(p.z, gpu), _t(p.v, gpu), _t(p.qx, gpu), _t(p.qu, gpu), p.e, p.thrust, pad=1e-6)
    mu, sg, lo, hi, cert = (_np(out[k]) for k in ("mu", "sigma", "r_lo", "r_hi", "certified"))
    assert (cert == 1).all() and np.isfinite(sg).all()
    for b in (0, 77, 200, 255):
        mo, so, loo, hio = _oracle_update(orc, sls, p, b, 1e-6)
        _close_tube(mu[b], sg[b], mo, so, "full-size tube b=%d" % b)
        _close_interval(lo[b], hi[b], loo, hio, "full-size bounds b=%d" % b)


def test_sls_update_sampled_soundness_1e6(gpu, orc, sls):
    """The bench workload's residual enclosures hold at 10^6 sampled points:
    for (x, u) in each step's tube box (z_k, v_k) + mu_k +- sigma_k (half
    uniform, a quarter vertices, a quarter mixed) and w in the unit box
    (vertices and uniform), the realised residual
        f(x, u) + E(x) w - f(z, v) - A_k dx - B_k du - E_k w
    (eq. linearization_error_all: r_lin + r_dist) lies in [r_lo, r_hi],
    up to its FP64 evaluation error."""
    import paper_2607_01203_amd as leb
    p = W.sls_cfg()
    dyn = leb.dynamics_like(p.dyn)
    d = orc.Dyn.like(p.dyn)
    print("case: sls update sampled soundness", flush=True)
    out = leb.sls_update(dyn, _t(p.z, gpu), _t(p.v, gpu), _t(p.qx, gpu), _t(p.qu, gpu), p.e, p.thrust, pad=1e-6)
    mu, sg, lo, hi, E = (_np(out[k]) for k in ("mu", "sigma", "r_lo", "r_hi", "E"))
    nx, n = p.dyn.nx, p.dyn.n
    nom = np.concatenate([p.z, p.v], -1).reshape(-1, n)
    blo = (nom + mu.reshape(-1, n) - sg.reshape(-1, n))
    bhi = (nom + mu.reshape(-1, n) + sg.reshape(-1, n))
    lo, hi, E = lo.reshape(-1, nx), hi.reshape(-1, nx), E.reshape(-1, nx, E.shape[-1])
    units = nom.shape[0]
    per = 98                                   # 10,240 units x 98 = 1.0e6 samples
    rng = W.rng_for(77)
    viol = 0
    total = 0
    for s0 in range(0, units, 512):
        s1 = min(units, s0 + 512)
        U = s1 - s0
        pts = W.sample_box_points(rng, blo[s0:s1], bhi[s0:s1], per)          # [U][per][n]
        uo = np.repeat(np.arange(U), per)
        r, eps = orc.remainder(d, nom[s0:s1], pts.reshape(-1, n), uo)
        w = np.where(rng.random((U * per, E.shape[-1])) < 0.5, rng.uniform(-1, 1, (U * per, E.shape[-1])),
                     np.sign(rng.uniform(-1, 1, (U * per, E.shape[-1]))))
        Ex = sls.disturbance_matrix(d, pts.reshape(-1, n)[:, :nx], p.e, p.thrust)
        rd = np.einsum("sij,sj->si", Ex - E[s0:s1][uo], w)
        tot = r + rd
        allow = eps + 1e-15 * (1.0 + np.abs(rd))
        L = lo[s0:s1][uo]
        H = hi[s0:s1][uo]
        viol += int(((tot > H + allow) | (tot < L - allow)).sum())
        total += U * per
    assert total >= 1_000_000
    assert viol == 0, viol


@pytest.mark.parametrize("N", [1, 2])
def test_sls_update_shortest_horizons(gpu, orc, sls, N):
    """N = 1: no responses, the tube is 0 and the bound is the nominal
    point's; N = 2: one response block."""
    import paper_2607_01203_amd as leb
    p = W.sls_cfg(seed=60 + N, batch=2, N=N, n_units=2, thrust=0.3)
    dyn = leb.dynamics_like(p.dyn)
    print("case: sls update N=%d" % N, flush=True)
    out = leb.sls_update(dyn, _t(p.z, gpu), _t(p.v, gpu), _t(p.qx, gpu), _t(p.qu, gpu), p.e, p.thrust, pad=1e-6)
    mu, sg, lo, hi, cert = (_np(out[k]) for k in ("mu", "sigma", "r_lo", "r_hi", "certified"))
    assert (cert == 1).all() and (mu[:, 0] == 0).all() and (sg[:, 0] == 0).all()
    for b in range(p.batch):
        mo, so, loo, hio = _oracle_update(orc, sls, p, b, 1e-6)
        _close_tube(mu[b], sg[b], mo, so, "N=%d tube b=%d" % (N, b))
        _close_interval(lo[b], hi[b], loo, hio, "N=%d bounds b=%d" % (N, b))


def test_sls_fixed_point_bad_nominal(gpu):
    """A non-finite nominal state at step 5 of one trajectory: that step's
    bound is [-inf, inf], every later tube entry +inf, the trajectory is not
    certified; the other trajectory is unaffected."""
    import torch
    import paper_2607_01203_amd as leb
    p = W.sls_cfg(seed=71, batch=2, N=12, n_units=1)
    dyn = leb.dynamics_like(p.dyn)
    z, v = _t(p.z, gpu), _t(p.v, gpu)
    A, B, E = leb.linearize(dyn, z, v, p.e, p.thrust)
    _, phi = leb.sls_responses(A, B, _t(p.qx, gpu), _t(p.qu, gpu))
    ref = leb.sls_fixed_point(dyn, z, v, phi, E, p.thrust, 1e-6)
    z2 = z.clone()
    z2[0, 5, 1] = float("nan")
    print("case: sls fixed point with a NaN nominal", flush=True)
    mu, sg, lo, hi, cert = leb.sls_fixed_point(dyn, z2, v, phi, E, p.thrust, 1e-6)
    torch.cuda.synchronize()
    assert cert.tolist() == [0, 1]
    assert torch.isinf(lo[0, 5]).all() and torch.isinf(hi[0, 5]).all()
    assert torch.isinf(sg[0, 6:]).all() and torch.isfinite(sg[0, :6]).all()
    assert torch.equal(sg[0, :6], ref[1][0, :6]) and torch.equal(mu[0, :6], ref[0][0, :6])
    for t_new, t_ref in zip((mu, sg, lo, hi), ref[:4]):
        assert torch.equal(t_new[1], t_ref[1])
