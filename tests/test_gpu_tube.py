"""GPU tube map and certified tube/LEB fixed point against the oracle."""
import numpy as np
import pytest

import workloads as W

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


def test_tube_map_parity(gpu, orc):
    import torch
    import paper_2607_01203_amd as leb
    from oracle import tube
    tp = W.fixed_point_cfg(seed=44, batch=5, N=23, n_units=7)
    B, N, nx = tp.batch.z.shape
    r = np.random.default_rng(2)
    cb = r.normal(size=(B, N, nx)) * 1e-3
    rb = r.uniform(0, 1e-3, (B, N, nx))
    print("case: tube map B=5 N=23 U=7", flush=True)
    mu, sg = leb.tube_map(7, _t(tp.phi, gpu), tp.e, _t(cb, gpu), _t(rb, gpu))
    torch.cuda.synchronize()
    mo, so = tube.tube_map(tp.phi, tp.e, cb, rb)
    mu, sg = mu.cpu().numpy(), sg.cpu().numpy()
    np.testing.assert_allclose(mu, mo, rtol=1e-12, atol=1e-15)
    assert (sg >= so).all() and (sg <= so * (1 + 1e-11) + 1e-15).all()


def test_tube_map_non_finite_residual(gpu, orc):
    """A residual that is not finite at step j of one node makes sigma +inf
    at that node's later steps only; earlier steps and other nodes keep the
    finite result (the zero blocks of the contraction never turn it to NaN)."""
    import torch
    import paper_2607_01203_amd as leb
    from oracle import tube
    tp = W.fixed_point_cfg(seed=51, batch=2, N=10, n_units=5)
    B, N, nx = tp.batch.z.shape
    r = np.random.default_rng(3)
    cb = r.normal(size=(B, N, nx)) * 1e-3
    rb = r.uniform(0, 1e-3, (B, N, nx))
    mo, so = tube.tube_map(tp.phi, tp.e, cb, rb)
    cb2, rb2 = cb.copy(), rb.copy()
    rb2[1, 4, 6 * 2 + 3] = np.inf          # trajectory 1, step 4, node 2, vx row
    cb2[0, 6, 6 * 4 + 1] = np.nan          # trajectory 0, step 6, node 4
    print("case: tube map with non-finite residuals", flush=True)
    mu, sg = leb.tube_map(5, _t(tp.phi, gpu), tp.e, _t(cb2, gpu), _t(rb2, gpu))
    torch.cuda.synchronize()
    mu, sg = mu.cpu().numpy(), sg.cpu().numpy()
    n = 8 * 5
    node = lambda i: list(range(6 * i, 6 * i + 6)) + [30 + 2 * i, 31 + 2 * i]
    inf_mask = np.zeros(sg.shape, dtype=bool)
    inf_mask[1, 5:, node(2)] = True
    inf_mask[0, 7:, node(4)] = True
    assert np.isinf(sg[inf_mask]).all() and not np.isnan(sg).any() and not np.isnan(mu).any()
    fin = ~inf_mask
    assert (sg[fin] >= so[fin]).all() and (sg[fin] <= so[fin] * (1 + 1e-11) + 1e-15).all()
    ok_mu = np.ones(mu.shape, dtype=bool)
    ok_mu[0, 7:, node(4)] = False          # the NaN centre entered as 0: only sigma is meaningful there
    np.testing.assert_allclose(mu[ok_mu], mo[ok_mu], rtol=1e-12, atol=1e-15)


def _solve(leb, tp, dev, **kw):
    import torch
    b = tp.batch
    dyn = leb.dynamics_like(b.dyn)
    mu, sg, cert, sweeps = leb.fixed_point_solve(dyn, _t(b.z, dev), _t(b.v, dev), _t(tp.phi, dev), tp.e, **kw)
    torch.cuda.synchronize()
    return mu.cpu().numpy(), sg.cpu().numpy(), cert.cpu().numpy(), sweeps


def _check_against_oracle(orc, tp, mu, sg, idx):
    from oracle import tube
    b = tp.batch
    d = orc.Dyn.like(b.dyn)
    mo, so, _, _ = tube.fixed_point(d, b.z[idx], b.v[idx], tp.phi, tp.e)
    # the certified tube contains the least fixed point and is close to it
    assert (sg[idx] >= so * (1 - 1e-12)).all()
    M = np.maximum(so, 1e-300)
    rel = np.where(so > 0, (sg[idx] - so) / M, 0.0)
    assert rel.max() <= 1e-4, rel.max()
    assert (np.abs(mu[idx] - mo) <= 1e-4 * np.maximum(so, 1e-12)).all()


def test_fixed_point_small(gpu, orc):
    import paper_2607_01203_amd as leb
    tp = W.fixed_point_cfg(seed=45, batch=6, N=12, n_units=4)
    print("case: fixed point B=6 N=12 U=4", flush=True)
    mu, sg, cert, sweeps = _solve(leb, tp, gpu)
    assert (cert == 1).all()
    assert 2 <= sweeps <= 12 + 2
    _check_against_oracle(orc, tp, mu, sg, np.arange(6))


def test_fixed_point_full_shape(gpu, orc):
    """256 trajectories x 40 steps, 168 states; oracle on a sample."""
    import paper_2607_01203_amd as leb
    tp = W.fixed_point_cfg()
    print("case: fixed point 256x40x168", flush=True)
    mu, sg, cert, sweeps = _solve(leb, tp, gpu)
    print("sweeps", sweeps)
    assert (cert == 1).all()
    _check_against_oracle(orc, tp, mu, sg, np.array([0, 77, 255]))


def test_fixed_point_large_batch(gpu, orc):
    """1,024 trajectories x 40 steps, 168 states (four times the bench
    batch: 4,552 bound workgroups, a fold over four state words per lane);
    the oracle on a sample."""
    import paper_2607_01203_amd as leb
    tp = W.fixed_point_cfg(seed=5, batch=1024, N=40)
    print("case: fixed point 1024x40x168", flush=True)
    mu, sg, cert, sweeps = _solve(leb, tp, gpu)
    print("sweeps", sweeps)
    assert (cert == 1).all()
    _check_against_oracle(orc, tp, mu, sg, np.array([0, 513, 1023]))


@pytest.mark.parametrize("batch,N,U", [(3, 46, 6), (2, 9, 40), (2, 70, 3), (1, 131, 2), (300, 2, 1), (4, 1, 3), (1, 210, 2)])
def test_fixed_point_long_horizon_and_long_chain(gpu, orc, batch, N, U):
    """A horizon of 46 steps (two row groups in the tube map), a chain of 40
    nodes (6 steps per bound workgroup), horizons of 70 and 131 steps (Phi
    and the residuals staged in two and three passes, up to four row
    groups), and 300 two-step trajectories of one node (a bound workgroup
    spans 128 trajectories; the fold covers more trajectories than lanes),
    a horizon of one step (no Phi: the tube is the known initial state), and
    the longest horizon the compact tube map keeps in LDS (210 steps)."""
    import paper_2607_01203_amd as leb
    tp = W.fixed_point_cfg(seed=60 + N, batch=batch, N=N, n_units=U)
    print("case: fixed point B=%d N=%d U=%d" % (batch, N, U), flush=True)
    mu, sg, cert, sweeps = _solve(leb, tp, gpu)
    assert (cert == 1).all()
    _check_against_oracle(orc, tp, mu, sg, np.arange(batch))


def test_fixed_point_certificate_holds(gpu, orc):
    """Recheck the certificate with the oracle: F(B) inside B."""
    import paper_2607_01203_amd as leb
    from oracle import tube
    tp = W.fixed_point_cfg(seed=46, batch=4, N=15, n_units=5)
    mu, sg, cert, _ = _solve(leb, tp, gpu)
    assert (cert == 1).all()
    b = tp.batch
    d = orc.Dyn.like(b.dyn)
    lo, hi, _ = orc.leb(d, b.z, b.v, sg, mu=mu)
    c, r = tube.zono(lo, hi)
    m2, s2 = tube.tube_map(tp.phi, tp.e, c, r)
    assert tube.contains(mu, sg, m2, s2).all()


def test_fixed_point_warm_start_from_above(gpu, orc):
    """A warm start 1% above the certified tube is a post-fixed point, so
    every iterate is certified; the solve keeps sweeping until the iterates
    converge (conv_tol), ending within the parity tolerance of the least
    fixed point like the cold start, never below it, no wider than the tube
    passed in, and in no more sweeps than the cold start."""
    import torch
    import paper_2607_01203_amd as leb
    tp = W.fixed_point_cfg(seed=48, batch=4, N=14, n_units=4)
    print("case: warm start B=4 N=14 U=4", flush=True)
    mu, sg, cert, sweeps = _solve(leb, tp, gpu)
    assert (cert == 1).all()
    b = tp.batch
    dyn = leb.dynamics_like(b.dyn)
    s_in = sg * (1 + 1e-2)
    mu2, sg2, cert2, sw2 = leb.fixed_point_solve(dyn, _t(b.z, gpu), _t(b.v, gpu), _t(tp.phi, gpu), tp.e,
                                                 mu=_t(mu, gpu), sigma=_t(s_in, gpu))
    torch.cuda.synchronize()
    mu2, sg2 = mu2.cpu().numpy(), sg2.cpu().numpy()
    print("sweeps: cold %d, warm from above %d" % (sweeps, sw2))
    assert (cert2.cpu().numpy() == 1).all() and 2 <= sw2 <= sweeps, (sw2, sweeps)
    assert (sg2 <= s_in * (1 + 1e-6) + 1e-11).all()
    _check_against_oracle(orc, tp, mu2, sg2, np.arange(4))


def test_fixed_point_warm_start_from_below(gpu, orc):
    """A warm start that is not a post-fixed point (half the least fixed
    point's width, zero centre) still ends certified at the cold start's
    tube: the causal map forgets its start within N + 1 sweeps."""
    import paper_2607_01203_amd as leb
    from oracle import tube
    tp = W.fixed_point_cfg(seed=49, batch=3, N=12, n_units=4)
    b = tp.batch
    d = orc.Dyn.like(b.dyn)
    mo, so, _, _ = tube.fixed_point(d, b.z, b.v, tp.phi, tp.e)
    print("case: warm start from below B=3 N=12 U=4", flush=True)
    mu, sg, cert, sweeps = _solve(leb, tp, gpu, mu=_t(np.zeros_like(mo), gpu), sigma=_t(0.5 * so, gpu))
    assert (cert == 1).all()
    assert 2 <= sweeps <= 12 + 2, sweeps
    _check_against_oracle(orc, tp, mu, sg, np.arange(3))


def test_fixed_point_trajectories_certified_at_different_sweeps(gpu, orc):
    """Half the batch starts from the accepted tube of a cold solve
    (certified and converged, so accepted by the first sweep and returned
    unchanged), half from a zero tube (accepted several sweeps later);
    5 x 7 nodes = 35 columns per trajectory, so columns of one trajectory
    straddle waves."""
    import torch
    import paper_2607_01203_amd as leb
    tp = W.fixed_point_cfg(seed=49, batch=6, N=13, n_units=7)
    print("case: mixed certification B=6 N=13 U=7", flush=True)
    mu, sg, cert, sweeps = _solve(leb, tp, gpu)
    assert (cert == 1).all()
    b = tp.batch
    dyn = leb.dynamics_like(b.dyn)
    m_in = mu.copy()
    s_in = sg.copy()
    m_in[1::2] = 0.0
    s_in[1::2] = 0.0
    mu2, sg2, cert2, sw2 = leb.fixed_point_solve(dyn, _t(b.z, gpu), _t(b.v, gpu), _t(tp.phi, gpu), tp.e,
                                                 mu=_t(m_in, gpu), sigma=_t(s_in, gpu))
    torch.cuda.synchronize()
    mu2, sg2 = mu2.cpu().numpy(), sg2.cpu().numpy()
    print("sweeps", sweeps, sw2)
    assert (cert2.cpu().numpy() == 1).all() and sw2 >= 3
    assert np.array_equal(sg2[0::2], s_in[0::2]) and np.array_equal(mu2[0::2], m_in[0::2])
    _check_against_oracle(orc, tp, mu2, sg2, np.arange(1, 6, 2))


def test_fixed_point_sweep_cap_not_certified(gpu):
    import paper_2607_01203_amd as leb
    tp = W.fixed_point_cfg(seed=47, batch=3, N=10, n_units=3)
    mu, sg, cert, sweeps = _solve(leb, tp, gpu, max_sweeps=1)
    assert sweeps == 1 and (cert == 0).all()


def test_fixed_point_boxes_sound_1e6(gpu, orc):
    """LEBs on the accepted tube boxes contain 10^6 sampled remainders."""
    import torch
    import paper_2607_01203_amd as leb
    tp = W.fixed_point_cfg(seed=4, batch=16, N=40)
    mu, sg, cert, _ = _solve(leb, tp, gpu)
    assert (cert == 1).all()
    b = tp.batch
    dyn = leb.dynamics_like(b.dyn)
    out = leb.analytic_bound(dyn, _t(b.z, gpu), _t(b.v, gpu), _t(sg, gpu), _t(mu, gpu))
    torch.cuda.synchronize()
    lo = out["r_lo"].cpu().numpy().reshape(-1, 168)
    hi = out["r_hi"].cpu().numpy().reshape(-1, 168)
    d = orc.Dyn.like(b.dyn)
    nom = np.concatenate([b.z, b.v], -1).reshape(-1, 224)
    blo, bhi = orc.box(nom, sg.reshape(-1, 224), mu.reshape(-1, 224))
    rng = W.rng_for(1_000_004)
    per = 1_000_000 // nom.shape[0] + 1
    viol = 0
    for s in range(0, nom.shape[0], 64):
        e = min(nom.shape[0], s + 64)
        pts = W.sample_box_points(rng, blo[s:e], bhi[s:e], per)
        r, eps = orc.remainder(d, nom[s:e], pts.reshape(-1, 224), np.repeat(np.arange(e - s), per))
        r = r.reshape(e - s, per, 168)
        eps = eps.reshape(e - s, per, 168)
        viol += int(((r > hi[s:e, None] + eps) | (r < lo[s:e, None] - eps)).sum())
    assert viol == 0
