"""Learned warm start on the GPU: chain surrogates trained by the library's
own kernels on certified bounds (one that maps a tube to its bound, one
that maps the cold start to the fixed point's bound), the bound-map
network's prediction quality on held-out trajectories, and the learned
fixed point: certified and converged like the cold start (checked again
with the oracle), within the parity tolerance of the least fixed point, and
what the trained network gains in certified sweeps."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _t(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


@pytest.fixture(scope="module")
def trained():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2607_01203_amd as leb
    from paper_2607_01203_amd import learned
    dev = torch.device("cuda:0")
    tp = W.fixed_point_cfg(seed=100, batch=32, N=40)
    b = tp.batch
    dyn = leb.dynamics_like(b.dyn)
    z, v = _t(b.z, dev), _t(b.v, dev)
    print("case: learned -- training set", flush=True)
    mu, sg, cert, _ = leb.fixed_point_solve(dyn, z, v, _t(tp.phi, dev), tp.e)
    assert bool((cert == 1).all())
    X, T = learned.chain_samples(dyn, z, v, mu.cpu().numpy(), sg.cpu().numpy(), draws=3, seed=1)
    net = leb.Surrogate(learned.CHAIN_WIDTHS, learned.he_init(learned.CHAIN_WIDTHS, 0))
    hist = learned.train(net, X, T, epochs=12, batch=1024, lr=2e-3)
    print("train loss", hist[0], hist[-1], flush=True)
    yield leb, net, dev, hist
    net.close()


def test_training_converges_and_generalises(trained):
    from paper_2607_01203_amd import learned
    leb, net, dev, hist = trained
    assert hist[-1] < 0.1 * hist[0]
    tp = W.fixed_point_cfg(seed=101, batch=8, N=40)
    b = tp.batch
    dyn = leb.dynamics_like(b.dyn)
    z, v = _t(b.z, dev), _t(b.v, dev)
    mu, sg, _, _ = leb.fixed_point_solve(dyn, z, v, _t(tp.phi, dev), tp.e)
    X, T = learned.chain_samples(dyn, z, v, mu.cpu().numpy(), sg.cpu().numpy(), draws=1, seed=2)
    ev = learned.evaluate(net, X, T)
    print("held-out", ev)
    # median error of the predicted bound within 25% (log space)
    assert ev["abs_log_err_q50_q90_q99"][0] < 0.22


def test_fused_surrogate_sweep_equals_its_parts(trained):
    """leb_chain_surrogate_bound (features, MLP and decoding in one kernel)
    equals the chain features, the MLP forward and the decoding run apart."""
    import torch
    leb, net, dev, _ = trained
    tp = W.fixed_point_cfg(seed=52, batch=3, N=9, n_units=28)
    b = tp.batch
    dyn = leb.dynamics_like(b.dyn)
    z, v = _t(b.z, dev), _t(b.v, dev)
    r = np.random.default_rng(5)
    sg = _t(r.uniform(0.0, 0.05, b.sigma.shape), dev)
    mu = _t(r.uniform(-0.01, 0.01, b.sigma.shape), dev)
    cb, rb = leb.chain_surrogate_bound(dyn, z, v, sg, net, mu=mu, pad=1e-9)
    x = leb.chain_features(dyn, z, v, sg, mu=mu).reshape(-1, leb.CHAIN_FEATURES)
    y = net.forward(x).cpu().numpy().astype(np.float64).reshape(3, 9, 28, 4)
    torch.cuda.synchronize()
    hi = np.exp(np.minimum(y[..., 0::2], 0.0))
    lo = -np.exp(np.minimum(y[..., 1::2], 0.0))
    c_exp = np.zeros((3, 9, 168))
    r_exp = np.full((3, 9, 168), 1e-9)
    for w in range(2):
        c_exp[..., 3 + w::6] = 0.5 * (lo[..., w] + hi[..., w])
        r_exp[..., 3 + w::6] = 0.5 * (hi[..., w] - lo[..., w]) + 1e-9
    np.testing.assert_allclose(cb.cpu().numpy(), c_exp, rtol=1e-13, atol=1e-300)
    np.testing.assert_allclose(rb.cpu().numpy(), r_exp, rtol=1e-13, atol=1e-300)


def _oracle_fixed_point(orc, tp, idx):
    from oracle import tube
    b = tp.batch
    d = orc.Dyn.like(b.dyn)
    return tube.fixed_point(d, b.z[idx], b.v[idx], tp.phi, tp.e)


@pytest.fixture(scope="module")
def trained_fp(trained):
    """A fixed-point-target network: one sweep from the cold start predicts
    the bound at the fixed point (features of the disturbance-only tube,
    targets of the certified fixed point), trained on 64 other trajectories."""
    import torch
    from paper_2607_01203_amd import learned
    leb, _, dev, _ = trained
    tp = W.fixed_point_cfg(seed=100, batch=64, N=40)
    b = tp.batch
    dyn = leb.dynamics_like(b.dyn)
    z, v, phi = _t(b.z, dev), _t(b.v, dev), _t(tp.phi, dev)
    mu, sg, cert, _ = leb.fixed_point_solve(dyn, z, v, phi, tp.e)
    assert bool((cert == 1).all())
    X, T = learned.chain_fp_samples(dyn, z, v, phi, tp.e, mu, sg, seed=3)
    net = leb.Surrogate(learned.CHAIN_WIDTHS, learned.he_init(learned.CHAIN_WIDTHS, 0))
    hist = learned.train(net, X, T, epochs=100, batch=1024, lr=2e-3)
    torch.cuda.synchronize()
    print("fixed-point-target loss", hist[0], hist[-1], flush=True)
    yield net, hist
    net.close()


def test_learned_fixed_point_equal_tightness(trained, trained_fp, orc):
    """The learned form on the full fixed-point workload (256 x 40 x 168),
    with both networks: every trajectory certified and converged like the
    cold start, so the accepted tube lies within the parity tolerance of the
    oracle's least fixed point on sampled trajectories (and of the cold
    start's tube everywhere); the certificate rechecked by the oracle."""
    import torch
    from oracle import tube
    leb, net, dev, _ = trained
    net_fp, _ = trained_fp
    tp = W.fixed_point_cfg(seed=4, batch=256, N=40)
    b = tp.batch
    dyn = leb.dynamics_like(b.dyn)
    z, v, phi = _t(b.z, dev), _t(b.v, dev), _t(tp.phi, dev)
    print("case: learned fixed point 256x40x168", flush=True)
    _, sg0, c0, sw0 = leb.fixed_point_solve(dyn, z, v, phi, tp.e)
    sg0 = sg0.cpu().numpy()
    idx = np.array([0, 77, 255])
    mo, so, _, _ = _oracle_fixed_point(orc, tp, idx)
    d = orc.Dyn.like(b.dyn)
    for name, nw in (("bound-map", net), ("fixed-point-target", net_fp)):
        mu1, sg1, c1, sw1 = leb.fixed_point_learned(dyn, z, v, phi, tp.e, nw, sweeps=1, margin=0.0)
        torch.cuda.synchronize()
        mu1, sg1 = mu1.cpu().numpy(), sg1.cpu().numpy()
        pos = sg0 > 0
        rel = np.abs(sg1[pos] / sg0[pos] - 1.0)
        print("%s: certified sweeps %d (cold %d); |sigma / cold - 1| max %.2e" % (name, sw1, sw0, rel.max()))
        assert bool((c1 == 1).all()) and bool((c0 == 1).all())
        assert rel.max() <= 1e-4
        assert (sg1[idx] >= so * (1 - 1e-12)).all()
        r = np.where(so > 0, (sg1[idx] - so) / np.maximum(so, 1e-300), 0.0)
        assert r.max() <= 1e-4, r.max()
        assert (np.abs(mu1[idx] - mo) <= 1e-4 * np.maximum(so, 1e-12)).all()
        lo, hi, _ = orc.leb(d, b.z[idx], b.v[idx], sg1[idx], mu=mu1[idx])
        c, rr = tube.zono(lo, hi)
        m2, s2 = tube.tube_map(tp.phi, tp.e, c, rr)
        assert tube.contains(mu1[idx], sg1[idx], m2, s2).all()


def test_learned_start_gain(trained, trained_fp):
    """What the trained network gains over the method without it, at equal
    tightness (every form accepted only when certified and converged): the
    certified sweeps and wall time of the cold start, of one exact sweep
    then the iteration (the start the surrogate sweep emulates), and of the
    learned start with each network and with an untrained network.  The
    trained fixed-point-target start needs fewer certified sweeps than the
    cold start and than the untrained network's start."""
    import time
    import torch
    from paper_2607_01203_amd import learned
    leb, net, dev, _ = trained
    net_fp, _ = trained_fp
    tp = W.fixed_point_cfg(seed=4, batch=256, N=40)
    b = tp.batch
    dyn = leb.dynamics_like(b.dyn)
    z, v, phi = _t(b.z, dev), _t(b.v, dev), _t(tp.phi, dev)
    untrained = leb.Surrogate(learned.CHAIN_WIDTHS, learned.he_init(learned.CHAIN_WIDTHS, 9))

    def exact_start():
        m, s_, _, _ = leb.fixed_point_solve(dyn, z, v, phi, tp.e, max_sweeps=1)
        r = leb.fixed_point_solve(dyn, z, v, phi, tp.e, mu=m, sigma=s_)
        return r[0], r[1], r[2], 1 + r[3]

    forms = {"cold": lambda: leb.fixed_point_solve(dyn, z, v, phi, tp.e),
             "exact first sweep": exact_start,
             "bound-map net": lambda: leb.fixed_point_learned(dyn, z, v, phi, tp.e, net, sweeps=1, margin=0.0),
             "fixed-point net": lambda: leb.fixed_point_learned(dyn, z, v, phi, tp.e, net_fp, sweeps=1, margin=0.0),
             "untrained net": lambda: leb.fixed_point_learned(dyn, z, v, phi, tp.e, untrained, sweeps=1,
                                                              margin=0.0)}
    sweeps, ms = {}, {}
    for k, fn in forms.items():
        r = fn()
        torch.cuda.synchronize()
        assert bool((r[2] == 1).all()), k
        t0 = time.perf_counter()
        for _ in range(5):
            r = fn()
        torch.cuda.synchronize()
        ms[k] = (time.perf_counter() - t0) / 5 * 1e3
        sweeps[k] = r[3]
        print("%-18s certified sweeps %2d  %.3f ms" % (k, sweeps[k], ms[k]))
    untrained.close()
    assert sweeps["fixed-point net"] < sweeps["cold"]
    assert sweeps["fixed-point net"] < sweeps["untrained net"]


@pytest.mark.parametrize("batch,N,U", [(4, 12, 28), (2, 70, 3)])
def test_untrained_surrogate_still_certifies(trained, orc, batch, N, U):
    """A surrogate that predicts nonsense changes the start, not the
    certificate: the certified iteration converges from any start (also at
    70 steps, where the tube maps stage their inputs in passes)."""
    import torch
    from paper_2607_01203_amd import learned
    leb, _, dev, _ = trained
    bad = leb.Surrogate(learned.CHAIN_WIDTHS, learned.he_init(learned.CHAIN_WIDTHS, 9))
    tp = W.fixed_point_cfg(seed=50, batch=batch, N=N, n_units=U)
    b = tp.batch
    dyn = leb.dynamics_like(b.dyn)
    print("case: untrained surrogate B=%d N=%d U=%d" % (batch, N, U), flush=True)
    mu, sg, cert, sw = leb.fixed_point_learned(dyn, _t(b.z, dev), _t(b.v, dev), _t(tp.phi, dev), tp.e, bad,
                                               sweeps=3, margin=0.0)
    torch.cuda.synchronize()
    bad.close()
    assert bool((cert == 1).all())
    mo, so, _, _ = _oracle_fixed_point(orc, tp, np.arange(batch))
    assert (sg.cpu().numpy() >= so * (1 - 1e-12)).all()


def test_learned_form_without_surrogate_sweeps(trained, orc):
    """No surrogate sweeps: the start is the disturbance-only tube inflated
    by the margin, and the certified iteration runs from there to the same
    converged tube as the cold start."""
    import torch
    leb, net, dev, _ = trained
    tp = W.fixed_point_cfg(seed=51, batch=3, N=12, n_units=5)
    b = tp.batch
    dyn = leb.dynamics_like(b.dyn)
    print("case: learned form, 0 surrogate sweeps B=3 N=12 U=5", flush=True)
    mu, sg, cert, sw = leb.fixed_point_learned(dyn, _t(b.z, dev), _t(b.v, dev), _t(tp.phi, dev), tp.e, net,
                                               sweeps=0, margin=0.1)
    torch.cuda.synchronize()
    assert bool((cert == 1).all()) and 1 <= sw <= 12 + 2
    mo, so, _, _ = _oracle_fixed_point(orc, tp, np.arange(3))
    sg = sg.cpu().numpy()
    assert (sg >= so * (1 - 1e-12)).all()
    pos = so > 0
    ratio = sg[pos] / so[pos]
    print("sigma / least fixed point: median %.6f max %.6f" % (np.median(ratio), ratio.max()))
    # accepted only once converged: within the parity tolerance of the least fixed point
    assert sw >= 2 and ratio.max() <= 1 + 1e-4
