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


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2607_01203_amd as leb
    leb.lib()
    return torch.device("cuda:0")


def _chain_features_numpy(z, v, mu, sg, U, L0):
    """The 32 chain-surrogate inputs of every (unit, node), written out from
    their definition in leb.h (FP64 arithmetic, then rounded to FP32)."""
    nx = 6 * U
    B, N = z.shape[:2]
    X = np.zeros((B, N, U, 32), dtype=np.float32)
    dlo = lambda c: np.float32(np.fmin(mu[..., c] - sg[..., c], 0.0) * 20.0)
    dhi = lambda c: np.float32(np.fmax(mu[..., c] + sg[..., c], 0.0) * 20.0)
    for i in range(U):
        th, px, pz, u1, u2 = 6 * i + 2, 6 * i, 6 * i + 1, nx + 2 * i, nx + 2 * i + 1
        f = X[:, :, i]
        f[..., 0] = z[..., th]
        f[..., 1] = (v[..., 2 * i] + v[..., 2 * i + 1]) * 0.1
        for k, c in enumerate((th, u1, u2, px, pz)):
            f[..., 2 + 2 * k] = dlo(c)
            f[..., 3 + 2 * k] = dhi(c)
        for side, j in ((0, i + 1), (1, i - 1)):
            o = 12 + 7 * side
            if 0 <= j < U:
                a, b = (i, j) if side == 0 else (j, i)
                f[..., o] = 1.0
                f[..., o + 1] = (L0 + z[..., 6 * b]) - z[..., 6 * a]
                f[..., o + 2] = z[..., 6 * b + 1] - z[..., 6 * a + 1]
                f[..., o + 3], f[..., o + 4] = dlo(6 * j), dhi(6 * j)
                f[..., o + 5], f[..., o + 6] = dlo(6 * j + 1), dhi(6 * j + 1)
    return X


@pytest.mark.parametrize("with_mu", [False, True])
def test_chain_features_definition(dev, with_mu):
    """leb_chain_features against its definition (leb.h): nominal attitude
    and thrust, displacement intervals of the node's attitude, inputs and
    position, and of each spring's far node, the spring separations and
    presence flags, zeros past feature 26; the first and last nodes of the
    chain have one spring each."""
    import paper_2607_01203_amd as leb
    b = W.chain_batch(71, 3, 5, 6)
    r = np.random.default_rng(8)
    mu = r.uniform(-1.5, 1.5, b.sigma.shape) * b.sigma if with_mu else np.zeros_like(b.sigma)
    dyn = leb.dynamics_like(b.dyn)
    print("case: chain features, mu=%s" % with_mu, flush=True)
    x = leb.chain_features(dyn, _t(b.z, dev), _t(b.v, dev), _t(b.sigma, dev),
                           mu=_t(mu, dev) if with_mu else None).cpu().numpy()
    want = _chain_features_numpy(b.z, b.v, mu, b.sigma, 6, b.dyn.rest_len)
    assert x.shape == (3, 5, 6, 32)
    np.testing.assert_array_equal(x, want)
    assert (x[:, :, 0, 19] == 0).all() and (x[:, :, -1, 12] == 0).all()     # chain ends


def test_chain_targets_definition(dev):
    """leb_chain_targets against its definition: log(max(hi, 1e-14)) and
    log(max(-lo, 1e-14)) of rows 3 (vx) and 4 (vz) of every node, in FP32."""
    import paper_2607_01203_amd as leb
    rng = np.random.default_rng(4)
    U = 5
    hi = rng.exponential(1e-3, (2, 3, 6 * U))
    lo = -rng.exponential(1e-3, (2, 3, 6 * U))
    hi[0, 0, 3], lo[0, 0, 3] = 0.0, -0.0
    hi[0, 0, 9], lo[0, 0, 10] = 1e-20, -2.5
    dyn = leb.chain_dynamics(U)
    print("case: chain targets", flush=True)
    t = leb.chain_targets(dyn, _t(lo, dev), _t(hi, dev)).cpu().numpy()
    f = np.float32(1e-14)
    L = lambda a: np.log(np.maximum(a.astype(np.float32), f))
    want = np.stack([L(hi[..., 3::6]), L(-lo[..., 3::6]), L(hi[..., 4::6]), L(-lo[..., 4::6])], -1)
    np.testing.assert_allclose(t, want, rtol=1e-6, atol=1e-6)


def test_learned_boxes_sound_1e6(trained, trained_fp, orc):
    """The bound on every accepted box of the learned form (fixed-point-target
    network, 256 x 40 x 168) contains 10^6 sampled true remainders."""
    import torch
    from parity import sampled_violations
    leb, _, dev, _ = trained
    net_fp, _ = trained_fp
    tp = W.fixed_point_cfg(seed=4, batch=256, N=40)
    b = tp.batch
    dyn = leb.dynamics_like(b.dyn)
    z, v, phi = _t(b.z, dev), _t(b.v, dev), _t(tp.phi, dev)
    print("case: learned boxes, 10^6 samples", flush=True)
    mu, sg, cert, _ = leb.fixed_point_learned(dyn, z, v, phi, tp.e, net_fp, sweeps=1, margin=0.0)
    out = leb.analytic_bound(dyn, z, v, sg, mu)
    torch.cuda.synchronize()
    assert bool((cert == 1).all())
    lo = out["r_lo"].cpu().numpy().reshape(-1, 168)
    hi = out["r_hi"].cpu().numpy().reshape(-1, 168)
    d = orc.Dyn.like(b.dyn)
    nom = np.concatenate([b.z, b.v], -1).reshape(-1, 224)
    blo, bhi = orc.box(nom, sg.cpu().numpy().reshape(-1, 224), mu.cpu().numpy().reshape(-1, 224))
    per = 1_000_000 // nom.shape[0] + 1

    def rem(nm, pts):
        U, P, n = pts.shape
        r, eps = orc.remainder(d, nm, pts.reshape(-1, n), np.repeat(np.arange(U), P))
        return r.reshape(U, P, -1), eps.reshape(U, P, -1)

    viol, count = sampled_violations(rem, nom, blo, bhi, lo, hi, per, seed=1_000_004, chunk=256)
    print("samples %d violations %d" % (count, viol))
    assert count >= 1_000_000 and viol == 0
