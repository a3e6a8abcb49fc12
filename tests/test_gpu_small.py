"""GPU interval-Hessian bounds of the small analytic systems (satellite,
3-D quadrotor, and the closed-form test kinds) in the three forms of
section IV.A against the FP64 oracle; Corollary 1's ordering on the GPU's
own outputs; the sampled remainder against the oracle's at the same points
and inside the GPU bound."""
import numpy as np
import pytest

import workloads as W
from parity import check_bounds

pytestmark = pytest.mark.gpu

MODES = ("path", "expand", "classic")


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


def _sys(name):
    return W.SATELLITE if name == "satellite" else W.QUAD3D


def _gpu_bound(leb, b, dev, mode, mu=None, z=None):
    import torch
    dyn = leb.dynamics_like(b.dyn)
    lo, hi, fl = leb.interval_hessian_bound(dyn, _t(b.z if z is None else z, dev), _t(b.v, dev),
                                            _t(b.sigma, dev), None if mu is None else _t(mu, dev), mode=mode)
    torch.cuda.synchronize()
    return lo.cpu().numpy(), hi.cpu().numpy(), fl.cpu().numpy()


@pytest.mark.parametrize("name", ["satellite", "quad3d"])
@pytest.mark.parametrize("eps", [0.01, 0.2])
@pytest.mark.parametrize("mode", MODES)
def test_small_parity(gpu, orc, name, eps, mode):
    import paper_2607_01203_amd as leb
    b = W.small_batch(_sys(name), 50, 300, eps)
    print("case: %s eps=%g mode=%s" % (name, eps, mode), flush=True)
    lo, hi, fl = _gpu_bound(leb, b, gpu, mode)
    d = orc.Dyn.like(b.dyn)
    olo, ohi, ofl = orc.leb(d, b.z, b.v, b.sigma, mode=mode)
    check_bounds(lo, hi, olo, ohi, "%s %s" % (name, mode))
    assert (fl == ofl.astype(np.int32)).all()


@pytest.mark.parametrize("name", ["satellite", "quad3d"])
@pytest.mark.parametrize("mode", MODES)
def test_small_offcentre_zero_radii_and_bad_input(gpu, orc, name, mode):
    import paper_2607_01203_amd as leb
    b = W.small_batch(_sys(name), 51, 40, 0.05)
    rng = np.random.default_rng(3)
    mu = rng.uniform(-0.08, 0.08, b.sigma.shape)          # some |mu| > sigma: hull with the nominal
    b.sigma[0, 5:9, :] = 0.0                               # exactly zero radii
    b.sigma[0, 10, 2] = 0.0
    b.sigma[0, 12, 3] = -1.0                               # invalid
    b.z[0, 13, 0] = np.nan
    mu[0, 5:9] = 0.0
    print("case: %s %s off-centre / zero / bad" % (name, mode), flush=True)
    lo, hi, fl = _gpu_bound(leb, b, gpu, mode, mu=mu)
    d = orc.Dyn.like(b.dyn)
    olo, ohi, ofl = orc.leb(d, b.z, b.v, b.sigma, mu=mu, mode=mode)
    check_bounds(lo, hi, olo, ohi, "%s %s" % (name, mode))
    assert (fl == ofl.astype(np.int32)).all()
    assert (lo[0, 5:9] == 0).all() and (hi[0, 5:9] == 0).all()
    assert np.isinf(lo[0, 12]).all() and np.isinf(lo[0, 13]).all()


def test_quad3d_unbounded_rows(gpu, orc):
    import paper_2607_01203_amd as leb
    b = W.small_batch(W.QUAD3D, 52, 4, 0.1)
    b.z[0, 1, 4] = np.pi / 2 - 0.05
    for mode in MODES:
        lo, hi, fl = _gpu_bound(leb, b, gpu, mode)
        d = orc.Dyn.like(b.dyn)
        olo, ohi, ofl = orc.leb(d, b.z, b.v, b.sigma, mode=mode)
        assert (fl == ofl.astype(np.int32)).all() and fl[0, 1] & leb.FLAG_UNBOUNDED
        check_bounds(lo, hi, olo, ohi, "quad3d unbounded %s" % mode)


@pytest.mark.parametrize("kind", ["quadratic", "sin1d", "sincos2d"])
@pytest.mark.parametrize("mode", ["expand", "classic"])
def test_test_kinds_expand_classic(gpu, orc, kind, mode):
    import torch
    import paper_2607_01203_amd as leb
    rng = np.random.default_rng(7)
    U = 97
    if kind == "quadratic":
        nx, nu = 5, 3
        n = nx + nu
        A = rng.normal(size=(nx, n, n))
        Q = 0.5 * (A + A.transpose(0, 2, 1))
        Q[:, 2, 1] = Q[:, 1, 2] = 0.0
        dyn = leb.quadratic_dynamics(_t(Q, gpu), nu=nu)
        d = orc.Dyn("quadratic", nx=nx, nu=nu, Q=Q)
    else:
        nx, nu = (1, 0) if kind == "sin1d" else (2, 0)
        n = nx
        dyn = leb.sincos_dynamics(nx)
        d = orc.Dyn(kind, nx=nx)
    z = rng.uniform(-2.0, 2.0, (1, U, nx))
    v = rng.uniform(-1.0, 1.0, (1, U, max(nu, 1)))[..., :nu]
    sg = rng.uniform(0.0, 0.8, (1, U, n))
    mu = rng.uniform(-0.3, 0.3, (1, U, n))
    print("case: %s %s" % (kind, mode), flush=True)
    lo, hi, fl = leb.interval_hessian_bound(dyn, _t(z, gpu), _t(v, gpu), _t(sg, gpu), _t(mu, gpu), mode=mode)
    torch.cuda.synchronize()
    olo, ohi, ofl = orc.leb(d, z, v, sg, mu=mu, mode=mode)
    check_bounds(lo.cpu().numpy(), hi.cpu().numpy(), olo, ohi, "%s %s" % (kind, mode))
    assert (fl.cpu().numpy() == ofl.astype(np.int32)).all()


@pytest.mark.parametrize("name", ["satellite", "quad3d"])
def test_corollary_1_on_gpu(gpu, name):
    import paper_2607_01203_amd as leb
    b = W.small_batch(_sys(name), 53, 500, 0.15)
    P, E, C = (_gpu_bound(leb, b, gpu, m) for m in MODES)
    for (l1, h1, _), (l2, h2, _) in ((P, E), (E, C)):
        s = np.maximum(np.abs(l2), np.abs(h2)) * 1e-6
        assert (l1 >= l2 - s).all() and (h1 <= h2 + s).all()


@pytest.mark.parametrize("name", ["satellite", "quad3d"])
def test_sampled_remainder(gpu, orc, name):
    """GPU minimum / maximum of the remainder over shared sample offsets equal
    the oracle's remainder at the same points (within its FP64 allowance),
    and lie inside the GPU path bound."""
    import torch
    import paper_2607_01203_amd as leb
    b = W.small_batch(_sys(name), 54, 64, 0.1)
    d = orc.Dyn.like(b.dyn)
    n = b.dyn.n
    K = 2000
    rng = np.random.default_rng(9)
    t = rng.uniform(-1.0, 1.0, (K, n))
    t[:8] = np.sign(t[:8])                                 # a few vertices
    dyn = leb.dynamics_like(b.dyn)
    print("case: sampled remainder %s" % name, flush=True)
    slo, shi = leb.sample_remainder(dyn, _t(b.z, gpu), _t(b.v, gpu), _t(b.sigma, gpu), _t(t, gpu))
    torch.cuda.synchronize()
    slo, shi = slo.cpu().numpy()[0], shi.cpu().numpy()[0]
    nom = np.concatenate([b.z, b.v], -1)[0]
    U = nom.shape[0]
    pts = (nom[:, None, :] + t[None] * b.sigma[0][:, None, :]).reshape(-1, n)
    uo = np.repeat(np.arange(U), K)
    r, e = orc.remainder(d, nom, pts, uo)
    r = r.reshape(U, K, d.nx)
    e = e.reshape(U, K, d.nx).max(1)
    rlo = np.minimum(r.min(1), 0.0)
    rhi = np.maximum(r.max(1), 0.0)
    assert (np.abs(slo - rlo) <= e + 1e-15).all() and (np.abs(shi - rhi) <= e + 1e-15).all()
    lo, hi, _ = _gpu_bound(leb, b, gpu, "path")
    assert (slo >= lo[0] - e).all() and (shi <= hi[0] + e).all()
