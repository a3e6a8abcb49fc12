"""GPU adjoint of the path-based bound (leb_backward) against the oracle's
forward-mode gradient, central differences of the oracle bound, and the
torch.autograd wrapper."""
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


def _gpu_grad(leb, b, dev, gl, gh, mu=None):
    import torch
    dyn = leb.dynamics_like(b.dyn)
    gz, gv, gs, gm = leb.backward(dyn, _t(b.z, dev), _t(b.v, dev), _t(b.sigma, dev), _t(gl, dev), _t(gh, dev),
                                  None if mu is None else _t(mu, dev))
    torch.cuda.synchronize()
    return {"gz": gz.cpu().numpy(), "gv": gv.cpu().numpy(), "gsigma": gs.cpu().numpy(),
            "gmu": None if gm is None else gm.cpu().numpy()}


def _compare(g, o, units_ok, keys):
    """|g - o| <= 1e-4 max(|o|, scale) with scale = max |o| of the unit and kind."""
    worst = 0.0
    for k in keys:
        a = g[k].reshape(-1, g[k].shape[-1])[units_ok]
        e = o[k].reshape(-1, o[k].shape[-1])[units_ok]
        scale = np.abs(e).max(axis=1, keepdims=True)
        den = np.maximum(np.abs(e), np.maximum(scale, 1e-300))
        err = (np.abs(a - e) / den).max(initial=0.0)
        worst = max(worst, err)
        assert err <= 1e-4, (k, err)
    return worst


@pytest.mark.parametrize("n_units,batch,N,offc", [(1, 2, 25, False), (1, 1, 20, True), (4, 2, 7, False),
                                                  (4, 1, 9, True), (28, 1, 6, False), (9, 3, 5, True)])
def test_backward_matches_oracle_gradient(gpu, orc, n_units, batch, N, offc):
    import paper_2607_01203_amd as leb
    b = W.chain_batch(400 + n_units, batch, N, n_units)
    r = np.random.default_rng(n_units)
    gl = r.normal(size=b.z.shape)
    gh = r.normal(size=b.z.shape)
    mu = r.uniform(-0.02, 0.02, b.sigma.shape) if offc else None
    print("case: backward U=%d batch=%d N=%d offcentre=%s" % (n_units, batch, N, offc), flush=True)
    g = _gpu_grad(leb, b, gpu, gl, gh, mu)
    d = orc.Dyn.like(b.dyn)
    o = orc.leb_grad(d, b.z, b.v, b.sigma, gl, gh, mu=mu)
    ok = o["margin"].reshape(-1) > 1e-5
    assert ok.sum() >= 0.5 * ok.size
    keys = ["gz", "gv", "gsigma"] + (["gmu"] if offc else [])
    print("worst", _compare(g, o, ok, keys))


def test_backward_chain168_and_finite_differences(gpu, orc):
    """The adjoint at the 28-node, 40-step shape against the oracle gradient
    (every unit clear of kinks) and central differences of the oracle bound
    at three units spread over the horizon."""
    import paper_2607_01203_amd as leb
    b = W.chain_cfg(N=40)
    r = np.random.default_rng(7)
    gl = r.normal(size=b.z.shape)
    gh = r.normal(size=b.z.shape)
    print("case: backward chain 168", flush=True)
    g = _gpu_grad(leb, b, gpu, gl, gh)
    d = orc.Dyn.like(b.dyn)
    o = orc.leb_grad(d, b.z, b.v, b.sigma, gl, gh)
    ok = o["margin"].reshape(-1) > 1e-5
    _compare(g, o, ok, ["gz", "gv", "gsigma"])
    # central differences (h = 1e-6) of the oracle bound against the GPU gradient
    h = 1e-6
    okt = np.nonzero(ok)[0]
    assert len(okt) >= 20
    for t in (int(okt[0]), int(okt[len(okt) // 2]), int(okt[-1])):
        _fd_at(orc, d, b, gl, gh, g, t, h)


def _fd_at(orc, d, b, gl, gh, g, t, h):
    def L(z, v, s):
        lo, hi, _ = orc.leb(d, z[:, t:t + 1], v[:, t:t + 1], s[:, t:t + 1])
        return float((gl[:, t:t + 1] * lo + gh[:, t:t + 1] * hi).sum())

    for name, arr, key, idx in [("z", b.z, "gz", 2), ("z", b.z, "gz", 6), ("z", b.z, "gz", 13),
                                ("v", b.v, "gv", 0), ("s", b.sigma, "gsigma", 1), ("s", b.sigma, "gsigma", 8),
                                ("s", b.sigma, "gsigma", 170)]:
        p = {"z": b.z.copy(), "v": b.v.copy(), "s": b.sigma.copy()}
        m = {"z": b.z.copy(), "v": b.v.copy(), "s": b.sigma.copy()}
        p[name][0, t, idx] += h
        m[name][0, t, idx] -= h
        fd = (L(p["z"], p["v"], p["s"]) - L(m["z"], m["v"], m["s"])) / (2 * h)
        an = g[key][0, t, idx]
        assert abs(fd - an) <= 1e-4 * max(abs(fd), 1e-3 * np.abs(g[key][0, t]).max()) + 1e-9, (name, idx, fd, an)


def test_autograd_function_and_determinism(gpu):
    import torch
    import paper_2607_01203_amd as leb
    b = W.chain_batch(11, 2, 5, 3)
    dyn = leb.dynamics_like(b.dyn)
    z = _t(b.z, gpu).requires_grad_(True)
    v = _t(b.v, gpu).requires_grad_(True)
    s = _t(b.sigma, gpu).requires_grad_(True)
    lo, hi = leb.leb_analytic(dyn, z, v, s)
    r = np.random.default_rng(1)
    gl = _t(r.normal(size=b.z.shape), gpu)
    gh = _t(r.normal(size=b.z.shape), gpu)
    (gl * lo + gh * hi).sum().backward()
    gz, gv, gs, _ = leb.backward(dyn, z.detach(), v.detach(), s.detach(), gl, gh)
    gz2, gv2, gs2, _ = leb.backward(dyn, z.detach(), v.detach(), s.detach(), gl, gh)
    torch.cuda.synchronize()
    assert torch.equal(z.grad, gz) and torch.equal(v.grad, gv) and torch.equal(s.grad, gs)
    assert torch.equal(gz, gz2) and torch.equal(gs, gs2)


def test_backward_rejects_mu_gradient_without_mu(gpu):
    import torch
    import paper_2607_01203_amd as leb
    b = W.chain_batch(12, 1, 2, 2)
    dyn = leb.dynamics_like(b.dyn)
    z, v, s = _t(b.z, gpu), _t(b.v, gpu), _t(b.sigma, gpu)
    g = torch.zeros_like(z)
    with pytest.raises(leb.LebError):
        out = torch.empty_like(s)
        rc = leb.lib().leb_backward(__import__("ctypes").byref(dyn), 1, 2, leb._dev_ptr(z, "z"), leb._dev_ptr(v, "v"),
                                    None, leb._dev_ptr(s, "s"), leb._dev_ptr(g, "g"), leb._dev_ptr(g, "g"),
                                    leb._dev_ptr(torch.empty_like(z), "a"), leb._dev_ptr(torch.empty_like(v), "b"),
                                    leb._dev_ptr(out, "c"), leb._dev_ptr(torch.empty_like(s), "d"), None)
        leb._check(rc)
