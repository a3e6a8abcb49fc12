"""GPU adjoint of the MLP bound (leb_nn_backward) against the oracle's
forward-mode gradient: several widths and depths (narrow and non-power-of-two
layers, one hidden layer without control inputs, the MFMA and VALU forms),
with and without mu, ragged chunks,
the 16-256-256-256-12 workload on sampled boxes, invalid boxes, determinism."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

# FP64 on both sides, sums in different orders: 1e-9 of the box's largest
# gradient entry (plus 1e-12 absolute for all-zero boxes)
RTOL = 1e-9


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


def _gpu_grad(leb, net, z, v, sg, mu, g_lo, g_hi, dev):
    import torch
    mlp = leb.MLP(net.W, net.b, net.nx, True)
    out = leb.nn_backward(mlp, _t(z, dev), _t(v, dev), _t(sg, dev), _t(g_lo, dev), _t(g_hi, dev),
                          mu=None if mu is None else _t(mu, dev))
    torch.cuda.synchronize()
    res = {k: x.cpu().numpy() for k, x in out.items()}
    mlp.close()
    return res


def _check_box(net, g, b, k, z, v, sg, mu, g_lo, g_hi, tag):
    from oracle import nn_grad
    a = np.concatenate([z[b, k], v[b, k]])
    ga, gs, gm = nn_grad.leb_grad([np.asarray(w, np.float64) for w in net.W],
                                  [np.asarray(x, np.float64) for x in net.b], a, sg[b, k],
                                  None if mu is None else mu[b, k], g_lo[b, k], g_hi[b, k])
    got_a = np.concatenate([g["gz"][b, k], g["gv"][b, k]])
    scale = max(np.abs(ga).max(), np.abs(gs).max(), np.abs(gm).max())
    tol = RTOL * scale + 1e-12
    err = max(np.abs(got_a - ga).max(), np.abs(g["gsigma"][b, k] - gs).max())
    if mu is not None:
        err = max(err, np.abs(g["gmu"][b, k] - gm).max())
    assert err <= tol, "%s box (%d, %d): err %.3e scale %.3e" % (tag, b, k, err, scale)
    return err / max(scale, 1e-300)


def _case(rng, widths, nx, batch, N, sg_lo, sg_hi, with_mu):
    Wl, bl = W.mlp_weights(rng, widths)
    net = W.MLPNet(Wl, bl, nx, widths[0] - nx, True)
    a = rng.uniform(-1, 1, (batch, N, widths[0]))
    sg = rng.uniform(sg_lo, sg_hi, (batch, N, widths[0]))
    mu = sg * rng.uniform(-1.5, 1.5, sg.shape) if with_mu else None
    m = widths[-1]
    g_lo, g_hi = rng.normal(0, 1, (batch, N, m)), rng.normal(0, 1, (batch, N, m))
    return net, a[..., :nx].copy(), a[..., nx:].copy(), sg, mu, g_lo, g_hi


@pytest.mark.parametrize("widths,nx,with_mu", [([16, 32, 32, 12], 12, False), ([16, 64, 48, 32, 8], 8, True),
                                               ([32, 16, 16, 16, 16, 16, 4], 4, True),
                                               ([16, 256, 96, 12], 12, False), ([16, 48, 16], 16, True)])
def test_nn_backward_parity_shapes(gpu, widths, nx, with_mu):
    import paper_2607_01203_amd as leb
    rng = W.rng_for(300 + len(widths) + widths[1])
    net, z, v, sg, mu, g_lo, g_hi = _case(rng, widths, nx, 2, 3, 0.05, 0.4, with_mu)
    print("case: nn backward widths %s mu %s" % (widths, with_mu), flush=True)
    g = _gpu_grad(leb, net, z, v, sg, mu, g_lo, g_hi, gpu)
    worst = max(_check_box(net, g, b, k, z, v, sg, mu, g_lo, g_hi, str(widths)) for b in range(2) for k in range(3))
    print("worst relative error %.2e" % worst)
    assert np.abs(g["gsigma"]).max() > 0


def test_nn_backward_ragged_chunks(gpu):
    """4,200 boxes: two chunks of the workspace (4,096 boxes each at most),
    the second ragged."""
    import paper_2607_01203_amd as leb
    rng = W.rng_for(311)
    net, z, v, sg, mu, g_lo, g_hi = _case(rng, [16, 32, 32, 12], 12, 1, 4200, 0.05, 0.4, True)
    print("case: nn backward 4200 boxes", flush=True)
    g = _gpu_grad(leb, net, z, v, sg, mu, g_lo, g_hi, gpu)
    for k in (0, 1, 4095, 4096, 4097, 4199):
        _check_box(net, g, 0, k, z, v, sg, mu, g_lo, g_hi, "ragged")


def test_nn_backward_full_workload_sampled(gpu):
    """The MLP-bound workload (64 x 50 boxes of a 16-256-256-256-12 network),
    with seeds g_lo = -1, g_hi = 1 (the gradient of the bound's total width)."""
    import paper_2607_01203_amd as leb
    b = W.nn_cfg()
    g_hi = np.ones((64, 50, 12))
    g_lo = -g_hi
    print("case: nn backward 64x50 workload", flush=True)
    g = _gpu_grad(leb, b.net, b.z, b.v, b.sigma, None, g_lo, g_hi, gpu)
    for bt, kt in ((0, 0), (17, 23), (63, 49)):
        _check_box(b.net, g, bt, kt, b.z, b.v, b.sigma, None, g_lo, g_hi, "workload")
    # the width grows with the radii
    assert (g["gsigma"] >= 0).mean() > 0.9


def test_nn_backward_invalid_boxes_and_determinism(gpu):
    import torch
    import paper_2607_01203_amd as leb
    rng = W.rng_for(321)
    net, z, v, sg, mu, g_lo, g_hi = _case(rng, [16, 32, 32, 12], 12, 1, 6, 0.05, 0.4, True)
    z[0, 1, 3] = np.nan
    sg[0, 2, 0] = -1.0
    mu[0, 4, 5] = np.inf
    print("case: nn backward invalid boxes", flush=True)
    g1 = _gpu_grad(leb, net, z, v, sg, mu, g_lo, g_hi, gpu)
    g2 = _gpu_grad(leb, net, z, v, sg, mu, g_lo, g_hi, gpu)
    for k in (1, 2, 4):
        for key in ("gz", "gv", "gsigma", "gmu"):
            assert (g1[key][0, k] == 0).all(), (key, k)
    for k in (0, 3, 5):
        _check_box(net, g1, 0, k, z, v, sg, mu, g_lo, g_hi, "valid next to invalid")
    for key in g1:
        assert np.array_equal(g1[key], g2[key])
    # gmu without mu is refused
    mlp = leb.MLP(net.W, net.b, net.nx, True)
    tz, tv, ts, tl, th = (_t(x, gpu) for x in (z, v, sg, g_lo, g_hi))
    oz, ov, os_, om = torch.empty_like(tz), torch.empty_like(tv), torch.empty_like(ts), torch.empty_like(ts)
    rc = leb.lib().leb_nn_backward(mlp.handle, 1, 6, tz.data_ptr(), tv.data_ptr(), None, ts.data_ptr(),
                                   tl.data_ptr(), th.data_ptr(), oz.data_ptr(), ov.data_ptr(), om.data_ptr(),
                                   os_.data_ptr(), None)
    assert rc == -1
    torch.cuda.synchronize()
    mlp.close()


def test_nn_autograd_function(gpu):
    """leb_nn: torch autograd through the MLP bound equals the direct adjoint."""
    import torch
    import paper_2607_01203_amd as leb
    rng = W.rng_for(331)
    net, z, v, sg, mu, g_lo, g_hi = _case(rng, [16, 64, 64, 12], 12, 2, 4, 0.05, 0.3, True)
    mlp = leb.MLP(net.W, net.b, net.nx, True)
    tz, tv, ts, tm = (_t(x, gpu).requires_grad_(True) for x in (z, v, sg, mu))
    print("case: nn autograd", flush=True)
    lo, hi = leb.leb_nn(mlp, tz, tv, ts, tm)
    gl, gh = _t(g_lo, gpu), _t(g_hi, gpu)
    (gl * lo + gh * hi).sum().backward()
    g = leb.nn_backward(mlp, tz.detach(), tv.detach(), ts.detach(), gl, gh, mu=tm.detach())
    torch.cuda.synchronize()
    assert torch.equal(tz.grad, g["gz"]) and torch.equal(tv.grad, g["gv"])
    assert torch.equal(ts.grad, g["gsigma"]) and torch.equal(tm.grad, g["gmu"])
    mlp.close()


@pytest.mark.parametrize("case", ["layer1_inactive", "tiny_box", "wide_box"])
def test_nn_backward_edge_boxes(gpu, case):
    """Neuron lists at their extremes: a first hidden layer stably inactive
    on every box (empty list: the bound and its gradient are 0), boxes so
    small that every neuron is stable (gradient 0), and boxes so wide that
    nearly every neuron is unstable."""
    import paper_2607_01203_amd as leb
    rng = W.rng_for(341)
    sg_lo, sg_hi = {"layer1_inactive": (0.05, 0.4), "tiny_box": (1e-9, 2e-9), "wide_box": (2.0, 3.0)}[case]
    net, z, v, sg, mu, g_lo, g_hi = _case(rng, [16, 64, 48, 12], 12, 2, 3, sg_lo, sg_hi, True)
    if case == "layer1_inactive":
        net.b[0][:] = np.float32(-100.0)
    print("case: nn backward edge %s" % case, flush=True)
    g = _gpu_grad(leb, net, z, v, sg, mu, g_lo, g_hi, gpu)
    for b in range(2):
        for k in range(3):
            _check_box(net, g, b, k, z, v, sg, mu, g_lo, g_hi, case)
    if case != "wide_box":
        for key in g:
            assert np.abs(g[key]).max() <= 1e-12, key
