"""GPU BF16 MFMA kernels of the warm-start MLP against the MLP oracle
(FP64 with BF16 rounding at the same points): forward, backward, Adam and
the fused training step.

Tolerance: the kernels accumulate in FP32 (relative error of a sum of K
terms at most about K 2^-24 of the sum of magnitudes) and may round an
activation to the neighbouring BF16 value where the FP32 and FP64 values
straddle a rounding midpoint (a change of 2^-8 in one of K terms).  Per
tensor: max |gpu - oracle| <= 4e-3 max |oracle|, and the median relative
error over entries above 1% of the tensor's scale is below 1e-4."""
import numpy as np
import pytest

from oracle import mlp

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
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)


def _close(g, o, what, max_rel=4e-3, med_rel=1e-4):
    g = np.asarray(g, dtype=np.float64)
    o = np.asarray(o, dtype=np.float64)
    scale = np.abs(o).max()
    assert np.isfinite(g).all(), what
    err = np.abs(g - o)
    assert err.max() <= max_rel * scale + 1e-30, (what, err.max() / max(scale, 1e-300))
    big = np.abs(o) > 0.01 * scale
    if big.sum() >= 10:
        med = np.median(err[big] / np.abs(o[big]))
        assert med <= med_rel, (what, med)
    return err.max() / max(scale, 1e-300)


def _net(seed, widths, bias_scale=0.1):
    rng = np.random.default_rng(seed)
    p = mlp.init_params(rng, widths).astype(np.float64)
    W, b = mlp.unpack(p, widths)
    b = [rng.uniform(-bias_scale, bias_scale, x.shape) for x in b]
    return mlp.pack(W, b).astype(np.float32), rng


@pytest.mark.parametrize("widths,B", [([26, 128, 128, 128, 4], 200), ([32, 128, 128, 128, 24], 64),
                                      ([5, 40, 17, 3], 37), ([16, 256, 256, 12], 130)])
def test_forward_matches_oracle(gpu, widths, B):
    import torch
    import paper_2607_01203_amd as leb
    p, rng = _net(widths[0] + B, widths)
    x = rng.normal(size=(B, widths[0])).astype(np.float32)
    print("case: mlp forward widths %s B=%d" % (widths, B), flush=True)
    s = leb.Surrogate(widths, p)
    y = s.forward(_t(x, gpu))
    torch.cuda.synchronize()
    yo, _ = mlp.forward(p, widths, x)
    print("rel", _close(y.cpu().numpy(), yo, "y"))
    np.testing.assert_array_equal(s.params(), p)
    s.close()


def _grad_parts(flat, widths):
    W, b = mlp.unpack(flat, widths)
    return [(f"W{l}", w) for l, w in enumerate(W)] + [(f"b{l}", x) for l, x in enumerate(b)]


@pytest.mark.parametrize("widths,B", [([26, 128, 128, 128, 4], 256), ([32, 128, 128, 128, 24], 96),
                                      ([5, 40, 17, 3], 32)])
def test_backward_matches_oracle(gpu, widths, B):
    import torch
    import paper_2607_01203_amd as leb
    p, rng = _net(7 + B, widths)
    x = rng.normal(size=(B, widths[0])).astype(np.float32)
    dy = (rng.normal(size=(B, widths[-1])) / B).astype(np.float32)
    print("case: mlp backward widths %s B=%d" % (widths, B), flush=True)
    s = leb.Surrogate(widths, p)
    g = s.backward(_t(x, gpu), _t(dy, gpu))
    torch.cuda.synchronize()
    go = mlp.backward(p, widths, x, dy.astype(np.float64))
    for (name, a), (_, e) in zip(_grad_parts(g.cpu().numpy(), widths), _grad_parts(go, widths)):
        _close(a, e, name)
    s.close()


def test_adam_matches_oracle(gpu):
    import torch
    import paper_2607_01203_amd as leb
    widths = [26, 128, 128, 128, 4]
    p, rng = _net(11, widths)
    s = leb.Surrogate(widths, p)
    po = p.astype(np.float64)
    m = np.zeros_like(po)
    v = np.zeros_like(po)
    for step in range(1, 4):
        g = (rng.normal(size=p.size) * 10.0 ** rng.uniform(-6, 0, p.size)).astype(np.float32)
        s.adam(_t(g, gpu), step, 1e-3)
        po, m, v = mlp.adam(po, g.astype(np.float64), m, v, step, 1e-3)
    torch.cuda.synchronize()
    got = s.params().astype(np.float64)
    # FP32 arithmetic on FP32 parameters: a few ulps of the update and of p
    np.testing.assert_allclose(got, po, rtol=2e-6, atol=1e-9)
    s.close()


def test_train_step_is_forward_backward_adam(gpu):
    """The fused step equals MSE gradient + backward + Adam of the oracle,
    and reports the pre-update loss."""
    import torch
    import paper_2607_01203_amd as leb
    widths = [26, 128, 128, 128, 4]
    p, rng = _net(12, widths)
    B = 128
    x = rng.normal(size=(B, 26)).astype(np.float32)
    t = rng.normal(size=(B, 4)).astype(np.float32)
    s = leb.Surrogate(widths, p)
    loss = torch.zeros(1, dtype=torch.float32, device=gpu)
    s.train_step(_t(x, gpu), _t(t, gpu), 1, 1e-3, loss)
    torch.cuda.synchronize()
    yo, _ = mlp.forward(p, widths, x)
    lo, dy = mlp.mse(yo, t.astype(np.float64))
    assert abs(loss.item() - lo) <= 1e-4 * lo
    go = mlp.backward(p, widths, x, dy)
    po, _, _ = mlp.adam(p.astype(np.float64), go, np.zeros(p.size), np.zeros(p.size), 1, 1e-3)
    got = s.params().astype(np.float64)
    # the first Adam step moves every parameter with a non-negligible
    # gradient by about lr sign(g): compare the moves
    moved = np.abs(go) > 1e-3 * np.abs(go).max()
    d_g = got - p
    d_o = po - p
    assert (np.sign(d_g[moved]) == np.sign(d_o[moved])).mean() > 0.999
    np.testing.assert_allclose(d_g[moved], d_o[moved], rtol=2e-2, atol=1e-6)
    s.close()


def test_training_fits_a_smooth_map(gpu):
    import torch
    import paper_2607_01203_amd as leb
    widths = [8, 128, 128, 128, 2]
    p, rng = _net(13, widths, 0.0)
    B = 512
    x = rng.uniform(-1, 1, (4096, 8)).astype(np.float32)
    t = np.stack([np.sin(2 * x[:, 0]) * x[:, 1], x[:, 2] * x[:, 3] - 0.5 * x[:, 4] ** 2], 1).astype(np.float32)
    X, T = _t(x, gpu), _t(t, gpu)
    s = leb.Surrogate(widths, p)
    loss = torch.zeros(1, dtype=torch.float32, device=gpu)
    losses = []
    step = 0
    for ep in range(30):
        for i in range(0, 4096, B):
            step += 1
            s.train_step(X[i:i + B], T[i:i + B], step, 2e-3, loss)
        losses.append(loss.item())
    print("loss", losses[0], losses[-1])
    assert losses[-1] < 0.05 * losses[0]
    y = s.forward(X).cpu().numpy()
    yo, _ = mlp.forward(s.params(), widths, x)
    _close(y, yo, "trained forward")
    s.close()


def test_rejects_bad_shapes(gpu):
    import torch
    import paper_2607_01203_amd as leb
    widths = [4, 32, 2]
    p, _ = _net(14, widths)
    with pytest.raises(leb.LebError):
        leb.Surrogate([4, 300, 2], np.zeros(4 * 300 + 300 + 600 + 2, dtype=np.float32))
    with pytest.raises(leb.LebError):
        leb.Surrogate(widths, p[:-1])
    s = leb.Surrogate(widths, p)
    x = torch.zeros((33, 4), dtype=torch.float32, device=gpu)
    with pytest.raises(leb.LebError):
        s.backward(x, torch.zeros((33, 2), dtype=torch.float32, device=gpu))   # batch not a multiple of 32
    y = s.forward(x[:0])
    assert y.shape == (0, 2)
    s.close()
