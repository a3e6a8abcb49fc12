"""Pins of the warm-start MLP oracle: BF16 rounding at known values, GELU
closed forms and derivative, backward pass against FP64 central
differences of the smooth (exact=True) network, the BF16 path's backward
against the exact one, and Adam against its closed form for a constant
gradient."""
import math

import numpy as np
import pytest

from oracle import mlp

pytest.importorskip("scipy.special")


def test_bf16_rounding_known_values():
    v = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -9, 1.0 + 2.0 ** -7 + 2.0 ** -8, -2.5, 0.0,
                  65504.0, 1.0 + 2.0 ** -8 + 2.0 ** -20, 3.0e38, 1e-40])
    want = np.array([1.0, 1.0, 1.0 + 2.0 ** -7, 1.0 + 2.0 ** -6, -2.5, 0.0,
                     65536.0, 1.0 + 2.0 ** -7, 2.9983e38, None], dtype=object)
    got = mlp.bf16(v)
    for g, w in zip(got[:8], want[:8]):
        assert g == w, (g, w)
    # 3e38 -> nearest bf16 (8 significant bits) keeps the exponent
    assert abs(got[8] / 3.0e38 - 1) < 2.0 ** -8
    # FP32 subnormals keep the top 16 bits of the FP32 field: spacing 2^-133 here
    assert got[9] == 2.0 ** -133
    # every output has at most 8 significant bits
    r = np.random.default_rng(0).normal(size=1000) * 10.0 ** np.random.default_rng(1).integers(-20, 20, 1000)
    b = mlp.bf16(r)
    u = b.astype(np.float32).view(np.uint32)
    assert (u & 0xFFFF == 0).all()
    assert (np.abs(b - r) <= np.abs(r) * 2.0 ** -8).all()


def test_gelu_closed_forms_and_derivative():
    assert mlp.gelu(0.0) == 0.0
    x = np.linspace(-6, 6, 241)
    # gelu(x) - gelu(-x) = x, since Phi(x) + Phi(-x) = 1
    np.testing.assert_allclose(mlp.gelu(x) - mlp.gelu(-x), x, atol=1e-14)
    # gelu(1) = Phi(1) = 0.841344746068543 (normal table value)
    assert abs(mlp.gelu(1.0) - 0.8413447460685429) < 1e-15
    assert abs(mlp.gelu_grad(0.0) - 0.5) < 1e-16
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    np.testing.assert_allclose(mlp.gelu_grad(x), fd, atol=1e-8)


def _small():
    rng = np.random.default_rng(3)
    widths = [5, 7, 6, 4, 3]
    p = mlp.init_params(rng, widths).astype(np.float64)
    p += rng.normal(0, 0.05, p.size)          # non-zero biases
    x = rng.normal(size=(9, 5))
    t = rng.normal(size=(9, 3))
    return widths, p, x, t


def test_backward_matches_central_differences_exact():
    widths, p, x, t = _small()

    def loss(q):
        y, _ = mlp.forward(q, widths, x, exact=True)
        return mlp.mse(y, t)[0]

    y, _ = mlp.forward(p, widths, x, exact=True)
    _, dy = mlp.mse(y, t)
    g = mlp.backward(p, widths, x, dy, exact=True)
    h = 1e-6
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        fd = (loss(p + e) - loss(p - e)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(fd)), (i, fd, g[i])


def test_bf16_path_close_to_exact_path():
    """The BF16 network differs from the exact one by BF16 rounding only:
    relative differences of a few 2^-8 units, never structural."""
    widths, p, x, t = _small()
    y0, _ = mlp.forward(p, widths, x, exact=True)
    y1, _ = mlp.forward(p, widths, x)
    assert np.abs(y1 - y0).max() <= 2.0 ** -5 * np.abs(y0).max()
    _, dy = mlp.mse(y0, t)
    g0 = mlp.backward(p, widths, x, dy, exact=True)
    g1 = mlp.backward(p, widths, x, dy)
    assert np.linalg.norm(g1 - g0) <= 2.0 ** -4 * np.linalg.norm(g0)
    assert not np.array_equal(g1, g0)


def test_pack_unpack_layout():
    widths = [2, 3, 1]
    p = np.arange(mlp.n_params(widths), dtype=np.float64)
    W, b = mlp.unpack(p, widths)
    assert W[0].tolist() == [[0, 1], [2, 3], [4, 5]] and b[0].tolist() == [6, 7, 8]
    assert W[1].tolist() == [[9, 10, 11]] and b[1].tolist() == [12]
    np.testing.assert_array_equal(mlp.pack(W, b), p)


def test_adam_constant_gradient_closed_form():
    """With a constant gradient g, m_hat = g and v_hat = g^2 at every step,
    so each step moves by lr g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3])
    p = np.zeros(3)
    m = np.zeros(3)
    v = np.zeros(3)
    for step in range(1, 6):
        p, m, v = mlp.adam(p, g, m, v, step, lr=0.01)
    np.testing.assert_allclose(p, -5 * 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    # first step of Adam: m = 0.1 g, v = 0.001 g^2
    p1, m1, v1 = mlp.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=1.0)
    np.testing.assert_allclose(m1, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v1, 0.001 * g * g, rtol=1e-14)


def test_training_reduces_loss():
    """A few hundred exact-path Adam steps fit a smooth target."""
    rng = np.random.default_rng(5)
    widths = [2, 16, 16, 16, 1]
    p = mlp.init_params(rng, widths).astype(np.float64)
    x = rng.uniform(-1, 1, (64, 2))
    t = (np.sin(2 * x[:, :1]) * x[:, 1:]) * 0.5
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    y, _ = mlp.forward(p, widths, x)
    l0 = mlp.mse(y, t)[0]
    for step in range(1, 301):
        y, _ = mlp.forward(p, widths, x)
        _, dy = mlp.mse(y, t)
        p, m, v = mlp.adam(p, mlp.backward(p, widths, x, dy), m, v, step, lr=3e-3)
    y, _ = mlp.forward(p, widths, x)
    assert mlp.mse(y, t)[0] < 0.05 * l0
    assert math.isfinite(l0)
