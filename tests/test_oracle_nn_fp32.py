"""Pins of the FP32-rounding study of the CROWN chain (oracle/nn_fp32.py):
the rounding bound it charges holds for an emulated FP32 product with FP64
chunk sums, the widening shrinks with the chunk length, and with
Jacobian-deviation coefficients it vanishes on a box with no unstable
neuron (the relaxation then equals the nominal mask)."""
import numpy as np

import workloads as W
from oracle import nn_fp32 as F


def test_chunked_product_error_within_gamma():
    rng = np.random.default_rng(0)
    for K in (4, 16, 256):
        A = rng.normal(size=(16, 256)) * np.exp(rng.uniform(-3, 3, (16, 256)))
        B = rng.normal(size=(256, 32)).astype(np.float32).astype(np.float64)   # FP32 weights, exact
        P = F.fp32_chunked_product(A, B, K)
        err = np.abs(P - A @ B)
        bound = F.gamma(K + 1) * (np.abs(A) @ np.abs(B))
        # the FP64 reference product and the chunk sums add a few 2^-53 on top
        assert (err <= bound * (1 + 1e-6) + 1e-15 * (np.abs(A) @ np.abs(B))).all(), K
        assert err.max() > 0


def test_widening_shrinks_with_chunk_length_and_vanishes_on_stable_boxes():
    b = W.nn_cfg()
    rng = np.random.default_rng(2)
    a = rng.uniform(-1, 1, (3, 16))
    s = rng.uniform(0.01, 0.03, (3, 16))
    w4, _ = F.output_chain_widening(b.net.W, b.net.b, a, s, 4)
    w16, _ = F.output_chain_widening(b.net.W, b.net.b, a, s, 16)
    w256, _ = F.output_chain_widening(b.net.W, b.net.b, a, s, 256)
    assert (w4 <= w16).all() and (w16 <= w256).all() and (w4 > 0).all()
    n4, _ = F.output_chain_widening(b.net.W, b.net.b, a, s, 4, jac_dev=False)
    assert (w4 <= n4).all()
    # no unstable neuron: Lambda . S = M . D at every step
    tiny = np.full((3, 16), 1e-9)
    wu, wl = F.output_chain_widening(b.net.W, b.net.b, a, tiny, 16)
    assert (wu == 0).all() and (wl == 0).all()


def test_study_reports_every_variant():
    b = W.nn_cfg()
    rng = np.random.default_rng(3)
    r = F.study(b.net.W, b.net.b, rng.uniform(-1, 1, (2, 16)), rng.uniform(0.005, 0.05, (2, 16)), Ks=(4, 16))
    assert set(r) == {(4, False), (4, True), (16, False), (16, True)}
    assert all(v.shape == (2,) and (v >= 0).all() for v in r.values())
