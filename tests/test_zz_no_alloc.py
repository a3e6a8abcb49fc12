"""The no-allocation fixed point (leb_fixed_point_solve_noalloc, through the
C ABI) against leb_fixed_point_solve: the same tube, centre and certificate
flags, bit for bit, on two calls in a row (the second smaller, so it reuses
the static scratch the first left behind), at a sweep cap that leaves the
trajectories uncertified, and the scratch limit refused before any launch."""
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


def _both(leb, tp, dev, max_sweeps=20):
    import torch
    b = tp.batch
    dyn = leb.dynamics_like(b.dyn)
    z, v, phi = _t(b.z, dev), _t(b.v, dev), _t(tp.phi, dev)
    B, N = b.z.shape[:2]
    n = b.z.shape[2] + b.v.shape[2]
    mu_r, sg_r, c_r, sw_r = leb.fixed_point_solve(dyn, z, v, phi, tp.e, max_sweeps=max_sweeps)
    mu = torch.full((B, N, n), float("nan"), dtype=torch.float64, device=dev)
    sg = torch.full((B, N, n), float("nan"), dtype=torch.float64, device=dev)
    cert = torch.full((B,), 7, dtype=torch.int32, device=dev)
    sw = leb.fixed_point_solve_noalloc(dyn, z, v, phi, tp.e, mu, sg, cert, max_sweeps=max_sweeps)
    torch.cuda.synchronize()
    return (mu_r, sg_r, c_r, sw_r), (mu, sg, cert, sw)


def test_noalloc_matches_fixed_point_solve_twice(gpu):
    import torch
    import paper_2607_01203_amd as leb
    print("case: no-alloc fixed point 64x40x168, then 8x13x40", flush=True)
    for tp in (W.fixed_point_cfg(seed=4, batch=64, N=40), W.fixed_point_cfg(seed=5, batch=8, N=13, n_units=5)):
        (mu_r, sg_r, c_r, sw_r), (mu, sg, cert, sw) = _both(leb, tp, gpu)
        assert bool((c_r == 1).all()) and sw == 20 and sw_r < 20
        assert torch.equal(cert, c_r)
        assert torch.equal(mu, mu_r) and torch.equal(sg, sg_r)


def test_noalloc_sweep_cap(gpu):
    """At a cap of 3 sweeps nothing is accepted: both forms return the same
    latest iterate and all-zero flags."""
    import torch
    import paper_2607_01203_amd as leb
    print("case: no-alloc fixed point at a cap of 3 sweeps", flush=True)
    tp = W.fixed_point_cfg(seed=6, batch=5, N=17, n_units=3)
    (mu_r, sg_r, c_r, _), (mu, sg, cert, sw) = _both(leb, tp, gpu, max_sweeps=3)
    assert sw == 3 and bool((c_r == 0).all())
    assert torch.equal(cert, c_r) and torch.equal(mu, mu_r) and torch.equal(sg, sg_r)


def test_noalloc_refuses_problems_beyond_its_scratch(gpu):
    import torch
    import paper_2607_01203_amd as leb
    dyn = leb.chain_dynamics(28)
    B, N, n = 1024, 40, 224
    z = torch.zeros((B, N, 168), dtype=torch.float64, device=gpu)
    v = torch.zeros((B, N, 56), dtype=torch.float64, device=gpu)
    phi = torch.zeros((N - 1, 8, 6), dtype=torch.float64, device=gpu)
    mu = torch.zeros((B, N, n), dtype=torch.float64, device=gpu)
    sg = torch.zeros((B, N, n), dtype=torch.float64, device=gpu)
    cert = torch.zeros((B,), dtype=torch.int32, device=gpu)
    with pytest.raises(leb.LebError, match="scratch"):
        leb.fixed_point_solve_noalloc(dyn, z, v, phi, [0.0] * 6, mu, sg, cert)
