"""Failure handling on the GPU: a forced device-allocation failure is
reported as LEB_ENOMEM and leaves the library usable, and a corrupted or
stale autotuner cache only costs a re-tune (results stay bit-identical to
standalone calls)."""
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


def test_forced_allocation_failure_reports_enomem_and_recovers(gpu, monkeypatch):
    """leb_mlp_create allocates the network's device copies on every call; the
    test hook makes that allocation fail."""
    import torch
    import paper_2607_01203_amd as leb
    rng = W.rng_for(5)
    Wm, bm = W.mlp_weights(rng, [16, 32, 12])
    monkeypatch.setenv("LEB_TEST_FAIL_ALLOC", "1")
    print("case: forced allocation failure", flush=True)
    with pytest.raises(leb.LebError, match=r"\(-2\)"):
        leb.MLP(Wm, bm, nx=12)
    monkeypatch.delenv("LEB_TEST_FAIL_ALLOC")
    net = leb.MLP(Wm, bm, nx=12)
    z = torch.zeros((1, 3, 12), dtype=torch.float64, device=gpu)
    v = torch.zeros((1, 3, 4), dtype=torch.float64, device=gpu)
    sg = torch.full((1, 3, 16), 0.01, dtype=torch.float64, device=gpu)
    out = leb.nn_bound(net, z, v, sg)
    torch.cuda.synchronize()
    assert torch.isfinite(out["r_lo"]).all() and (out["r_lo"] <= out["r_hi"]).all()
    net.close()


def test_corrupted_tune_cache_is_retuned(gpu, tmp_path):
    import torch
    import paper_2607_01203_amd as leb
    mb = W.mixed_batch_cfg(seed=7, count=12)
    probs = []
    for kind, cfg in mb.problems:
        if kind != "analytic":
            continue
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(gpu)
        b = cfg
        probs.append({"kind": "analytic", "dyn": leb.dynamics_like(b.dyn), "z": t(b.z[0]), "v": t(b.v[0]),
                      "sigma": t(b.sigma[0]),
                      "r_lo": torch.empty((b.z.shape[1], b.z.shape[2]), dtype=torch.float64, device=gpu),
                      "r_hi": torch.empty((b.z.shape[1], b.z.shape[2]), dtype=torch.float64, device=gpu)})
    assert probs
    cache = tmp_path / "tune.txt"
    # keys with impossible tiles for every node count, then garbage and a binary tail
    keys = b"".join(b"gfx950|pbh|U=%d|units=%d 3\n" % (u, 1 << e) for u in (1, 2, 8, 28) for e in range(12))
    cache.write_bytes(keys + b"not a key line\n\x00\xff\xfe garbage 12 13\n")
    print("case: corrupted tune cache (%d problems)" % len(probs), flush=True)
    bt = leb.Batch(probs, tune_cache=cache)
    bt.submit()
    torch.cuda.synchronize()
    for p in probs:
        o = leb.analytic_bound(p["dyn"], p["z"][None], p["v"][None], p["sigma"][None])
        assert torch.equal(p["r_lo"], o["r_lo"][0]) and torch.equal(p["r_hi"], o["r_hi"][0])
    assert "(cached)" not in bt.info()
    bt.close()
