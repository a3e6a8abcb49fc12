"""Uneven problems in one graph launch (leb_batch_*): analytic chains of
1, 2, 8 and 28 nodes and ReLU-MLP dynamics of hidden width 128 and 256,
horizons 10..80.  Every problem's result must equal the standalone entry
point bit for bit, on every graph replay, also after the inputs change in
place between replays; a sample is checked against the oracle; the tune
cache is written and then used."""
import numpy as np
import pytest

import workloads as W
from parity import check_bounds

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
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)


def _problems(leb, mb, dev, nets):
    import torch
    out = []
    for kind, cfg in mb.problems:
        if kind == "analytic":
            z, v, sg = cfg.z[0], cfg.v[0], cfg.sigma[0]
            p = {"kind": "analytic", "dyn": leb.dynamics_like(cfg.dyn), "cfg": cfg}
            nx = z.shape[1]
        else:
            z, v, sg = cfg.z[0], cfg.v[0], cfg.sigma[0]
            key = id(cfg.net)
            if key not in nets:
                nets[key] = leb.MLP(cfg.net.W, cfg.net.b, cfg.net.nx, True)
            p = {"kind": "nn", "net": nets[key], "cfg": cfg}
            nx = cfg.net.W[-1].shape[0]
        N = z.shape[0]
        p.update(z=_t(z, dev), v=_t(v, dev), sigma=_t(sg, dev),
                 r_lo=torch.full((N, nx), np.nan, dtype=torch.float64, device=dev),
                 r_hi=torch.full((N, nx), np.nan, dtype=torch.float64, device=dev))
        out.append(p)
    return out


def _standalone(leb, p):
    z, v, sg = p["z"][None], p["v"][None], p["sigma"][None]
    if p["kind"] == "analytic":
        o = leb.analytic_bound(p["dyn"], z, v, sg)
    else:
        o = leb.nn_bound(p["net"], z, v, sg)
    return o["r_lo"][0], o["r_hi"][0]


def test_batch_matches_standalone_on_every_replay(gpu, tmp_path, orc):
    import torch
    import paper_2607_01203_amd as leb
    mb = W.mixed_batch_cfg(seed=3, count=40)
    nets = {}
    probs = _problems(leb, mb, gpu, nets)
    kinds = sorted({(p["kind"], p["z"].shape[1]) for p in probs})
    print("case: batch of %d problems, kinds %s" % (len(probs), kinds), flush=True)
    cache = tmp_path / "tune.txt"
    b = leb.Batch(probs, tune_cache=cache)
    print(b.info())
    assert cache.exists() and len(cache.read_text().splitlines()) >= 3
    ref = [_standalone(leb, p) for p in probs]
    for rep in range(3):
        for p in probs:
            p["r_lo"].fill_(np.nan)
            p["r_hi"].fill_(np.nan)
        b.submit()
        torch.cuda.synchronize()
        for p, (lo, hi) in zip(probs, ref):
            assert torch.equal(p["r_lo"], lo) and torch.equal(p["r_hi"], hi), (rep, p["kind"])
        # eager work between replays: grow every tube in place, recompute the reference
        for p in probs:
            p["sigma"].mul_(1.1)
        ref = [_standalone(leb, p) for p in probs]
        torch.cuda.synchronize()
    # oracle on one analytic and one MLP problem (inputs as now in the buffers)
    b.submit()
    torch.cuda.synchronize()
    from oracle import nn as onn
    for p in probs:
        if p["kind"] == "analytic" and p["z"].shape[1] == 48:
            cfg = p["cfg"]
            d = orc.Dyn.like(cfg.dyn)
            lo, hi, _ = orc.leb(d, cfg.z, cfg.v, p["sigma"].cpu().numpy()[None])
            check_bounds(p["r_lo"].cpu().numpy()[None], p["r_hi"].cpu().numpy()[None], lo, hi, "batch analytic")
            break
    for p in probs:
        if p["kind"] == "nn":
            cfg = p["cfg"]
            a = np.concatenate([cfg.z, cfg.v], -1)
            o = onn.leb(cfg.net.W, cfg.net.b, a, p["sigma"].cpu().numpy()[None])
            check_bounds(p["r_lo"].cpu().numpy()[None], p["r_hi"].cpu().numpy()[None], o["r_lo"], o["r_hi"],
                         "batch nn")
            break
    b.close()
    # a second batch of the same shapes takes its tiles from the cache
    b2 = leb.Batch(probs, tune_cache=cache)
    info = b2.info()
    print(info)
    assert "(cached)" in info
    b2.submit()
    torch.cuda.synchronize()
    b2.close()
    for n in nets.values():
        n.close()


def test_batch_rejects_bad_problems(gpu):
    import torch
    import paper_2607_01203_amd as leb
    dyn = leb.chain_dynamics(2)
    z = torch.zeros((5, 12), dtype=torch.float64, device=gpu)
    v = torch.zeros((5, 4), dtype=torch.float64, device=gpu)
    s = torch.zeros((5, 16), dtype=torch.float64, device=gpu)
    lo = torch.zeros((5, 12), dtype=torch.float64, device=gpu)
    p = {"kind": "analytic", "dyn": dyn, "z": z, "v": v, "sigma": s, "r_lo": lo, "r_hi": lo.clone()}
    with pytest.raises(leb.LebError):
        leb.Batch([dict(p, z=z[:0], v=v[:0], sigma=s[:0], r_lo=lo[:0], r_hi=lo[:0])])   # N = 0
    bad = leb.chain_dynamics(2)
    bad.nx = 13
    with pytest.raises(leb.LebError):
        leb.Batch([dict(p, dyn=bad)])
    b = leb.Batch([])
    b.submit()
    torch.cuda.synchronize()
    b.close()


def test_batch_256_problems_oracle_and_1e6_samples(gpu, orc):
    """The uneven-batch workload at full size (256 problems, nx in {6, 12,
    48, 168}, N in 10..80, about 11,000 units): every problem equals its
    standalone call bit for bit and the oracle within the parity tolerance,
    and the bounds contain 10^6 sampled true remainders (spread over all
    units, analytic and MLP)."""
    import torch
    import paper_2607_01203_amd as leb
    from oracle import nn as onn
    from parity import sampled_violations
    mb = W.mixed_batch_cfg(seed=3, count=256)
    nets = {}
    probs = _problems(leb, mb, gpu, nets)
    print("case: batch of 256 problems", flush=True)
    b = leb.Batch(probs, tune_cache=None)
    b.submit()
    torch.cuda.synchronize()
    units = sum(int(p["z"].shape[0]) for p in probs)
    per = 1_000_000 // units + 1
    viol = count = 0
    for i, p in enumerate(probs):
        lo_s, hi_s = _standalone(leb, p)
        torch.cuda.synchronize()
        assert torch.equal(p["r_lo"], lo_s) and torch.equal(p["r_hi"], hi_s), i
        cfg = p["cfg"]
        lo_g, hi_g = p["r_lo"].cpu().numpy(), p["r_hi"].cpu().numpy()
        nom = np.concatenate([cfg.z[0], cfg.v[0]], -1)
        if p["kind"] == "analytic":
            d = orc.Dyn.like(cfg.dyn)
            lo, hi, _ = orc.leb(d, cfg.z[0], cfg.v[0], cfg.sigma[0])

            def rem(nm, pts, d=d):
                U, P, n = pts.shape
                r, eps = orc.remainder(d, nm, pts.reshape(-1, n), np.repeat(np.arange(U), P))
                return r.reshape(U, P, -1), eps.reshape(U, P, -1)
        else:
            o = onn.leb(cfg.net.W, cfg.net.b, nom, cfg.sigma[0])
            lo, hi = o["r_lo"], o["r_hi"]

            def rem(nm, pts, net=cfg.net):
                return onn.remainder(net.W, net.b, nm, pts)
        check_bounds(lo_g, hi_g, lo, hi, "problem %d (%s)" % (i, p["kind"]))
        blo, bhi = orc.box(nom, cfg.sigma[0])
        v_, c_ = sampled_violations(rem, nom, blo, bhi, lo_g, hi_g, per, seed=3_000_000 + i)
        viol += v_
        count += c_
    print("units %d samples %d violations %d" % (units, count, viol))
    assert count >= 1_000_000 and viol == 0
    b.close()
    for n in nets.values():
        n.close()
