"""Benchmark: certified LEB timestep-bounds per second at nx = 168.

Workload: 256 trajectories x 40 steps of a chain of 28 planar quadrotors
(nx = 168, nu = 56) with a decentralised hover-LQR closed loop.  One step
is one certified tube/LEB fixed-point solve from device-resident inputs to
a certified tube on the device (host orchestration included), in two forms:
  plain    Jacobi sweeps of the path-based Hessian bound over all 10,240
           (trajectory, step) units and the tube map, from the
           disturbance-only tube, until F(C) lies inside C;
  learned  a few tube sweeps with the BF16 surrogate's predicted bounds,
           inflation, then the same certified sweeps from that tube.
The surrogate is trained beforehand (outside the timed region) by the
library's kernels on certified bounds of other trajectories.
value = 10,240 / (learned ms per solve); the plain rate is reported too.

Prints ONE JSON line.  Extra objects:
  roofline      dominant kernel: the tube map of the certified sweeps (HBM;
                its FP64 MFMA rate beside), its launches in one learned
                solve timed with HIP events on the solve's stream;
                roofline_bound: the bound kernel of the same sweeps (HBM);
  cpu_baseline  the FP64 oracle solving (and certifying) the same fixed
                point on a bounded sample of trajectories, on host cores.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0            # MI355X HBM3E
# HBM traffic of one fixed-point tube-map launch at the bench shape, FETCH_SIZE and
# WRITE_SIZE (KiB per dispatch, rocprofv3 --pmc), and the factors that map each
# counter to bytes, measured on a copy kernel of known size; None until taken for
# the kernel as it is now.
TUBE_PMC_KIB = (27251, 35859)
FETCH_SCALE, WRITE_SCALE = 2.0, 1.0
FP64_PEAK_TFLOPS = 78.6          # MI355X FP64 matrix (= vector) peak
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12   # lane-ops/s of non-packed VALU issue (39.3 T)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--cpu-seconds", type=float, default=20.0, help="target CPU baseline duration")
    p.add_argument("--kernel-reps", type=int, default=50)
    p.add_argument("--epochs", type=int, default=20, help="surrogate training epochs (outside the timed region)")
    p.add_argument("--surrogate-sweeps", type=int, default=1)
    p.add_argument("--margin", type=float, default=5e-2, help="relative inflation of the surrogate tube")
    p.add_argument("--no-extra", action="store_true", help="skip the MLP-bound roofline and the uneven batch")
    p.add_argument("--nn-only", action="store_true",
                   help="only run the MLP-bound roofline measurement (for profiling its kernels)")
    p.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                   help="only run an elementwise copy (read BYTES, write BYTES) 5 times: the known-size "
                        "kernel that scales FETCH_SIZE / WRITE_SIZE counters")
    return p.parse_args()


def copy_calibration(nbytes):
    import torch
    dev = torch.device("cuda:0")
    src = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    for _ in range(5):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": nbytes, "launches": 5}))


def tube_flops_per_column(N):
    """Algorithmic FLOPs of the fixed point's tube map per (trajectory, node)
    column: for every step k and earlier step j < k, the products of the 8
    tube rows with the node's two non-affine residual rows (vx, vz), for the
    centre (Phi c_bar) and the width (|Phi| w), 2 FLOPs per multiply-add.  The
    four affine rows carry the residual (0, pad) exactly; their share of the
    width is one table over (k, row) for all columns."""
    return 2 * 2 * 8 * 2 * (N * (N - 1) // 2)


def tube_bytes_per_launch(B, N, nx, nu):
    """Algorithmic HBM bytes of the fixed-point tube-map launch: reads the
    residual rows 3 and 4 of each node (c_bar, rho_bar [B][N][U][2]) and
    C_{t-1} (mu, sigma) [B][N][nx+nu] for the containment test, writes C_t
    (mu, sigma), all FP64."""
    n = nx + nu
    return 8 * B * N * (2 * (2 * (nx // 6)) + 2 * n + 2 * n)


def bytes_per_unit_fixed_point_launch(nx, nu):
    """Algorithmic HBM bytes of one unit in the fixed point's bound launch:
    reads z, v, mu, sigma; writes c_bar, rho_bar of rows 3 and 4 of each node
    (all FP64)."""
    n = nx + nu
    return 8 * (nx + nu + n + n) + 8 * (2 * 2 * (nx // 6))


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    import numpy as np
    import torch

    import paper_2607_01203_amd as leb
    import workloads as W

    dev = torch.device("cuda:0")
    if args.nn_only:
        print(json.dumps({"roofline_nn": nn_roofline(leb, W, dev, torch.cuda.current_stream(), args)}))
        return
    tp = W.fixed_point_cfg()
    b = tp.batch
    B, N, nx = b.z.shape
    nu = b.v.shape[2]
    n = nx + nu
    units = B * N
    dyn = leb.dynamics_like(b.dyn)
    z = torch.from_numpy(b.z).to(dev)
    v = torch.from_numpy(b.v).to(dev)
    phi = torch.from_numpy(tp.phi).to(dev)
    stream = torch.cuda.current_stream()

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        sweeps = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            res = fn()
            sweeps.append(res[3])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        return (t1 - t0) * 1e3 / args.steps, res, int(np.median(sweeps))

    # plain form: certified fixed point from the disturbance-only tube
    plain_ms, (mu0, sg0, cert0, _), plain_sweeps = timed(
        lambda: leb.fixed_point_solve(dyn, z, v, phi, tp.e, tol=1e-6, max_sweeps=200))
    plain_cert = bool((cert0 == 1).all().item())

    # learned form: surrogate trained (outside the timed region) on certified
    # bounds of other trajectories, then surrogate sweeps + certified sweeps
    net, train_info = train_chain_surrogate(leb, W, dev, args)
    learned_ms, (mu, sg, cert, _), learned_sweeps = timed(
        lambda: leb.fixed_point_learned(dyn, z, v, phi, tp.e, net, sweeps=args.surrogate_sweeps,
                                        margin=args.margin, tol=1e-6, max_sweeps=200))
    certified = bool((cert == 1).all().item())
    s0 = sg0.cpu().numpy()
    s1 = sg.cpu().numpy()
    pos = s0 > 0
    excess = s1[pos] / s0[pos] - 1.0
    ms_per_step = learned_ms
    value = units * 1e3 / learned_ms

    # comparison start without the surrogate: one plain sweep from the
    # disturbance-only tube, sigma inflated by the same margin, then the
    # certified iteration (two library calls)
    def exact_start():
        m, s_, _, _ = leb.fixed_point_solve(dyn, z, v, phi, tp.e, tol=1e-6, max_sweeps=1)
        s_.mul_(1.0 + args.margin).add_(1e-12)
        return leb.fixed_point_solve(dyn, z, v, phi, tp.e, tol=1e-6, max_sweeps=200, mu=m, sigma=s_)
    exact_ms, (_, sg_x, cert_x, _), exact_sweeps = timed(exact_start)
    ex_x = sg_x.cpu().numpy()[pos] / s0[pos] - 1.0
    exact_line = {"ms_per_solve": round(exact_ms, 4), "certified_sweeps": 1 + exact_sweeps,
                  "certified": bool((cert_x == 1).all().item()),
                  "sigma_over_plain_median": round(float(np.median(ex_x)), 6),
                  "sigma_over_plain_max": round(float(ex_x.max()), 6)}

    # Dominant kernel: the tube map of the certified sweeps (6 of the ~11 launches
    # of a learned solve, the largest share of its time).  Its launches in one
    # learned solve are timed with HIP events on the solve's stream; the
    # speculative sweep after the certifying one is left out.
    leb.launch_timing(True)
    _, _, _, sw_t = leb.fixed_point_learned(dyn, z, v, phi, tp.e, net, sweeps=args.surrogate_sweeps,
                                            margin=args.margin, tol=1e-6, max_sweeps=200)
    torch.cuda.synchronize()
    tube_ms = leb.launch_times(leb.LAUNCH_TUBE)[:sw_t]
    bound_ms = leb.launch_times(leb.LAUNCH_BOUND)[:sw_t]
    leb.launch_timing(False)
    U = nx // 6
    tube_us = 1e3 * float(np.mean(tube_ms))
    tflops = tube_flops_per_column(N) * B * U / (tube_us * 1e-6) / 1e12
    tube_bytes = tube_bytes_per_launch(B, N, nx, nu)
    gbs = tube_bytes / (tube_us * 1e-6) / 1e9
    traffic = None
    if TUBE_PMC_KIB is not None:
        traffic = int(TUBE_PMC_KIB[0] * 1024 * FETCH_SCALE + TUBE_PMC_KIB[1] * 1024 * WRITE_SCALE)
    # HBM-bound: 82.6 MB against 0.36 GFLOP per launch at the bench shape
    roofline = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "tube_map2_kernel", "launch_us": round(tube_us, 2), "launches": len(tube_ms),
                "units_per_launch": B * U, "bytes_per_launch": tube_bytes,
                "flops_per_unit": tube_flops_per_column(N), "mfma_tflops": round(tflops, 2),
                "mfma_frac": round(tflops / FP64_PEAK_TFLOPS, 4)}
    # the bound kernel of the same sweeps
    bound_us = 1e3 * float(np.mean(bound_ms))
    bpu = bytes_per_unit_fixed_point_launch(nx, nu)
    achieved = bpu * units / (bound_us * 1e-6) / 1e9
    roofline_bound = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                      "frac": round(achieved / HBM_PEAK_GBS, 4), "kernel": "pbh_chain_fwd",
                      "launch_us": round(bound_us, 2), "launches": len(bound_ms), "units_per_launch": units,
                      "bytes_per_unit": bpu}

    nn_line = None if args.no_extra else nn_roofline(leb, W, dev, stream, args)
    nn_learned_line = None if args.no_extra else nn_learned(leb, W, dev, stream, args)
    batch_line = None if args.no_extra else batched_uneven(leb, W, dev, stream, args)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(W, tp, args.cpu_seconds)

    line = {
        "metric": "certified LEB timestep-bounds/s at nx=168 (plain vs batched+learned), 0 violations",
        "value": round(value, 1), "unit": "timestep-bounds/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32-interval+f64",
        "data": "synthetic",
        "config": {"workload": "certified tube/LEB fixed point, 256 chains of 28 planar quadrotors "
                               "(nx=168, nu=56), N=40, batched Jacobi sweeps; value: learned warm start",
                   "trajectories": B, "horizon": N, "nx": nx, "nu": nu, "tol": 1e-6,
                   "form": "batched + learned warm start"},
        "certified": certified,
        "learned": {"certified_sweeps": learned_sweeps, "surrogate_sweeps": args.surrogate_sweeps,
                    "margin": args.margin, "ms_per_solve": round(learned_ms, 4),
                    "sigma_over_plain_median": round(float(np.median(excess)), 6),
                    "sigma_over_plain_max": round(float(excess.max()), 6), "training": train_info},
        "exact_start_same_margin": exact_line,
        "plain": {"value": round(units * 1e3 / plain_ms, 1), "ms_per_solve": round(plain_ms, 4),
                  "certified_sweeps": plain_sweeps, "certified": plain_cert},
        "roofline": roofline, "cpu_baseline": cpu, "roofline_bound": roofline_bound,
        "roofline_nn": nn_line, "learned_nn": nn_learned_line, "batched_uneven": batch_line,
    }
    print(json.dumps(line))


def nn_crown_flops(widths):
    """Algorithmic FLOPs per box of the CROWN passes as the MLP bound runs
    them: for every target layer k >= 2 (hidden layers with 2 modes, upper
    and lower; the output layer with 3, adding the Jacobian), the chain of
    products through layers k-1 .. 1 is [w_k x w_j] . [w_j x w_{j-1}]."""
    L = len(widths) - 1
    mac = 0
    for k in range(2, L + 1):
        modes = 3 if k == L else 2
        for j in range(k - 1, 0, -1):
            mac += modes * widths[k] * widths[j] * widths[j - 1]
    return 2 * mac


def nn_roofline(leb, W, dev, stream, args):
    """MLP bound (CROWN + Theorem 2) on 64 x 50 boxes of the 16-256-256-256-12
    network: FP64 MFMA, timed with HIP events on its stream."""
    import torch
    b = W.nn_cfg()
    net = leb.MLP(b.net.W, b.net.b, b.net.nx, True)
    z = torch.from_numpy(b.z).to(dev)
    v = torch.from_numpy(b.v).to(dev)
    sg = torch.from_numpy(b.sigma).to(dev)
    for _ in range(2):
        leb.nn_bound(net, z, v, sg, stream=stream)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reps = 5
    e0.record(stream)
    for _ in range(reps):
        leb.nn_bound(net, z, v, sg, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    boxes = b.z.shape[0] * b.z.shape[1]
    widths = [b.net.W[0].shape[1]] + [w.shape[0] for w in b.net.W]
    fl = nn_crown_flops(widths) * boxes
    net.close()
    achieved = fl / (ms * 1e-3) / 1e12
    return {"workload": "MLP bound, 64 x 50 boxes, widths %s" % widths, "ms_per_call": round(ms, 4),
            "timestep_bounds_per_s": round(boxes / (ms * 1e-3), 1),
            "bound": "mfma", "achieved": round(achieved, 2), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / FP64_PEAK_TFLOPS, 4), "flops_per_box": nn_crown_flops(widths)}


def nn_learned(leb, W, dev, stream, args):
    """NN family of the learned start: 10^5 certified samples (boxes drawn
    like the MLP-bound workload's, bounded by CROWN + Theorem 2), the
    32-128-128-128-24 surrogate trained by the library's kernels, and its
    prediction for the 64 x 50 boxes of the MLP-bound workload against
    their certified bound (error in log space; call time, HIP events)."""
    import torch
    from paper_2607_01203_amd import learned
    b = W.nn_cfg()
    mlp = leb.MLP(b.net.W, b.net.b, b.net.nx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    X, T = learned.nn_samples(mlp, 100000, seed=31)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    widths = learned.nn_widths(mlp)
    net = leb.Surrogate(widths, learned.he_init(widths, 0))
    hist = learned.train(net, X, T, epochs=args.epochs, batch=512, lr=2e-3)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    z = torch.from_numpy(b.z).to(dev)
    v = torch.from_numpy(b.v).to(dev)
    sg = torch.from_numpy(b.sigma).to(dev)
    cert = leb.nn_bound(mlp, z, v, sg)
    lo, hi = leb.nn_surrogate_bound(net, z, v, sg, stream=stream)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reps = 20
    e0.record(stream)
    for _ in range(reps):
        leb.nn_surrogate_bound(net, z, v, sg, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    floor = 1e-14
    err = torch.cat([(hi.clamp_min(floor).log() - cert["r_hi"].clamp_min(floor).log()).abs().reshape(-1),
                     ((-lo).clamp_min(floor).log() - (-cert["r_lo"]).clamp_min(floor).log()).abs().reshape(-1)])
    q = torch.quantile(err, torch.tensor([0.5, 0.9], dtype=err.dtype, device=err.device)).cpu().numpy()
    under = float((hi < cert["r_hi"]).double().mean().item())
    net.close()
    mlp.close()
    return {"workload": "NN-family surrogate %s on 64 x 50 boxes of the MLP-bound workload" % widths,
            "samples": int(X.shape[0]), "epochs": args.epochs, "sample_s": round(t1 - t0, 2),
            "train_s": round(t2 - t1, 2), "loss_first": round(hist[0], 5), "loss_last": round(hist[-1], 5),
            "abs_log_err_q50_q90": [round(float(x), 4) for x in q],
            "hi_below_certified_frac": round(under, 4), "ms_per_call": round(ms, 4)}


def batched_uneven(leb, W, dev, stream, args):
    """256 uneven problems (nx in {6, 12, 48, 168}, horizons 10..80) in one
    graph launch, tiles from the autotuner."""
    import numpy as np
    import torch
    mb = W.mixed_batch_cfg(seed=3, count=256)
    nets = {}
    probs = []
    units = 0
    for kind, cfg in mb.problems:
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a[0])).to(dev)
        p = {"z": t(cfg.z), "v": t(cfg.v), "sigma": t(cfg.sigma)}
        if kind == "analytic":
            p.update(kind="analytic", dyn=leb.dynamics_like(cfg.dyn))
            nx = cfg.z.shape[2]
        else:
            if id(cfg.net) not in nets:
                nets[id(cfg.net)] = leb.MLP(cfg.net.W, cfg.net.b, cfg.net.nx, True)
            p.update(kind="nn", net=nets[id(cfg.net)])
            nx = cfg.net.W[-1].shape[0]
        N = cfg.z.shape[1]
        units += N
        p["r_lo"] = torch.empty((N, nx), dtype=torch.float64, device=dev)
        p["r_hi"] = torch.empty((N, nx), dtype=torch.float64, device=dev)
        probs.append(p)
    t0 = time.perf_counter()
    bt = leb.Batch(probs, tune_cache=None)
    create_s = time.perf_counter() - t0
    bt.submit(stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reps = 5
    e0.record(stream)
    for _ in range(reps):
        bt.submit(stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    info = bt.info().strip().splitlines()
    bt.close()
    for n in nets.values():
        n.close()
    return {"workload": "256 uneven problems, nx in {6,12,48,168}, N in 10..80, one graph launch",
            "timestep_bounds": units, "ms_per_submit": round(ms, 4),
            "timestep_bounds_per_s": round(units / (ms * 1e-3), 1), "create_s": round(create_s, 2),
            "groups": info}


def train_chain_surrogate(leb, W, dev, args):
    """Certified training samples from 64 other trajectories (seed 100),
    3 draws of scaled tubes around their certified fixed points (215,040
    node samples), trained with the library's BF16 kernels."""
    import torch
    from paper_2607_01203_amd import learned
    t0 = time.perf_counter()
    tp = W.fixed_point_cfg(seed=100, batch=64, N=40)
    b = tp.batch
    dyn = leb.dynamics_like(b.dyn)
    z = torch.from_numpy(b.z).to(dev)
    v = torch.from_numpy(b.v).to(dev)
    mu, sg, _, _ = leb.fixed_point_solve(dyn, z, v, torch.from_numpy(tp.phi).to(dev), tp.e)
    X, T = learned.chain_samples(dyn, z, v, mu.cpu().numpy(), sg.cpu().numpy(), draws=3, seed=1)
    net = leb.Surrogate(learned.CHAIN_WIDTHS, learned.he_init(learned.CHAIN_WIDTHS, 0))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    hist = learned.train(net, X, T, epochs=args.epochs, batch=1024, lr=2e-3)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    return net, {"samples": int(X.shape[0]), "epochs": args.epochs, "loss_first": round(hist[0], 5),
                 "loss_last": round(hist[-1], 6), "sample_s": round(t1 - t0, 2), "train_s": round(t2 - t1, 2)}


def cpu_baseline(W, tp, seconds):
    """Oracle fixed point (sequential sweep) plus its certifying sweep on a
    bounded sample of the trajectories, all host cores."""
    import numpy as np

    import oracle
    from oracle import tube

    cores = len(os.sched_getaffinity(0))
    b = tp.batch
    d = oracle.Dyn.like(b.dyn)

    def solve(idx):
        # exact fixed point by one sequential sweep, then the certifying sweep
        # (F(B) inside B; equality for the exact fixed point)
        mu, sg, _, _ = tube.fixed_point(d, b.z[idx], b.v[idx], tp.phi, tp.e, threads=cores)
        lo, hi, _ = oracle.leb(d, b.z[idx], b.v[idx], sg, mu=mu, threads=cores)
        c, r = tube.zono(lo, hi)
        m2, s2 = tube.tube_map(tp.phi, tp.e, c, r)
        return tube.contains(mu, sg, m2, s2)

    t0 = time.perf_counter()
    solve(np.arange(16))
    per_traj = (time.perf_counter() - t0) / 16
    count = int(max(16, min(b.z.shape[0], seconds / max(per_traj, 1e-6))))
    idx = np.arange(count)
    t0 = time.perf_counter()
    ok = solve(idx)
    dt = time.perf_counter() - t0
    N = b.z.shape[1]
    return {"value": round(count * N / dt, 2), "unit": "timestep-bounds/s", "cores": cores, "kind": "oracle",
            "sample": "%d of %d trajectories (N=%d, nx=168), exact fixed point + certifying sweep, %.1f s"
                      % (count, b.z.shape[0], N, dt),
            "certified": bool(ok.all())}


if __name__ == "__main__":
    main()
