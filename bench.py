"""Benchmark: certified LEB timestep-bounds per second at nx = 168.

Workload: 256 trajectories x 40 steps of a chain of 28 planar quadrotors
(nx = 168, nu = 56) with a decentralised hover-LQR closed loop.  One step
is one certified tube/LEB fixed-point solve from device-resident inputs to
a certified tube on the device: Jacobi sweeps of the path-based Hessian
bound over all 10,240 (trajectory, step) units, the tube map, the
convergence test, and the certifying sweep (host orchestration included).
value = 10,240 x steps / wall time.

Prints ONE JSON line.  Extra objects:
  roofline      dominant kernel (the bound kernel) at the solve's launch
                shape, timed with HIP events on its stream;
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
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12   # lane-ops/s of non-packed VALU issue (39.3 T)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--cpu-seconds", type=float, default=20.0, help="target CPU baseline duration")
    p.add_argument("--kernel-reps", type=int, default=50)
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


def bytes_per_unit_fixed_point_launch(nx, nu):
    """Algorithmic HBM bytes of one unit in the fixed point's bound launch:
    reads z, v, mu, sigma; writes c_bar, rho_bar (all FP64)."""
    n = nx + nu
    return 8 * (nx + nu + n + n) + 8 * (2 * nx)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
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

    def step():
        return leb.fixed_point_solve(dyn, z, v, phi, tp.e, tol=1e-6, max_sweeps=200)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    sweeps = []
    certified = True
    t0 = time.perf_counter()
    for _ in range(args.steps):
        mu, sg, cert, sw = step()
        sweeps.append(sw)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    certified = bool((cert == 1).all().item())
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = units * args.steps / (t1 - t0)

    # dominant kernel: the bound launch of a sweep, at the certified tube
    cb = torch.empty((B, N, nx), dtype=torch.float64, device=dev)
    rb = torch.empty_like(cb)
    out = {"r_lo": None, "r_hi": None, "c_bar": cb, "rho_bar": rb, "flags": None}

    def bound_launch():
        rc = leb.lib().leb_analytic_bound(
            ctypes.byref(dyn), B, N, leb._dev_ptr(z, "z"), leb._dev_ptr(v, "v"), leb._dev_ptr(mu, "mu"),
            leb._dev_ptr(sg, "sigma"), None, None, leb._dev_ptr(cb, "c"), leb._dev_ptr(rb, "r"), 0.0, None,
            leb._stream(stream))
        leb._check(rc)

    for _ in range(3):
        bound_launch()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.kernel_reps):
        bound_launch()
    e1.record(stream)
    torch.cuda.synchronize()
    kern_us = e0.elapsed_time(e1) * 1e3 / args.kernel_reps
    bpu = bytes_per_unit_fixed_point_launch(nx, nu)
    achieved = bpu * units / (kern_us * 1e-6) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "pbh_chain_fwd", "launch_us": round(kern_us, 3), "units_per_launch": units,
                "bytes_per_unit": bpu}

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
                               "(nx=168, nu=56), N=40, cold start, batched Jacobi sweeps",
                   "trajectories": B, "horizon": N, "nx": nx, "nu": nu, "tol": 1e-6,
                   "form": "batched, cold start"},
        "sweeps_per_solve": int(np.median(sweeps)), "certified": certified,
        "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(line))


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
