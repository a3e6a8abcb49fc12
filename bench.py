"""Benchmark: certified LEB timestep-bounds per second at nx = 168.

Workload: 256 trajectories x 40 steps of a chain of 28 planar quadrotors
(nx = 168, nu = 56) with a decentralised hover-LQR closed loop.  One step
is one certified tube/LEB fixed-point solve from device-resident inputs to
a certified tube on the device (host orchestration included).  Every form
accepts a trajectory only when its tube is certified (F(C) inside C) and
converged (relative change <= 1e-6), so all forms end at the same tube:
  plain    Jacobi sweeps of the path-based Hessian bound over all 10,240
           (trajectory, step) units and the tube map, from the
           disturbance-only tube;
  learned  one tube sweep with the BF16 surrogate's predicted bounds, then
           the same certified sweeps from that tube.  Two networks: one
           trained to map a tube to its bound, one trained to map the cold
           start to the fixed point's bound (value: the latter);
  exact    one plain sweep, then the certified iteration (the start that a
           bound-map surrogate sweep emulates).
The surrogates are trained beforehand (outside the timed region) by the
library's kernels on certified bounds of other trajectories.
value = 10,240 / (learned ms per solve); the plain rate is reported too.

Prints ONE JSON line.  Extra objects:
  roofline        dominant kernel: the tube map of the certified sweeps (HBM;
                  its FP64 MFMA rate beside), its launches in one learned
                  solve timed with HIP events on the solve's stream;
  roofline_bound  the path-based bound kernel at 2,560 x 40 units per launch
                  (VALU issue, HBM beside), and as one 40-step trajectory;
  cpu_baseline    the FP64 oracle solving (and certifying) the same fixed
                  point on a bounded sample of trajectories, on all host
                  cores and on one;
  latency, adjoint, batched_uneven (batch against per-problem launches),
  roofline_nn, nn_adjoint (the MLP bound's gradient, against the bound's own
  time), learned_nn, nominal_pgd (nominal points refined by projected
  gradient descent on the bound's width against random nominal points at
  an equal GPU time budget), interval_hessian_study (satellite and 3-D
  quadrotor: mean row width of the path, expanded and classic enclosures and
  of 10,000 random samples for radii 0.01 .. 0.2, and the time of one call
  for a single local set), sls_update (one controller update of the SLS
  layer: linearization, Riccati responses, exact tube/LEB fixed point with
  the state-dependent disturbance error, 256 trajectories of N = 40).
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
TUBE_PMC_KIB = (27280, 36110)
FETCH_SCALE, WRITE_SCALE = 2.0, 1.0
FP64_PEAK_TFLOPS = 78.6          # MI355X FP64 matrix (= vector) peak
FP32_MFMA_PEAK_TFLOPS = 157.3    # MI355X dense FP32 matrix peak (the compact tube map's contraction)
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12   # lane-ops/s of non-packed VALU issue (39.3 T)
# VALU lane-operations per unit of the path-based bound kernel at nx = 168:
# SQ_INSTS_VALU x 64 / units from rocprofv3 --pmc on the 2,560 x 40 launch
# (profiles/pbh_chain_fwd_plain_2560x40x168.md; None until taken for the kernel as it is now).
PBH_VALU_LANE_OPS_PER_UNIT = 52723


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
    p.add_argument("--margin", type=float, default=0.0, help="relative inflation of the surrogate tube")
    p.add_argument("--no-extra", action="store_true", help="skip the MLP-bound roofline and the uneven batch")
    p.add_argument("--nn-only", action="store_true",
                   help="only run the MLP-bound roofline measurement (for profiling its kernels)")
    p.add_argument("--m2-only", action="store_true",
                   help="only run the path-based bound at 2,560 x 40 units per launch (for profiling it)")
    p.add_argument("--sls-only", action="store_true",
                   help="only run the SLS controller-update leg (for profiling its kernels)")
    p.add_argument("--fp-epochs", type=int, default=100, help="epochs of the fixed-point-target surrogate")
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
        st = torch.cuda.current_stream()
        print(json.dumps({"roofline_nn": nn_roofline(leb, W, dev, st, args), "nn_adjoint": nn_adjoint(leb, W, dev, st)}))
        return
    if args.m2_only:
        print(json.dumps({"roofline_bound": plain_m2(leb, W, dev, torch.cuda.current_stream(), args)}))
        return
    if args.sls_only:
        print(json.dumps({"sls_update": sls_update(leb, W, dev, torch.cuda.current_stream())}))
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
    s0 = sg0.cpu().numpy()
    pos = s0 > 0

    def tightness(sg):
        ex = sg.cpu().numpy()[pos] / s0[pos] - 1.0
        return {"sigma_over_plain_median": float("%.3g" % np.median(ex)),
                "sigma_over_plain_max": float("%.3g" % np.abs(ex).max())}

    # learned forms: surrogates trained (outside the timed region) on certified
    # bounds of other trajectories, then one surrogate sweep + certified sweeps
    net, train_info = train_chain_surrogate(leb, W, dev, args)
    net_fp, train_fp_info = train_fp_surrogate(leb, W, dev, args)
    forms = {}
    for name, nw, info in (("bound_map", net, train_info), ("fixed_point_target", net_fp, train_fp_info)):
        ms, (_, sg, cert, _), sw = timed(
            lambda: leb.fixed_point_learned(dyn, z, v, phi, tp.e, nw, sweeps=args.surrogate_sweeps,
                                            margin=args.margin, tol=1e-6, max_sweeps=200))
        forms[name] = dict({"ms_per_solve": round(ms, 4), "value": round(units * 1e3 / ms, 1),
                            "certified_sweeps": sw, "certified": bool((cert == 1).all().item()),
                            "training": info}, **tightness(sg))
    learned_ms = forms["fixed_point_target"]["ms_per_solve"]
    certified = forms["fixed_point_target"]["certified"] and plain_cert
    ms_per_step = learned_ms
    value = units * 1e3 / learned_ms

    # comparison start without the surrogate: one plain sweep from the
    # disturbance-only tube (inflated by the same margin), then the certified
    # iteration (two library calls)
    def exact_start():
        m, s_, _, _ = leb.fixed_point_solve(dyn, z, v, phi, tp.e, tol=1e-6, max_sweeps=1)
        if args.margin:
            s_.mul_(1.0 + args.margin).add_(1e-12)
        return leb.fixed_point_solve(dyn, z, v, phi, tp.e, tol=1e-6, max_sweeps=200, mu=m, sigma=s_)
    exact_ms, (_, sg_x, cert_x, _), exact_sweeps = timed(exact_start)
    exact_line = dict({"ms_per_solve": round(exact_ms, 4), "certified_sweeps": 1 + exact_sweeps,
                       "certified": bool((cert_x == 1).all().item())}, **tightness(sg_x))

    # Dominant kernel: the tube map of the certified sweeps (6 of the ~11 launches
    # of a learned solve, the largest share of its time).  Its launches in one
    # learned solve are timed with HIP events on the solve's stream; the
    # speculative sweep after the certifying one is left out.
    leb.launch_timing(True)
    _, _, _, sw_t = leb.fixed_point_learned(dyn, z, v, phi, tp.e, net_fp, sweeps=args.surrogate_sweeps,
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
                "mfma_frac": round(tflops / FP32_MFMA_PEAK_TFLOPS, 4), "mfma_dtype": "f32"}
    # the bound kernel of the same sweeps (its own roofline is taken at the
    # replicated scale below)
    bound_us = 1e3 * float(np.mean(bound_ms))
    bpu = bytes_per_unit_fixed_point_launch(nx, nu)
    bound_in_sweeps = {"kernel": "pbh_chain_fwd (fixed-point sweeps, with the fold)", "launch_us": round(bound_us, 2),
                       "launches": len(bound_ms), "units_per_launch": units, "bytes_per_unit": bpu,
                       "hbm_frac": round(bpu * units / (bound_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}
    net.close()
    net_fp.close()

    roofline_bound = plain_m2(leb, W, dev, stream, args)
    roofline_bound["in_fixed_point_sweeps"] = bound_in_sweeps
    extra = {} if args.no_extra else {
        "latency": latency(leb, W, dev, stream),
        "adjoint": adjoint(leb, W, dev, stream),
        "nominal_pgd": nominal_pgd(leb, W, dev, stream),
        "interval_hessian_study": interval_hessian_study(leb, W, dev, stream),
        "sls_update": sls_update(leb, W, dev, stream),
        "roofline_nn": nn_roofline(leb, W, dev, stream, args),
        "nn_adjoint": nn_adjoint(leb, W, dev, stream),
        "learned_nn": nn_learned(leb, W, dev, stream, args),
        "batched_uneven": batched_uneven(leb, W, dev, stream, args)}

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
                               "(nx=168, nu=56), N=40, batched Jacobi sweeps, accepted when certified and "
                               "converged to 1e-6; value: learned warm start (fixed-point-target network)",
                   "trajectories": B, "horizon": N, "nx": nx, "nu": nu, "tol": 1e-6, "conv_tol": 1e-6,
                   "form": "batched + learned warm start"},
        "certified": certified,
        "learned": forms["fixed_point_target"],
        "learned_bound_map": forms["bound_map"],
        "exact_start_same_margin": exact_line,
        "plain": {"value": round(units * 1e3 / plain_ms, 1), "ms_per_solve": round(plain_ms, 4),
                  "certified_sweeps": plain_sweeps, "certified": plain_cert},
        "roofline": roofline, "cpu_baseline": cpu, "roofline_bound": roofline_bound,
    }
    line.update(extra)
    print(json.dumps(line))


def plain_m2(leb, W, dev, stream, args):
    """The path-based bound on its own at nx = 168: 2,560 trajectories x 40
    steps (102,400 units) per launch, 20 launches timed with HIP events on
    the stream (VALU issue rate against the non-packed peak; HBM beside),
    and one 40-step trajectory per launch (latency)."""
    import numpy as np
    import torch
    b = W.chain_cfg(seed=2, N=40, n_units=28, batch=2560)
    dyn = leb.dynamics_like(b.dyn)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    z, v, sg = t(b.z), t(b.v), t(b.sigma)
    B, N, nx = b.z.shape
    nu = b.v.shape[2]
    units = B * N
    out = {"r_lo": torch.empty((B, N, nx), dtype=torch.float64, device=dev),
           "r_hi": torch.empty((B, N, nx), dtype=torch.float64, device=dev),
           "flags": torch.empty((B, N), dtype=torch.int32, device=dev)}

    def per_launch(zz, vv, ss, oo, reps):
        for _ in range(3):
            leb.analytic_bound(dyn, zz, vv, ss, stream=stream, out=oo)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            leb.analytic_bound(dyn, zz, vv, ss, stream=stream, out=oo)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e3

    us = per_launch(z, v, sg, out, 20)
    bpu = 8 * (nx + nu + (nx + nu)) + 8 * 2 * nx       # z, v, sigma in; r_lo, r_hi out
    gbs = bpu * units / (us * 1e-6) / 1e9
    one = {k: x[:1].contiguous() for k, x in out.items()}
    us1 = per_launch(z[:1].contiguous(), v[:1].contiguous(), sg[:1].contiguous(), one, 200)
    line = {"kernel": "pbh_chain_fwd", "workload": "2,560 x 40 chain units (nx=168) per launch",
            "launch_us": round(us, 2), "launches": 20, "units_per_launch": units,
            "timestep_bounds_per_s": round(units / (us * 1e-6), 1), "bytes_per_unit": bpu,
            "hbm_achieved": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
            "one_trajectory_us": round(us1, 2)}
    if PBH_VALU_LANE_OPS_PER_UNIT is not None:
        tops = PBH_VALU_LANE_OPS_PER_UNIT * units / (us * 1e-6) / 1e12
        line.update({"bound": "valu", "achieved": round(tops, 2), "peak": round(VALU_PEAK_TOPS, 1),
                     "unit": "T lane-ops/s", "frac": round(tops / VALU_PEAK_TOPS, 4),
                     "lane_ops_per_unit": PBH_VALU_LANE_OPS_PER_UNIT})
    else:
        line.update({"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 4)})
    return line


def latency(leb, W, dev, stream):
    """The planar quadrotor of 20 steps, one call at a time: device time per
    launch (HIP events over 200 back-to-back calls) and host wall time per
    call including the binding."""
    import torch
    b = W.planar_quad_cfg()
    dyn = leb.dynamics_like(b.dyn)
    t = lambda a: torch.from_numpy(a).to(dev)
    z, v, sg = t(b.z), t(b.v), t(b.sigma)
    out = leb.analytic_bound(dyn, z, v, sg, stream=stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reps = 200
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(reps):
        leb.analytic_bound(dyn, z, v, sg, stream=stream, out=out)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / reps * 1e6
    return {"workload": "planar quadrotor, 1 x 20 steps (nx=6)", "device_us_per_call": round(e0.elapsed_time(e1) /
                                                                                          reps * 1e3, 2),
            "host_us_per_call": round(wall, 2)}


def adjoint(leb, W, dev, stream):
    """leb_backward (the adjoint of the path-based bound) at nx = 168: one
    trajectory of 40 steps and 256 of them, HIP events over 20 calls."""
    import torch
    res = {}
    for B in (1, 256):
        b = W.chain_cfg(seed=2, N=40, n_units=28, batch=B)
        dyn = leb.dynamics_like(b.dyn)
        t = lambda a: torch.from_numpy(a).to(dev)
        z, v, sg = t(b.z), t(b.v), t(b.sigma)
        g = torch.ones((B, 40, 168), dtype=torch.float64, device=dev)
        gn = -g
        for _ in range(2):
            leb.backward(dyn, z, v, sg, g, gn, stream=stream)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        reps = 20
        e0.record(stream)
        for _ in range(reps):
            leb.backward(dyn, z, v, sg, g, gn, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) / reps * 1e3
        res["%dx40" % B] = {"us_per_call": round(us, 2), "timestep_gradients_per_s": round(B * 40 / (us * 1e-6), 1)}
    return res


def _sample_nominal(leb, dyn, a0, sigma, radius, K, gen, stream, chunk=64):
    """Narrowest bound (travelling box) over K nominal points drawn uniformly
    from a0 +/- radius sigma, in batched launches of `chunk` candidates."""
    import torch
    nx = dyn.nx
    U = a0.shape[0] * a0.shape[1]
    best = None
    done = 0
    while done < K:
        k = min(chunk, K - done)
        u = torch.rand((k,) + tuple(a0.shape), generator=gen, dtype=torch.float64, device=a0.device)
        a = (a0.unsqueeze(0) + (2.0 * u - 1.0) * radius * sigma.unsqueeze(0)).reshape(k * a0.shape[0], a0.shape[1], -1)
        sg = sigma.unsqueeze(0).expand(k, -1, -1, -1).reshape(a.shape).contiguous()
        o = leb.analytic_bound(dyn, a[..., :nx].contiguous(), a[..., nx:].contiguous(), sg, stream=stream)
        w = (o["r_hi"] - o["r_lo"]).sum(-1).reshape(k, U).min(0).values
        best = w if best is None else torch.minimum(best, w)
        done += k
    return best


def nominal_pgd(leb, W, dev, stream):
    """Nominal-point refinement (leb_pgd_nominal, 10 steps, search radius
    sigma, travelling box) on the planar quadrotor (64 nominal points) and the
    28-quadrotor chain (40 steps), against the best of as many random nominal
    points as the GPU bounds in the same time."""
    import torch
    res = {}
    radius, steps, lr = 1.0, 10, 0.3
    for name, b in (("planar_quadrotor_64", W.planar_quad_cfg(N=64)), ("chain28_40", W.chain_cfg(N=40))):
        dyn = leb.dynamics_like(b.dyn)
        t = lambda a: torch.from_numpy(a).to(dev)
        z0, v0, sg = t(b.z), t(b.v), t(b.sigma)
        a0 = torch.cat([z0, v0], -1)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        leb.pgd_nominal(dyn, z0, v0, sg, radius=radius, steps=steps, lr=lr, stream=stream)
        reps = 10
        e0.record(stream)
        for _ in range(reps):
            z, v, w, w0 = leb.pgd_nominal(dyn, z0, v0, sg, radius=radius, steps=steps, lr=lr, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_pgd = e0.elapsed_time(e1) / reps
        gen = torch.Generator(device=dev)
        gen.manual_seed(11)
        _sample_nominal(leb, dyn, a0, sg, radius, 128, gen, stream)     # warm every library call
        e0.record(stream)
        _sample_nominal(leb, dyn, a0, sg, radius, 512, gen, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        per = e0.elapsed_time(e1) / 512
        K = max(4 * steps, int(-(-ms_pgd // per)))
        e0.record(stream)
        best = _sample_nominal(leb, dyn, a0, sg, radius, K, gen, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        w, w0 = w.reshape(-1), w0.reshape(-1)
        res[name] = {"ms_pgd": round(ms_pgd, 4), "ms_sampling": round(e0.elapsed_time(e1), 4), "samples": K,
                     "mean_width_start": float(w0.mean()), "mean_width_sampling": float(best.mean()),
                     "mean_width_pgd": float(w.mean()), "pgd_better_frac": float((w < best).double().mean()),
                     "pgd_not_worse_frac": float((w <= best).double().mean())}
    return res


def sls_update(leb, W, dev, stream):
    """One controller update of the SLS layer on 256 trajectories, N = 40:
    linearization with the thrust-disturbance matrix (leb_linearize),
    closed-loop responses by the parallel Riccati recursions
    (leb_sls_responses) and the exact tube/LEB fixed point with r_dist
    (leb_sls_fixed_point), for the planar quadrotor (nx = 6) and a chain of
    2 (nx = 12), and for 1,024 planar-quadrotor trajectories (four per
    compute unit in the causal pass).  Each call is timed with HIP events on the stream
    (buffers allocated beforehand); bytes are the algorithmic minimum: the
    responses write Phi and K once, the fixed point reads Phi once."""
    import numpy as np
    import torch
    L = leb.lib()
    vp = lambda t: ctypes.c_void_p(t.data_ptr())
    f64 = torch.float64
    res = {}
    for U, batch in ((1, 256), (2, 256), (1, 1024)):
        p = W.sls_cfg(n_units=U, batch=batch)
        dyn = leb.dynamics_like(p.dyn)
        B, N, nx, nu = p.batch, p.N, p.dyn.nx, p.dyn.nu
        n, nw = nx + nu, nx + U
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        z, v, qx, qu = t(p.z), t(p.v), t(p.qx), t(p.qu)
        A = torch.empty((B, N, nx, nx), dtype=f64, device=dev)
        Bm = torch.empty((B, N, nx, nu), dtype=f64, device=dev)
        E = torch.empty((B, N, nx, nw), dtype=f64, device=dev)
        K = torch.zeros((B, N, N, nu, nx), dtype=f64, device=dev)
        phi = torch.zeros((B, N, N, n, nx), dtype=f64, device=dev)
        mu = torch.empty((B, N, n), dtype=f64, device=dev)
        sg = torch.empty_like(mu)
        lo = torch.empty((B, N, nx), dtype=f64, device=dev)
        hi = torch.empty_like(lo)
        cert = torch.empty((B,), dtype=torch.int32, device=dev)
        eh = (ctypes.c_double * nx)(*[float(x) for x in p.e])
        sp = ctypes.c_void_p(stream.cuda_stream)

        def lin():
            leb._check(L.leb_linearize(ctypes.byref(dyn), B, N, vp(z), vp(v), ctypes.cast(eh, ctypes.c_void_p),
                                       p.thrust, vp(A), vp(Bm), vp(E), sp))

        def resp():
            leb._check(L.leb_sls_responses(nx, nu, B, N, vp(A), vp(Bm), vp(qx), vp(qu), vp(K), vp(phi), sp))

        def fp():
            leb._check(L.leb_sls_fixed_point(ctypes.byref(dyn), B, N, vp(z), vp(v), vp(phi), nw, vp(E), p.thrust,
                                             1e-6, vp(mu), vp(sg), vp(lo), vp(hi), vp(cert), sp))

        for _ in range(2):
            lin(); resp(); fp()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        reps = 10
        acc = [0.0, 0.0, 0.0]
        for _ in range(reps):
            ev[0].record(stream); lin(); ev[1].record(stream); resp(); ev[2].record(stream); fp(); ev[3].record(stream)
            torch.cuda.synchronize()
            for i in range(3):
                acc[i] += ev[i].elapsed_time(ev[i + 1]) / reps
        pairs = B * N * (N - 1) // 2
        phi_bytes = pairs * n * nx * 8
        k_bytes = pairs * nu * nx * 8
        # FP64 flops of the recursions per (trajectory, j, k): backward P A, P B, S, Bc, P update;
        # forward K X, A + B K, (A + B K) X
        fl_step = (2 * nx ** 3 + 2 * nx * nx * nu + 2 * nu * nu * nx + 2 * nu * nx * nx + 2 * nx ** 3 +
                   2 * nx * nx * nu) + (2 * nu * nx * nx + 2 * nx * nx * nu + 2 * nx ** 3)
        total = sum(acc)
        res["chain%d_%dx40" % (U, batch)] = {
            "nx": nx, "nu": nu, "nw": nw, "ms_linearize": round(acc[0], 4), "ms_responses": round(acc[1], 4),
            "ms_fixed_point": round(acc[2], 4), "ms_update": round(total, 4),
            "step_bounds_per_s": round(B * N / (total * 1e-3), 1),
            "responses_hbm_frac": round((phi_bytes + k_bytes) / (acc[1] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "responses_fp64_frac": round(pairs * fl_step / (acc[1] * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4),
            "fixed_point_phi_read_hbm_frac": round(phi_bytes / (acc[2] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "certified": int(cert.sum().item()),
            "mean_sigma_state_certified": float(sg[cert.bool()][..., :nx].mean()) if bool(cert.any()) else None}
    return res


def interval_hessian_study(leb, W, dev, stream):
    """Tightness against the radius and time per call of the three
    interval-Hessian forms and of random sampling (10,000 points), on the
    satellite and the 3-D quadrotor: 256 local sets (z, v) + eps [-1, 1]^n
    per radius; times from HIP events over 200 calls for one local set."""
    import torch
    res = {}
    K = 10000
    gen = torch.Generator(device=dev)
    gen.manual_seed(5)
    for name, sysd in (("satellite", W.SATELLITE), ("quad3d", W.QUAD3D)):
        dyn = leb.dynamics_like(sysd)
        t = (2.0 * torch.rand((K, sysd.n), generator=gen, dtype=torch.float64, device=dev) - 1.0).contiguous()
        widths = {}
        for eps in (0.01, 0.05, 0.1, 0.15, 0.2):
            b = W.small_batch(sysd, 60, 256, eps)
            z, v, sg = (torch.from_numpy(x).to(dev) for x in (b.z, b.v, b.sigma))
            row = {}
            for mode in ("path", "expand", "classic"):
                lo, hi, fl = leb.interval_hessian_bound(dyn, z, v, sg, mode=mode, stream=stream)
                row[mode] = float((hi - lo).mean())
            slo, shi = leb.sample_remainder(dyn, z, v, sg, t, stream=stream)
            row["random_10k"] = float((shi - slo).mean())
            widths[str(eps)] = {k: float("%.4g" % x) for k, x in row.items()}
        b = W.small_batch(sysd, 61, 1, 0.1)
        z, v, sg = (torch.from_numpy(x).to(dev) for x in (b.z, b.v, b.sigma))
        times = {}
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        for label, fn in (("path", lambda: leb.interval_hessian_bound(dyn, z, v, sg, mode="path", stream=stream)),
                          ("classic", lambda: leb.interval_hessian_bound(dyn, z, v, sg, mode="classic",
                                                                         stream=stream)),
                          ("random_10k", lambda: leb.sample_remainder(dyn, z, v, sg, t, stream=stream))):
            for _ in range(3):
                fn()
            reps = 200
            e0.record(stream)
            for _ in range(reps):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            times[label] = round(e0.elapsed_time(e1) / reps * 1e3, 2)
        res[name] = {"mean_row_width": widths, "us_per_call_one_set": times}
    return res


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


# MFMA instructions per box of the MLP bound on the 16-256-256-256-12 workload
# (SQ_INSTS_MFMA / boxes, profiles/nn_chain_kernel_mlp_bound_64x50.md), each
# v_mfma_f64_16x16x4f64 2,048 FLOP; None until taken for the kernels as they are now.
NN_MFMA_INSTS_PER_BOX = 76.96e6 / 3200


def nn_roofline(leb, W, dev, stream, args):
    """MLP bound (CROWN + Theorem 2) on 64 x 50 boxes of the 16-256-256-256-12
    network: FP64 MFMA, timed with HIP events on its stream.  `achieved` counts
    the dense CROWN FLOPs (the method's work); `executed_frac` the MFMA FLOPs
    the kernels issue (stably inactive neurons skipped) against the peak."""
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
            "frac": round(achieved / FP64_PEAK_TFLOPS, 4), "flops_per_box": nn_crown_flops(widths),
            "executed_frac": None if NN_MFMA_INSTS_PER_BOX is None else
            round(NN_MFMA_INSTS_PER_BOX * 2048 * boxes / (ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4)}


def nn_adjoint_flops(widths):
    """(algorithmic, executed) FLOPs per box of the MLP bound's adjoint.
    Algorithmic: the bound's own passes (nn_crown_flops) plus the reverse of
    every pass in both modes, each as large as the pass.  Executed, dense MFMA
    form (at most three hidden layers): a forward launch for every pass (the
    output pass's too, to store its levels), the reverse of every pass, and the
    Jacobian rows once per mode; the kernels skip the stably inactive neurons'
    share of it."""
    L = len(widths) - 1
    chain = lambda k: sum(widths[k] * widths[j] * widths[j - 1] for j in range(k - 1, 0, -1))
    rev = sum(2 * chain(k) for k in range(2, L + 1))
    fwd = sum(2 * chain(k) for k in range(2, L + 1))
    executed = fwd + rev + 2 * chain(L)
    return nn_crown_flops(widths) + 2 * rev, 2 * executed


def nn_adjoint(leb, W, dev, stream):
    """Adjoint of the MLP bound (leb_nn_backward) on the 64 x 50 boxes of the
    16-256-256-256-12 network, seeds g_lo = -1, g_hi = 1 (the gradient of the
    bound's total width); FP64 MFMA products, timed with HIP events on its stream."""
    import torch
    b = W.nn_cfg()
    net = leb.MLP(b.net.W, b.net.b, b.net.nx, True)
    z = torch.from_numpy(b.z).to(dev)
    v = torch.from_numpy(b.v).to(dev)
    sg = torch.from_numpy(b.sigma).to(dev)
    boxes = b.z.shape[0] * b.z.shape[1]
    m = b.net.W[-1].shape[0]
    g_hi = torch.ones((b.z.shape[0], b.z.shape[1], m), dtype=torch.float64, device=dev)
    g_lo = -g_hi
    for _ in range(2):
        leb.nn_backward(net, z, v, sg, g_lo, g_hi, stream=stream)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reps = 5
    e0.record(stream)
    for _ in range(reps):
        leb.nn_backward(net, z, v, sg, g_lo, g_hi, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    for _ in range(2):
        leb.nn_bound(net, z, v, sg, stream=stream)
    e0.record(stream)
    for _ in range(reps):
        leb.nn_bound(net, z, v, sg, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_bound = e0.elapsed_time(e1) / reps
    net.close()
    widths = [b.net.W[0].shape[1]] + [w.shape[0] for w in b.net.W]
    alg, exe = nn_adjoint_flops(widths)
    achieved = alg * boxes / (ms * 1e-3) / 1e12
    return {"workload": "MLP-bound adjoint, 64 x 50 boxes, widths %s" % widths, "ms_per_call": round(ms, 4),
            "box_gradients_per_s": round(boxes / (ms * 1e-3), 1), "ms_bound": round(ms_bound, 4),
            "over_bound": round(ms / ms_bound, 3), "bound": "mfma", "achieved": round(achieved, 2),
            "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
            "flops_per_box": alg, "executed_flops_per_box": exe,
            "executed_frac": round(exe * boxes / (ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4)}


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

    # the same problems, one library call each, back to back on the stream
    def per_problem():
        for p in probs:
            if p["kind"] == "analytic":
                leb.analytic_bound(p["dyn"], p["z"][None], p["v"][None], p["sigma"][None], stream=stream,
                                   out={"r_lo": p["r_lo"][None], "r_hi": p["r_hi"][None], "flags": None})
            else:
                leb.nn_bound(p["net"], p["z"][None], p["v"][None], p["sigma"][None], stream=stream)
    per_problem()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(reps):
        per_problem()
    e1.record(stream)
    torch.cuda.synchronize()
    ms_pp = e0.elapsed_time(e1) / reps
    wall_pp = (time.perf_counter() - t0) / reps * 1e3
    for n in nets.values():
        n.close()
    return {"workload": "256 uneven problems, nx in {6,12,48,168}, N in 10..80, one graph launch",
            "timestep_bounds": units, "ms_per_submit": round(ms, 4),
            "timestep_bounds_per_s": round(units / (ms * 1e-3), 1), "create_s": round(create_s, 2),
            "per_problem_calls": {"ms_device": round(ms_pp, 4), "ms_host_wall": round(wall_pp, 4),
                                  "timestep_bounds_per_s": round(units / (max(ms_pp, wall_pp) * 1e-3), 1)},
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


def train_fp_surrogate(leb, W, dev, args):
    """Fixed-point-target network: features of the disturbance-only tube of
    64 other trajectories (seed 100), targets of the certified bound at their
    fixed point (71,680 node samples), trained with the library's kernels."""
    import torch
    from paper_2607_01203_amd import learned
    t0 = time.perf_counter()
    tp = W.fixed_point_cfg(seed=100, batch=64, N=40)
    b = tp.batch
    dyn = leb.dynamics_like(b.dyn)
    z = torch.from_numpy(b.z).to(dev)
    v = torch.from_numpy(b.v).to(dev)
    phi = torch.from_numpy(tp.phi).to(dev)
    mu, sg, _, _ = leb.fixed_point_solve(dyn, z, v, phi, tp.e)
    X, T = learned.chain_fp_samples(dyn, z, v, phi, tp.e, mu, sg, seed=3)
    net = leb.Surrogate(learned.CHAIN_WIDTHS, learned.he_init(learned.CHAIN_WIDTHS, 0))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    hist = learned.train(net, X, T, epochs=args.fp_epochs, batch=1024, lr=2e-3)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    return net, {"samples": int(X.shape[0]), "epochs": args.fp_epochs, "loss_first": round(hist[0], 5),
                 "loss_last": round(hist[-1], 6), "sample_s": round(t1 - t0, 2), "train_s": round(t2 - t1, 2)}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(W, tp, seconds):
    """Oracle fixed point (sequential sweep) plus its certifying sweep on a
    bounded sample of the trajectories, all host cores."""
    import numpy as np

    import oracle
    from oracle import tube

    cores = len(os.sched_getaffinity(0))
    b = tp.batch
    d = oracle.Dyn.like(b.dyn)

    def solve(idx, threads):
        # exact fixed point by one sequential sweep, then the certifying sweep
        # (F(B) inside B; equality for the exact fixed point)
        mu, sg, _, _ = tube.fixed_point(d, b.z[idx], b.v[idx], tp.phi, tp.e, threads=threads)
        lo, hi, _ = oracle.leb(d, b.z[idx], b.v[idx], sg, mu=mu, threads=threads)
        c, r = tube.zono(lo, hi)
        m2, s2 = tube.tube_map(tp.phi, tp.e, c, r)
        return tube.contains(mu, sg, m2, s2)

    def rate(threads, budget):
        t0 = time.perf_counter()
        solve(np.arange(4), threads)
        per_traj = (time.perf_counter() - t0) / 4
        count = int(max(4, min(b.z.shape[0], budget / max(per_traj, 1e-6))))
        t0 = time.perf_counter()
        ok = solve(np.arange(count), threads)
        dt = time.perf_counter() - t0
        return count, dt, bool(ok.all())

    N = b.z.shape[1]
    count, dt, ok = rate(cores, seconds)
    c1, dt1, ok1 = rate(1, 0.4 * seconds)
    return {"value": round(count * N / dt, 2), "unit": "timestep-bounds/s", "cores": cores, "kind": "oracle",
            "sample": "%d of %d trajectories (N=%d, nx=168), exact fixed point + certifying sweep, %.1f s"
                      % (count, b.z.shape[0], N, dt),
            "certified": ok and ok1, "cpu_model": cpu_model(),
            "single_thread": {"value": round(c1 * N / dt1, 2), "cores": 1,
                              "sample": "%d trajectories, %.1f s" % (c1, dt1)}}


if __name__ == "__main__":
    main()
