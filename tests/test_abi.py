"""Host-side checks of the C ABI: the library loads, exports every symbol
that include/leb.h declares, and rejects bad arguments before touching the
device (these calls return before any HIP call)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w\s\*]*?\b(leb_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def L():
    import paper_2607_01203_amd as leb
    if not os.path.exists(leb.LIB_PATH):
        pytest.fail("libleb.so missing: run __graft_entry__.build() first")
    return leb.lib()


def test_header_declares_entry_points():
    names = _declared_symbols()
    assert "leb_analytic_bound" in names and "leb_strerror" in names


def test_library_exports_every_declared_symbol(L):
    for name in _declared_symbols():
        assert hasattr(L, name), name


def test_strerror_and_version(L):
    assert L.leb_strerror(0) == b"ok"
    assert L.leb_strerror(-1) == b"invalid argument"
    assert L.leb_version().startswith(b"leb-mi355x")


def _call(L, dyn, batch=1, N=1, z=8, v=8, mu=None, sigma=8, lo=8, hi=8, cb=None, rb=None, pad=0.0, flags=None,
          A=None, B=None):
    vp = lambda x: None if x is None else ctypes.c_void_p(x)
    return L.leb_analytic_bound(None if dyn is None else ctypes.byref(dyn), batch, N, vp(z), vp(v), vp(mu),
                                vp(sigma), vp(lo), vp(hi), vp(cb), vp(rb), pad, vp(flags), vp(A), vp(B), None)


def test_rejects_bad_arguments_without_launching(L):
    import paper_2607_01203_amd as leb
    d = leb.chain_dynamics(2)
    assert _call(L, None) == -1
    assert _call(L, d, batch=-1) == -1
    assert _call(L, d, N=-3) == -1
    assert _call(L, d, z=None) == -1                 # required pointer
    assert _call(L, d, sigma=None) == -1
    assert _call(L, d, lo=None) == -1
    assert _call(L, d, z=12) == -1                   # misaligned FP64 pointer
    assert _call(L, d, cb=8) == -1                   # c_bar without rho_bar
    assert _call(L, d, pad=-1.0) == -1
    bad = leb.chain_dynamics(2)
    bad.nx = 7
    assert _call(L, bad) == -1
    bad = leb.chain_dynamics(2, dt=0.0)
    assert _call(L, bad) == -1
    bad = leb.chain_dynamics(2, m=-1.0)
    assert _call(L, bad) == -1
    bad = leb.chain_dynamics(2, k_spring=-2.0)
    assert _call(L, bad) == -1
    bad = leb.chain_dynamics(300)
    assert _call(L, bad) == -4
    bad = leb.chain_dynamics(2)
    bad.kind = 17
    assert _call(L, bad) == -4
    assert _call(L, d, A=8) == -1                    # A without B
    assert _call(L, d, A=8, B=12) == -1              # misaligned B


def test_test_kinds_reject_bad_arguments_without_launching(L):
    import paper_2607_01203_amd as leb
    lin = leb.linear_dynamics(3, 1)
    assert _call(L, lin, sigma=None) == -1           # the linear kind validates its data too
    assert _call(L, lin, z=None) == -1
    assert _call(L, lin, A=8, B=8) == -1             # Jacobians: chain dynamics only
    q = leb.Dynamics(leb.DYN_QUADRATIC, 3, 1, 0, 0, 0, 0, 0, 0, 0, 0, None)
    assert _call(L, q) == -1                         # no Q
    q.coeffs = 12
    assert _call(L, q) == -1                         # misaligned Q
    q.coeffs = 8
    q.nx, q.nu = 60, 8
    assert _call(L, q) == -4                         # n > 64
    s = leb.sincos_dynamics(2)
    s.nu = 1
    assert _call(L, s) == -1
    s = leb.sincos_dynamics(3)
    assert _call(L, s) == -1
    assert _call(L, leb.sincos_dynamics(1), batch=0, z=None, v=None, sigma=None, lo=None, hi=None) == 0


def test_zonotope_hull_rejects_bad_arguments_without_launching(L):
    vp = ctypes.c_void_p
    assert L.leb_zonotope_hull(-1, 3, vp(8), None, vp(8), vp(8), None) == -1
    assert L.leb_zonotope_hull(2, -1, vp(8), None, vp(8), vp(8), None) == -1
    assert L.leb_zonotope_hull(2, 3, None, None, vp(8), vp(8), None) == -1     # no G
    assert L.leb_zonotope_hull(2, 3, vp(8), None, None, vp(8), None) == -1     # no mu
    assert L.leb_zonotope_hull(2, 3, vp(12), None, vp(8), vp(8), None) == -1   # misaligned
    assert L.leb_zonotope_hull(0, 3, None, None, None, None, None) == 0


def test_nn_bound_rejects_misaligned_jacobian_without_launching(L):
    vp = ctypes.c_void_p
    # leb_nn_bound(net, batch, N, z, v, mu, sigma, J, r_lo, r_hi, c_bar, rho_bar, pad, flags, stream):
    # a NULL network is refused first
    assert L.leb_nn_bound(None, 1, 1, vp(8), vp(8), None, vp(8), vp(12), vp(8), vp(8), None, None, 0.0, None,
                          None) == -1


def test_nn_backward_rejects_null_network_without_launching(L):
    vp = ctypes.c_void_p
    # leb_nn_backward(net, batch, N, z, v, mu, sigma, g_lo, g_hi, gz, gv, gmu, gsigma, stream)
    assert L.leb_nn_backward(None, 1, 1, vp(8), vp(8), None, vp(8), vp(8), vp(8), vp(8), vp(8), None, vp(8),
                             None) == -1


def test_empty_problem_is_ok_without_launching(L):
    import paper_2607_01203_amd as leb
    d = leb.chain_dynamics(3)
    assert _call(L, d, batch=0, N=5, z=None, v=None, sigma=None, lo=None, hi=None) == 0
    assert _call(L, d, batch=4, N=0, z=None, v=None, sigma=None, lo=None, hi=None) == 0


def test_nn_surrogate_entry_points_reject_bad_arguments_without_launching(L):
    vp = ctypes.c_void_p(8)
    # leb_nn_features(nx, nu, batch, N, z, v, mu, sigma, x, stream)
    assert L.leb_nn_features(0, 4, 1, 1, vp, vp, None, vp, vp, None) != 0
    assert L.leb_nn_features(12, -1, 1, 1, vp, vp, None, vp, vp, None) != 0
    assert L.leb_nn_features(100, 29, 1, 1, vp, vp, None, vp, vp, None) != 0     # 2n > 256
    assert L.leb_nn_features(12, 4, 1, 1, vp, vp, None, None, vp, None) != 0    # no sigma
    assert L.leb_nn_features(12, 4, 1, 1, vp, vp, None, vp, ctypes.c_void_p(12), None) != 0  # misaligned x
    assert L.leb_nn_features(12, 4, 0, 5, None, None, None, None, None, None) == 0
    # leb_nn_targets(m, batch, N, r_lo, r_hi, t, stream)
    assert L.leb_nn_targets(0, 1, 1, vp, vp, vp, None) != 0
    assert L.leb_nn_targets(129, 1, 1, vp, vp, vp, None) != 0
    assert L.leb_nn_targets(12, 1, 1, vp, None, vp, None) != 0
    assert L.leb_nn_targets(12, 3, 0, None, None, None, None) == 0
    # leb_nn_surrogate_bound(net, nx, nu, batch, N, z, v, mu, sigma, r_lo, r_hi, stream)
    assert L.leb_nn_surrogate_bound(None, 12, 4, 1, 1, vp, vp, None, vp, vp, vp, None) != 0


def test_binding_refuses_cpu_tensors():
    import torch
    import paper_2607_01203_amd as leb
    d = leb.chain_dynamics(1)
    z = torch.zeros((1, 2, 6), dtype=torch.float64)
    with pytest.raises(leb.LebError):
        leb.analytic_bound(d, z, torch.zeros((1, 2, 2), dtype=torch.float64),
                           torch.zeros((1, 2, 8), dtype=torch.float64),
                           out={"r_lo": z, "r_hi": z, "flags": torch.zeros((1, 2), dtype=torch.int32)})


def test_fixed_point_rejects_bad_options_without_launching(L):
    """Options are checked before anything touches a device: a tolerance below
    zero, no sweeps or no absolute inflation is LEB_EINVAL (-1)."""
    import ctypes
    import paper_2607_01203_amd as leb
    d = leb.chain_dynamics(2)
    e = (ctypes.c_double * 6)(*([0.0] * 3 + [0.01, 0.01, 0.0]))
    sw = ctypes.c_int32(7)
    vp = ctypes.c_void_p(8)

    def call(**kw):
        o = dict(tol=1e-6, max_sweeps=10, pad=0.0, inflate_abs=1e-12, warm=0, conv_tol=1e-6)
        o.update(kw)
        opt = leb.FPOptions(o["tol"], o["max_sweeps"], o["pad"], o["inflate_abs"], o["warm"], o["conv_tol"])
        return L.leb_fixed_point_solve(ctypes.byref(d), 4, 3, vp, vp, vp, e, ctypes.byref(opt), vp, vp, vp,
                                       ctypes.byref(sw), None)

    L.leb_fixed_point_solve.restype = ctypes.c_int
    assert call(tol=-1.0) == -1
    assert call(max_sweeps=0) == -1
    assert call(inflate_abs=0.0) == -1
    assert call(pad=-1.0) == -1
    assert call(conv_tol=1e-7) == -1          # convergence tolerance below the inflation
    assert call(conv_tol=float("nan")) == -1
    # a horizon beyond what the compact tube map keeps in LDS: LEB_ENOTSUP (-4)
    opt = leb.FPOptions(1e-6, 10, 0.0, 1e-12, 0, 1e-6)
    assert L.leb_fixed_point_solve(ctypes.byref(d), 4, 211, vp, vp, vp, e, ctypes.byref(opt), vp, vp, vp,
                                   ctypes.byref(sw), None) == -4
    # the learned form checks the same options before its surrogate sweeps (the
    # network handle is not touched on these paths)
    ws = leb.WarmStart(ctypes.c_void_p(8), 1, 0.05)

    def learned(N=3, **kw):
        o = dict(tol=1e-6, max_sweeps=10, pad=0.0, inflate_abs=1e-12, warm=0, conv_tol=1e-6)
        o.update(kw)
        opt = leb.FPOptions(o["tol"], o["max_sweeps"], o["pad"], o["inflate_abs"], o["warm"], o["conv_tol"])
        return L.leb_fixed_point_learned(ctypes.byref(d), 4, N, vp, vp, vp, e, ctypes.byref(opt), ctypes.byref(ws),
                                         vp, vp, vp, ctypes.byref(sw), None)

    assert learned(tol=-1.0) == -1
    assert learned(max_sweeps=0) == -1
    assert learned(inflate_abs=0.0) == -1
    assert learned(conv_tol=0.0) == -1
    assert learned(N=211) == -4
    # zero work: accepted without a launch
    opt = leb.FPOptions(1e-6, 10, 0.0, 1e-12, 0, 1e-6)
    assert L.leb_fixed_point_solve(ctypes.byref(d), 0, 3, None, None, None, e, ctypes.byref(opt), None, None, None,
                                   ctypes.byref(sw), None) == 0
    assert sw.value == 0


def test_sample_cache_round_trip(tmp_path):
    import numpy as np
    import torch
    from paper_2607_01203_amd import learned
    rng = np.random.default_rng(0)
    X = torch.from_numpy(rng.normal(size=(10, 32)).astype(np.float32))
    T = torch.from_numpy(rng.normal(size=(10, 24)).astype(np.float32))
    p = str(tmp_path / "samples.npz")
    learned.save_samples(p, X, T)
    X2, T2 = learned.load_samples(p, device="cpu")
    assert torch.equal(X, X2) and torch.equal(T, T2)
    np.savez(p, X=np.zeros((3, 2)), T=np.zeros((4, 2), dtype=np.float32))
    with pytest.raises(ValueError):
        learned.load_samples(p, device="cpu")


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus above 1 exits with a message and
    status 2 before touching a device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_sls_entry_points_reject_bad_arguments_without_launching(L):
    import paper_2607_01203_amd as leb
    vp = ctypes.c_void_p(8)
    mis = ctypes.c_void_p(12)
    # leb_sls_responses(nx, nu, batch, N, A, B, qx, qu, K, phi, stream)
    assert L.leb_sls_responses(0, 2, 1, 4, vp, vp, vp, vp, vp, vp, None) == -1
    assert L.leb_sls_responses(33, 2, 1, 4, vp, vp, vp, vp, vp, vp, None) == -1     # nx > 32
    assert L.leb_sls_responses(6, 0, 1, 4, vp, vp, vp, vp, vp, vp, None) == -1      # no input
    assert L.leb_sls_responses(6, 17, 1, 4, vp, vp, vp, vp, vp, vp, None) == -1     # nu > 16
    assert L.leb_sls_responses(6, 2, 1, 4, vp, vp, None, vp, vp, vp, None) == -1    # no weights
    assert L.leb_sls_responses(6, 2, 1, 4, vp, vp, vp, vp, vp, mis, None) == -1     # misaligned phi
    assert L.leb_sls_responses(6, 2, 70000, 4, vp, vp, vp, vp, vp, vp, None) == -4
    assert L.leb_sls_responses(6, 2, 0, 4, None, None, None, None, None, None, None) == 0
    # leb_sls_tube_map(nx, nu, nw, batch, N, phi, E, c_bar, rho_bar, mu, sigma, stream)
    assert L.leb_sls_tube_map(6, 2, 65, 1, 4, vp, vp, vp, vp, vp, vp, None) == -1   # nw > 64
    assert L.leb_sls_tube_map(6, 2, 7, 1, 4, vp, None, vp, vp, vp, vp, None) == -1  # no E
    assert L.leb_sls_tube_map(6, 2, 0, 1, 4, vp, None, vp, None, vp, vp, None) == -1  # no rho_bar
    assert L.leb_sls_tube_map(6, 2, 7, 1, 4, vp, vp, vp, vp, mis, vp, None) == -1
    assert L.leb_sls_tube_map(6, 2, 7, 3, 0, None, None, None, None, None, None, None) == 0
    # leb_sls_fixed_point(dyn, batch, N, z, v, phi, nw, E, thrust, pad, mu, sigma, r_lo, r_hi, cert, stream)
    d = leb.chain_dynamics(1)
    fp = L.leb_sls_fixed_point
    assert fp(ctypes.byref(d), 1, 4, vp, vp, vp, 7, vp, 0.1, -1.0, vp, vp, None, None, None, None) == -1  # pad
    assert fp(ctypes.byref(d), 1, 4, vp, vp, vp, 7, vp, -0.1, 0.0, vp, vp, None, None, None, None) == -1  # thrust
    assert fp(ctypes.byref(d), 1, 4, vp, vp, vp, 0, None, 0.1, 0.0, vp, vp, None, None, None, None) == -1  # nw < U
    assert fp(ctypes.byref(d), 1, 4, vp, vp, vp, 7, vp, 0.0, 0.0, vp, vp, vp, None, None, None) == -1  # r_lo only
    assert fp(ctypes.byref(d), 1, 4, vp, vp, vp, 7, vp, 0.0, 0.0, vp, vp, None, None, ctypes.c_void_p(6),
              None) == -1                                                                          # misaligned flags
    sat = leb.satellite_dynamics(0.1)
    assert fp(ctypes.byref(sat), 1, 4, vp, vp, vp, 7, vp, 0.1, 0.0, vp, vp, None, None, None, None) == -1
    assert fp(ctypes.byref(leb.linear_dynamics(3, 1)), 1, 4, vp, vp, vp, 3, vp, 0.0, 0.0, vp, vp, None, None,
              None, None) == -4
    big = leb.chain_dynamics(6)                       # nx = 36 > 32
    assert fp(ctypes.byref(big), 1, 4, vp, vp, vp, 36, vp, 0.0, 0.0, vp, vp, None, None, None, None) == -1
    assert fp(ctypes.byref(d), 0, 4, None, None, None, 7, None, 0.0, 0.0, None, None, None, None, None, None) == 0
    # leb_linearize(dyn, batch, N, z, v, e, thrust, A, B, E, stream)
    e = (ctypes.c_double * 6)(0.0, 0.0, 0.0, -1.0, 0.0, 0.0)
    assert L.leb_linearize(ctypes.byref(d), 1, 4, vp, vp, ctypes.cast(e, ctypes.c_void_p), 0.1, vp, vp, vp,
                           None) == -1                                                            # e < 0
    assert L.leb_linearize(ctypes.byref(d), 1, 4, vp, vp, None, 0.1, vp, vp, vp, None) == -1        # E without e
    assert L.leb_linearize(ctypes.byref(d), 1, 4, vp, vp, None, -1.0, vp, vp, None, None) == -1
    assert L.leb_linearize(ctypes.byref(sat), 1, 4, vp, vp, None, 0.0, vp, vp, None, None) == -4
