"""MI355X (gfx950) linearization-error bounds: Python binding of libleb.so.

The binding only marshals arguments: every step of the bound runs in the
HIP kernels of libleb.so.  PyTorch provides device memory and streams.
There is no CPU fallback: if the library is missing or a call fails, an
exception is raised.
"""
from __future__ import annotations

import ctypes
import os

__all__ = ["lib", "Dynamics", "LebError", "analytic_bound", "chain_dynamics", "linear_dynamics", "quadratic_dynamics",
           "sincos_dynamics", "tube_map", "zonotope_hull", "fixed_point_solve", "FLAG_UNBOUNDED",
           "FLAG_BAD_INPUT", "FLAG_HULL_EXTENDED", "DYN_LINEAR", "DYN_QUADRATIC", "DYN_SINCOS", "DYN_PQUAD_CHAIN",
           "DYN_SATELLITE", "DYN_QUAD3D", "IH_MODES"]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libleb.so")

FLAG_UNBOUNDED, FLAG_BAD_INPUT, FLAG_HULL_EXTENDED = 1, 2, 4
DYN_LINEAR, DYN_QUADRATIC, DYN_SINCOS, DYN_PQUAD_CHAIN, DYN_SATELLITE, DYN_QUAD3D = 0, 1, 2, 4, 5, 6
IH_MODES = {"path": 0, "expand": 1, "classic": 2}

_lib = None


class LebError(RuntimeError):
    pass


class Dynamics(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("nx", ctypes.c_int32), ("nu", ctypes.c_int32),
                ("n_units", ctypes.c_int32), ("dt", ctypes.c_double), ("m", ctypes.c_double),
                ("g", ctypes.c_double), ("arm", ctypes.c_double), ("inertia", ctypes.c_double),
                ("k_spring", ctypes.c_double), ("rest_len", ctypes.c_double), ("coeffs", ctypes.c_void_p),
                ("J", ctypes.c_double * 3)]


class WarmStart(ctypes.Structure):
    _fields_ = [("net", ctypes.c_void_p), ("sweeps", ctypes.c_int32), ("margin", ctypes.c_double)]


CHAIN_FEATURES = 32
CHAIN_OUTPUTS = 4


class Problem(ctypes.Structure):
    _fields_ = [("type", ctypes.c_int32), ("dyn", ctypes.POINTER(Dynamics)), ("net", ctypes.c_void_p),
                ("N", ctypes.c_int32), ("z", ctypes.c_void_p), ("v", ctypes.c_void_p), ("mu", ctypes.c_void_p),
                ("sigma", ctypes.c_void_p), ("r_lo", ctypes.c_void_p), ("r_hi", ctypes.c_void_p)]


PROBLEM_ANALYTIC = 0
PROBLEM_NN = 1


class FPOptions(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_sweeps", ctypes.c_int32), ("pad", ctypes.c_double),
                ("inflate_abs", ctypes.c_double), ("warm", ctypes.c_int32), ("conv_tol", ctypes.c_double)]


def chain_dynamics(n_units, dt=0.05, m=1.0, g=9.81, arm=0.25, inertia=0.01, k_spring=2.0,
                   rest_len=1.0) -> Dynamics:
    return Dynamics(DYN_PQUAD_CHAIN, 6 * n_units, 2 * n_units, n_units, dt, m, g, arm, inertia,
                    k_spring, rest_len, None)


def linear_dynamics(nx, nu=0) -> Dynamics:
    """Affine dynamics: the remainder is identically 0."""
    return Dynamics(DYN_LINEAR, int(nx), int(nu), 0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, None)


def quadratic_dynamics(Q, nu=0) -> Dynamics:
    """f_l(a) = 1/2 a^T Q_l a + affine, Q a float64 GPU tensor [nx][n][n]
    (kept alive by the returned object while it is in use)."""
    import torch
    Q = Q.contiguous()
    nx, n = int(Q.shape[0]), int(Q.shape[1])
    d = Dynamics(DYN_QUADRATIC, nx, n - nx if nu is None else int(nu), 0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0,
                 _dev_ptr(Q, "Q", torch.float64).value)
    d._Q = Q
    return d


def sincos_dynamics(nx) -> Dynamics:
    """nx = 1: f = sin(a_1); nx = 2: f = (sin a_1 cos a_2, cos a_1 sin a_2)."""
    return Dynamics(DYN_SINCOS, int(nx), 0, 0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, None)


def satellite_dynamics(dt, inertia=(5.0, 2.0, 1.0)) -> Dynamics:
    """Satellite attitude (quaternion, body rates; torques): nx = 7, nu = 3."""
    return Dynamics(DYN_SATELLITE, 7, 3, 0, float(dt), 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, None,
                    (ctypes.c_double * 3)(*inertia))


def quad3d_dynamics(dt, m, g, J) -> Dynamics:
    """3-D quadrotor (position, Euler angles, velocity, body rates; thrust, torques): nx = 12, nu = 4."""
    return Dynamics(DYN_QUAD3D, 12, 4, 0, float(dt), float(m), float(g), 0.0, 0.0, 0.0, 0.0, None,
                    (ctypes.c_double * 3)(*J))


def dynamics_like(obj) -> Dynamics:
    """From any object exposing n_units, dt, m, g, arm, inertia, k_spring, rest_len
    (a chain), or kind "satellite" / "quad3d" with dt, m, g, J."""
    kind = getattr(obj, "kind", "chain")
    if kind == "satellite":
        return satellite_dynamics(obj.dt, obj.J)
    if kind == "quad3d":
        return quad3d_dynamics(obj.dt, obj.m, obj.g, obj.J)
    return chain_dynamics(obj.n_units, obj.dt, obj.m, obj.g, obj.arm, obj.inertia, obj.k_spring,
                          obj.rest_len)


def lib():
    """Load libleb.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LebError("libleb.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        L.leb_analytic_bound.argtypes = [ctypes.POINTER(Dynamics), ctypes.c_int32, ctypes.c_int32,
                                         vp, vp, vp, vp, vp, vp, vp, vp, ctypes.c_double, vp, vp, vp, vp]
        L.leb_analytic_bound.restype = ctypes.c_int
        L.leb_backward.argtypes = [ctypes.POINTER(Dynamics), ctypes.c_int32, ctypes.c_int32] + [vp] * 11
        L.leb_backward.restype = ctypes.c_int
        L.leb_mlp_create.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.POINTER(ctypes.c_float)),
                                     ctypes.POINTER(ctypes.POINTER(ctypes.c_float)), ctypes.c_int32, ctypes.c_int32,
                                     ctypes.POINTER(ctypes.c_void_p)]
        L.leb_mlp_create.restype = ctypes.c_int
        L.leb_mlp_destroy.argtypes = [ctypes.c_void_p]
        L.leb_mlp_destroy.restype = ctypes.c_int
        L.leb_nn_bound.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32] + [vp] * 9 + [ctypes.c_double, vp, vp]
        L.leb_nn_bound.restype = ctypes.c_int
        L.leb_nn_backward.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32] + [vp] * 11
        L.leb_nn_backward.restype = ctypes.c_int
        L.leb_tube_map.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp,
                                   ctypes.POINTER(ctypes.c_double), vp, vp, vp, vp, vp]
        L.leb_tube_map.restype = ctypes.c_int
        L.leb_zonotope_hull.argtypes = [ctypes.c_int32, ctypes.c_int32, vp, vp, vp, vp, vp]
        L.leb_zonotope_hull.restype = ctypes.c_int
        L.leb_interval_hessian_bound.argtypes = [ctypes.POINTER(Dynamics), ctypes.c_int32, ctypes.c_int32,
                                                 ctypes.c_int32, vp, vp, vp, vp, vp, vp, vp, vp]
        L.leb_interval_hessian_bound.restype = ctypes.c_int
        L.leb_sample_remainder.argtypes = [ctypes.POINTER(Dynamics), ctypes.c_int32, ctypes.c_int32, vp, vp, vp, vp,
                                           ctypes.c_int32, vp, vp, vp, vp]
        L.leb_sample_remainder.restype = ctypes.c_int
        L.leb_pgd_nominal.argtypes = [ctypes.POINTER(Dynamics), ctypes.c_int32, ctypes.c_int32, vp, vp, vp, vp,
                                      ctypes.c_int32, ctypes.c_double, ctypes.c_int32, ctypes.c_double, vp, vp, vp,
                                      vp, vp]
        L.leb_pgd_nominal.restype = ctypes.c_int
        L.leb_launch_timing.argtypes = [ctypes.c_int32]
        L.leb_launch_timing.restype = ctypes.c_int
        L.leb_launch_times.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_float), ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_int32)]
        L.leb_launch_times.restype = ctypes.c_int
        L.leb_fixed_point_solve.argtypes = [ctypes.POINTER(Dynamics), ctypes.c_int32, ctypes.c_int32, vp, vp,
                                            vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(FPOptions),
                                            vp, vp, vp, ctypes.POINTER(ctypes.c_int32), vp]
        L.leb_fixed_point_solve.restype = ctypes.c_int
        L.leb_fixed_point_solve_noalloc.argtypes = L.leb_fixed_point_solve.argtypes
        L.leb_fixed_point_solve_noalloc.restype = ctypes.c_int
        f32 = ctypes.c_float
        L.leb_surrogate_create.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), vp,
                                           ctypes.POINTER(ctypes.c_void_p)]
        L.leb_surrogate_create.restype = ctypes.c_int
        L.leb_surrogate_destroy.argtypes = [vp]
        L.leb_surrogate_destroy.restype = ctypes.c_int
        L.leb_surrogate_n_params.argtypes = [vp]
        L.leb_surrogate_n_params.restype = ctypes.c_int64
        L.leb_surrogate_params.argtypes = [vp, vp]
        L.leb_surrogate_params.restype = ctypes.c_int
        L.leb_mlp_fwd_bf16.argtypes = [vp, ctypes.c_int32, vp, vp, vp]
        L.leb_mlp_fwd_bf16.restype = ctypes.c_int
        L.leb_mlp_bwd_bf16.argtypes = [vp, ctypes.c_int32, vp, vp, vp, vp]
        L.leb_mlp_bwd_bf16.restype = ctypes.c_int
        f64c = ctypes.c_double
        L.leb_adam_step.argtypes = [vp, vp, ctypes.c_int32, f64c, f64c, f64c, f64c, vp]
        L.leb_adam_step.restype = ctypes.c_int
        L.leb_surrogate_train_step.argtypes = [vp, ctypes.c_int32, vp, vp, ctypes.c_int32, ctypes.c_double, vp, vp]
        L.leb_surrogate_train_step.restype = ctypes.c_int
        L.leb_surrogate_dims.argtypes = [vp, vp, vp]
        L.leb_surrogate_dims.restype = ctypes.c_int
        L.leb_chain_features.argtypes = [ctypes.POINTER(Dynamics), ctypes.c_int32, ctypes.c_int32] + [vp] * 6
        L.leb_chain_features.restype = ctypes.c_int
        L.leb_chain_targets.argtypes = [ctypes.POINTER(Dynamics), ctypes.c_int32, ctypes.c_int32] + [vp] * 4
        L.leb_chain_targets.restype = ctypes.c_int
        L.leb_fixed_point_learned.argtypes = [ctypes.POINTER(Dynamics), ctypes.c_int32, ctypes.c_int32, vp, vp,
                                              vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(FPOptions),
                                              ctypes.POINTER(WarmStart), vp, vp, vp, ctypes.POINTER(ctypes.c_int32),
                                              vp]
        L.leb_fixed_point_learned.restype = ctypes.c_int
        L.leb_batch_create.argtypes = [vp, ctypes.c_int32, ctypes.c_char_p, ctypes.POINTER(ctypes.c_void_p)]
        L.leb_batch_create.restype = ctypes.c_int
        L.leb_batch_submit.argtypes = [vp, vp]
        L.leb_batch_submit.restype = ctypes.c_int
        L.leb_batch_destroy.argtypes = [vp]
        L.leb_batch_destroy.restype = ctypes.c_int
        L.leb_batch_info.argtypes = [vp, ctypes.c_char_p, ctypes.c_int32]
        L.leb_batch_info.restype = ctypes.c_int
        L.leb_chain_surrogate_bound.argtypes = [ctypes.POINTER(Dynamics), ctypes.c_int32, ctypes.c_int32] + \
            [vp] * 5 + [vp, vp, ctypes.c_double, vp]
        L.leb_chain_surrogate_bound.restype = ctypes.c_int
        i32 = ctypes.c_int32
        L.leb_nn_features.argtypes = [i32, i32, i32, i32] + [vp] * 6
        L.leb_nn_features.restype = ctypes.c_int
        L.leb_nn_targets.argtypes = [i32, i32, i32] + [vp] * 4
        L.leb_nn_targets.restype = ctypes.c_int
        L.leb_nn_surrogate_bound.argtypes = [vp, i32, i32, i32, i32] + [vp] * 7
        L.leb_nn_surrogate_bound.restype = ctypes.c_int
        f64c_ = ctypes.c_double
        L.leb_linearize.argtypes = [ctypes.POINTER(Dynamics), i32, i32, vp, vp, vp, f64c_, vp, vp, vp, vp]
        L.leb_linearize.restype = ctypes.c_int
        L.leb_sls_responses.argtypes = [i32, i32, i32, i32] + [vp] * 7
        L.leb_sls_responses.restype = ctypes.c_int
        L.leb_sls_tube_map.argtypes = [i32, i32, i32, i32, i32] + [vp] * 7
        L.leb_sls_tube_map.restype = ctypes.c_int
        L.leb_sls_fixed_point.argtypes = [ctypes.POINTER(Dynamics), i32, i32, vp, vp, vp, i32, vp, f64c_, f64c_] + \
            [vp] * 6
        L.leb_sls_fixed_point.restype = ctypes.c_int
        L.leb_strerror.argtypes = [ctypes.c_int]
        L.leb_strerror.restype = ctypes.c_char_p
        L.leb_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise LebError("libleb: %s (%d)" % (lib().leb_strerror(rc).decode(), rc))


def _dev_ptr(t, name, dtype=None):
    if t is None:
        return None
    import torch
    if not t.is_cuda:
        raise LebError("%s must be a GPU tensor" % name)
    if dtype is not None and t.dtype != dtype:
        raise LebError("%s must be %s" % (name, dtype))
    if not t.is_contiguous():
        raise LebError("%s must be contiguous" % name)
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def analytic_bound(dyn: Dynamics, z, v, sigma, mu=None, pad: float = 0.0, zonotope: bool = False,
                   jacobians: bool = False, stream=None, out=None):
    """Path-based Hessian bound for every (trajectory, timestep).

    z [B][N][nx], v [B][N][nu], sigma (and mu) [B][N][nx+nu]: float64 GPU
    tensors.  Returns dict with r_lo, r_hi [B][N][nx], flags [B][N] (int32
    view of the uint32 flags), if zonotope c_bar and rho_bar, and if
    jacobians the point Jacobians A [B][N][nx][nx], B [B][N][nx][nu]."""
    import torch
    B, N = int(z.shape[0]), int(z.shape[1])
    f64 = torch.float64
    if out is None:
        out = {"r_lo": torch.empty((B, N, dyn.nx), dtype=f64, device=z.device),
               "r_hi": torch.empty((B, N, dyn.nx), dtype=f64, device=z.device),
               "flags": torch.empty((B, N), dtype=torch.int32, device=z.device)}
        if zonotope:
            out["c_bar"] = torch.empty((B, N, dyn.nx), dtype=f64, device=z.device)
            out["rho_bar"] = torch.empty((B, N, dyn.nx), dtype=f64, device=z.device)
        if jacobians:
            out["A"] = torch.empty((B, N, dyn.nx, dyn.nx), dtype=f64, device=z.device)
            out["B"] = torch.empty((B, N, dyn.nx, dyn.nu), dtype=f64, device=z.device)
    rc = lib().leb_analytic_bound(
        ctypes.byref(dyn), B, N, _dev_ptr(z, "z", f64), _dev_ptr(v, "v", f64), _dev_ptr(mu, "mu", f64),
        _dev_ptr(sigma, "sigma", f64), _dev_ptr(out.get("r_lo"), "r_lo", f64), _dev_ptr(out.get("r_hi"), "r_hi", f64),
        _dev_ptr(out.get("c_bar"), "c_bar", f64), _dev_ptr(out.get("rho_bar"), "rho_bar", f64),
        float(pad), _dev_ptr(out.get("flags"), "flags"), _dev_ptr(out.get("A"), "A", f64),
        _dev_ptr(out.get("B"), "B", f64), _stream(stream))
    _check(rc)
    return out


def pgd_nominal(dyn: Dynamics, z0, v0, sigma, mu0=None, radius=0.5, steps=20, lr=0.25, fixed_box=False,
                stream=None):
    """Linearization point refined by projected gradient descent on the
    bound's width (see leb.h: leb_pgd_nominal).  Returns (z, v, width, width0)."""
    import torch
    f64 = torch.float64
    B, N = int(z0.shape[0]), int(z0.shape[1])
    z = torch.empty_like(z0)
    v = torch.empty_like(v0)
    w = torch.empty((B, N), dtype=f64, device=z0.device)
    w0 = torch.empty((B, N), dtype=f64, device=z0.device)
    _check(lib().leb_pgd_nominal(ctypes.byref(dyn), B, N, _dev_ptr(z0, "z0", f64), _dev_ptr(v0, "v0", f64),
                                 _dev_ptr(mu0, "mu0", f64), _dev_ptr(sigma, "sigma", f64), int(bool(fixed_box)),
                                 float(radius), int(steps), float(lr),
                                 _dev_ptr(z, "z", f64), _dev_ptr(v, "v", f64), _dev_ptr(w, "width", f64),
                                 _dev_ptr(w0, "width0", f64), _stream(stream)))
    return z, v, w, w0


def interval_hessian_bound(dyn: Dynamics, z, v, sigma, mu=None, mode="path", stream=None):
    """One of the three interval-Hessian enclosures (see leb.h:
    leb_interval_hessian_bound): mode "path" (Theorem 1), "expand" or
    "classic".  Returns (r_lo, r_hi, flags)."""
    import torch
    f64 = torch.float64
    B, N = int(z.shape[0]), int(z.shape[1])
    lo = torch.empty((B, N, dyn.nx), dtype=f64, device=z.device)
    hi = torch.empty_like(lo)
    fl = torch.empty((B, N), dtype=torch.int32, device=z.device)
    _check(lib().leb_interval_hessian_bound(ctypes.byref(dyn), IH_MODES[mode], B, N, _dev_ptr(z, "z", f64),
                                            _dev_ptr(v, "v", f64), _dev_ptr(mu, "mu", f64),
                                            _dev_ptr(sigma, "sigma", f64), _dev_ptr(lo, "r_lo", f64),
                                            _dev_ptr(hi, "r_hi", f64), _dev_ptr(fl, "flags"), _stream(stream)))
    return lo, hi, fl


def sample_remainder(dyn: Dynamics, z, v, sigma, t, mu=None, stream=None):
    """Minimum and maximum of the true remainder over the points
    a~ + mu + t_s * sigma (t [K][nx+nu] in [-1, 1], a float64 GPU tensor) and
    the nominal (see leb.h: leb_sample_remainder).  Returns (s_lo, s_hi)."""
    import torch
    f64 = torch.float64
    B, N = int(z.shape[0]), int(z.shape[1])
    lo = torch.empty((B, N, dyn.nx), dtype=f64, device=z.device)
    hi = torch.empty_like(lo)
    _check(lib().leb_sample_remainder(ctypes.byref(dyn), B, N, _dev_ptr(z, "z", f64), _dev_ptr(v, "v", f64),
                                      _dev_ptr(mu, "mu", f64), _dev_ptr(sigma, "sigma", f64), int(t.shape[0]),
                                      _dev_ptr(t, "t", f64), _dev_ptr(lo, "s_lo", f64), _dev_ptr(hi, "s_hi", f64),
                                      _stream(stream)))
    return lo, hi


def linearize(dyn: Dynamics, z, v, e=None, thrust=0.0, stream=None):
    """Point Jacobians A, B and, when e is given (nx values), the disturbance
    matrices E(z_k) of the thrust model (see leb.h: leb_linearize).
    Returns (A, B, E or None)."""
    import torch
    f64 = torch.float64
    B_, N = int(z.shape[0]), int(z.shape[1])
    nx, nu = dyn.nx, dyn.nu
    A = torch.empty((B_, N, nx, nx), dtype=f64, device=z.device)
    Bm = torch.empty((B_, N, nx, nu), dtype=f64, device=z.device)
    E = None
    eh = None
    if e is not None:
        E = torch.empty((B_, N, nx, nx + dyn.n_units), dtype=f64, device=z.device)
        eh = (ctypes.c_double * nx)(*[float(x) for x in e])
    _check(lib().leb_linearize(ctypes.byref(dyn), B_, N, _dev_ptr(z, "z", f64), _dev_ptr(v, "v", f64),
                               None if eh is None else ctypes.cast(eh, ctypes.c_void_p), float(thrust),
                               _dev_ptr(A, "A", f64), _dev_ptr(Bm, "B", f64), _dev_ptr(E, "E", f64),
                               _stream(stream)))
    return A, Bm, E


def sls_responses(A, B, qx, qu, stream=None):
    """Closed-loop responses by the parallel Riccati recursions (see leb.h:
    leb_sls_responses).  A [b][N][nx][nx], B [b][N][nx][nu], qx [b][N+1][N][nx],
    qu [b][N][N][nu] float64 GPU tensors.  Returns (K, phi); entries k <= j are
    zero."""
    import torch
    f64 = torch.float64
    b, N, nx, nu = (int(x) for x in B.shape)
    K = torch.zeros((b, N, N, nu, nx), dtype=f64, device=A.device)
    phi = torch.zeros((b, N, N, nx + nu, nx), dtype=f64, device=A.device)
    _check(lib().leb_sls_responses(nx, nu, b, N, _dev_ptr(A, "A", f64), _dev_ptr(B, "B", f64),
                                   _dev_ptr(qx, "qx", f64), _dev_ptr(qu, "qu", f64), _dev_ptr(K, "K", f64),
                                   _dev_ptr(phi, "phi", f64), _stream(stream)))
    return K, phi


def sls_tube_map(phi, E, c_bar, rho_bar, stream=None):
    """Tube of time-varying responses (see leb.h: leb_sls_tube_map).
    phi [b][N][N][n][nx], E [b][N][nx][nw], c_bar, rho_bar [b][N][nx].
    Returns (mu, sigma) [b][N][n]."""
    import torch
    f64 = torch.float64
    b, N, _, n, nx = (int(x) for x in phi.shape)
    nw = int(E.shape[3]) if E is not None else 0
    mu = torch.empty((b, N, n), dtype=f64, device=phi.device)
    sg = torch.empty_like(mu)
    _check(lib().leb_sls_tube_map(nx, n - nx, nw, b, N, _dev_ptr(phi, "phi", f64), _dev_ptr(E, "E", f64),
                                  _dev_ptr(c_bar, "c_bar", f64), _dev_ptr(rho_bar, "rho_bar", f64),
                                  _dev_ptr(mu, "mu", f64), _dev_ptr(sg, "sigma", f64), _stream(stream)))
    return mu, sg


def sls_fixed_point(dyn: Dynamics, z, v, phi, E, thrust=0.0, pad=0.0, stream=None):
    """Exact tube/LEB fixed point of one controller update (see leb.h:
    leb_sls_fixed_point).  Returns (mu, sigma, r_lo, r_hi, certified)."""
    import torch
    f64 = torch.float64
    b, N = int(z.shape[0]), int(z.shape[1])
    n = dyn.nx + dyn.nu
    nw = int(E.shape[3]) if E is not None else 0
    mu = torch.empty((b, N, n), dtype=f64, device=z.device)
    sg = torch.empty_like(mu)
    lo = torch.empty((b, N, dyn.nx), dtype=f64, device=z.device)
    hi = torch.empty_like(lo)
    cert = torch.empty((b,), dtype=torch.int32, device=z.device)
    _check(lib().leb_sls_fixed_point(ctypes.byref(dyn), b, N, _dev_ptr(z, "z", f64), _dev_ptr(v, "v", f64),
                                     _dev_ptr(phi, "phi", f64), nw, _dev_ptr(E, "E", f64), float(thrust),
                                     float(pad), _dev_ptr(mu, "mu", f64), _dev_ptr(sg, "sigma", f64),
                                     _dev_ptr(lo, "r_lo", f64), _dev_ptr(hi, "r_hi", f64),
                                     _dev_ptr(cert, "certified"), _stream(stream)))
    return mu, sg, lo, hi, cert


def sls_update(dyn: Dynamics, z, v, qx, qu, e, thrust=0.0, pad=0.0, stream=None):
    """One controller update on the GPU: linearization, responses from the
    Riccati recursions, and the exact tube/LEB fixed point.  Returns a dict
    with A, B, E, K, phi, mu, sigma, r_lo, r_hi, certified."""
    A, Bm, E = linearize(dyn, z, v, e, thrust, stream)
    K, phi = sls_responses(A, Bm, qx, qu, stream)
    mu, sg, lo, hi, cert = sls_fixed_point(dyn, z, v, phi, E, thrust, pad, stream)
    return dict(A=A, B=Bm, E=E, K=K, phi=phi, mu=mu, sigma=sg, r_lo=lo, r_hi=hi, certified=cert)


def zonotope_hull(G, c=None, stream=None):
    """Interval hull of zonotopes (see leb.h: leb_zonotope_hull): G [rows][n_gen],
    c [rows] float64 GPU tensors -> (mu, sigma) [rows]."""
    import torch
    f64 = torch.float64
    rows, ng = int(G.shape[0]), int(G.shape[1])
    mu = torch.empty((rows,), dtype=f64, device=G.device)
    sg = torch.empty((rows,), dtype=f64, device=G.device)
    _check(lib().leb_zonotope_hull(rows, ng, _dev_ptr(G, "G", f64), _dev_ptr(c, "c", f64), _dev_ptr(mu, "mu", f64),
                                   _dev_ptr(sg, "sigma", f64), _stream(stream)))
    return mu, sg


def backward(dyn: Dynamics, z, v, sigma, g_lo, g_hi, mu=None, stream=None):
    """Gradient of sum(g_lo r_lo + g_hi r_hi) of the path-based bound with
    respect to z, v, sigma (and mu when given): see leb.h, leb_backward."""
    import torch
    f64 = torch.float64
    gz = torch.empty_like(z)
    gv = torch.empty_like(v)
    gs = torch.empty_like(sigma)
    gm = None if mu is None else torch.empty_like(mu)
    B, N = int(z.shape[0]), int(z.shape[1])
    rc = lib().leb_backward(ctypes.byref(dyn), B, N, _dev_ptr(z, "z", f64), _dev_ptr(v, "v", f64),
                            _dev_ptr(mu, "mu", f64), _dev_ptr(sigma, "sigma", f64), _dev_ptr(g_lo, "g_lo", f64),
                            _dev_ptr(g_hi, "g_hi", f64), _dev_ptr(gz, "gz", f64), _dev_ptr(gv, "gv", f64),
                            _dev_ptr(gm, "gmu", f64), _dev_ptr(gs, "gsigma", f64), _stream(stream))
    _check(rc)
    return gz, gv, gs, gm


def _autograd_class():
    import torch

    class LEBAnalytic(torch.autograd.Function):
        """(z, v, sigma, mu) -> (r_lo, r_hi) with the hand-written adjoint.
        Saves only the inputs; the backward recomputes the intervals."""

        @staticmethod
        def forward(ctx, dyn_box, z, v, sigma, mu):
            dyn = dyn_box[0]
            out = analytic_bound(dyn, z, v, sigma, mu)
            ctx.dyn = dyn
            ctx.has_mu = mu is not None
            ctx.save_for_backward(z, v, sigma, mu if mu is not None else sigma)
            return out["r_lo"], out["r_hi"]

        @staticmethod
        def backward(ctx, g_lo, g_hi):
            z, v, sigma, mu = ctx.saved_tensors
            mu = mu if ctx.has_mu else None
            gz, gv, gs, gm = backward(ctx.dyn, z, v, sigma, g_lo.contiguous(), g_hi.contiguous(), mu)
            return None, gz, gv, gs, gm

    return LEBAnalytic


def _autograd_nn_class():
    import torch

    class LEBNN(torch.autograd.Function):
        """(z, v, sigma, mu) -> (r_lo, r_hi) of the MLP bound with the
        hand-written adjoint (leb_nn_backward recomputes every pass)."""

        @staticmethod
        def forward(ctx, net_box, z, v, sigma, mu):
            net = net_box[0]
            out = nn_bound(net, z, v, sigma, mu)
            ctx.net = net
            ctx.has_mu = mu is not None
            ctx.save_for_backward(z, v, sigma, mu if mu is not None else sigma)
            return out["r_lo"], out["r_hi"]

        @staticmethod
        def backward(ctx, g_lo, g_hi):
            z, v, sigma, mu = ctx.saved_tensors
            mu = mu if ctx.has_mu else None
            g = nn_backward(ctx.net, z, v, sigma, g_lo.contiguous(), g_hi.contiguous(), mu=mu)
            return None, g["gz"], g["gv"], g["gsigma"], g.get("gmu")

    return LEBNN


_LEBAnalytic = None
_LEBNN = None


def leb_nn(net, z, v, sigma, mu=None):
    """Differentiable MLP bound: returns (r_lo, r_hi) tensors that
    back-propagate through leb_nn_backward."""
    global _LEBNN
    if _LEBNN is None:
        _LEBNN = _autograd_nn_class()
    return _LEBNN.apply((net,), z, v, sigma, mu)


def leb_analytic(dyn: Dynamics, z, v, sigma, mu=None):
    """Differentiable path-based bound: returns (r_lo, r_hi) tensors that
    back-propagate through leb_backward."""
    global _LEBAnalytic
    if _LEBAnalytic is None:
        _LEBAnalytic = _autograd_class()
    return _LEBAnalytic.apply((dyn,), z, v, sigma, mu)


def _host6(e):
    arr = (ctypes.c_double * 6)(*[float(x) for x in e])
    return arr


LAUNCH_BOUND, LAUNCH_TUBE = 0, 1


def launch_timing(enable: bool):
    """Start (clearing the record) or stop timing the fixed-point sweeps'
    bound and tube-map launches (see leb.h: leb_launch_timing)."""
    _check(lib().leb_launch_timing(1 if enable else 0))


def launch_times(kernel: int):
    """Durations in ms of the recorded launches of kernel (LAUNCH_BOUND or
    LAUNCH_TUBE), in launch order."""
    n = ctypes.c_int32(0)
    _check(lib().leb_launch_times(kernel, None, 0, ctypes.byref(n)))
    buf = (ctypes.c_float * max(1, n.value))()
    _check(lib().leb_launch_times(kernel, buf, n.value, ctypes.byref(n)))
    return [float(buf[i]) for i in range(n.value)]


def tube_map(n_units, phi, e, c_bar, rho_bar, stream=None, out=None):
    """Tube centre/width from residual zonotopes (see leb.h: leb_tube_map).

    phi [N-1][8][6] float64 GPU tensor, e: 6 host floats, c_bar/rho_bar
    [B][N][6U] GPU tensors.  Returns (mu, sigma) [B][N][8U]."""
    import torch
    B, N = int(c_bar.shape[0]), int(c_bar.shape[1])
    f64 = torch.float64
    if out is None:
        out = (torch.empty((B, N, 8 * n_units), dtype=f64, device=c_bar.device),
               torch.empty((B, N, 8 * n_units), dtype=f64, device=c_bar.device))
    rc = lib().leb_tube_map(B, N, int(n_units), _dev_ptr(phi, "phi", f64), _host6(e),
                            _dev_ptr(c_bar, "c_bar", f64), _dev_ptr(rho_bar, "rho_bar", f64),
                            _dev_ptr(out[0], "mu", f64), _dev_ptr(out[1], "sigma", f64), _stream(stream))
    _check(rc)
    return out


def _cert_out(B, N, device):
    """The certificate flags: every entry is written by a solve with
    timesteps; an empty horizon launches nothing, so its flags start at 0."""
    import torch
    if B * N == 0:
        return torch.zeros((B,), dtype=torch.int32, device=device)
    return torch.empty((B,), dtype=torch.int32, device=device)


def fixed_point_solve(dyn: Dynamics, z, v, phi, e, tol=1e-6, max_sweeps=200, pad=0.0, inflate_abs=1e-12,
                      mu=None, sigma=None, stream=None, conv_tol=None):
    """Certified tube/LEB fixed point (see leb.h: leb_fixed_point_solve).

    Warm start when mu and sigma are given (they are updated in place).
    Returns (mu, sigma, certified [B] int32 tensor, sweeps)."""
    import torch
    B, N = int(z.shape[0]), int(z.shape[1])
    n = dyn.nx + dyn.nu
    warm = mu is not None
    if not warm:        # the cold start writes every entry
        mu = torch.empty((B, N, n), dtype=torch.float64, device=z.device)
        sigma = torch.empty((B, N, n), dtype=torch.float64, device=z.device)
    cert = _cert_out(B, N, z.device)
    opt = FPOptions(tol, max_sweeps, pad, inflate_abs, 1 if warm else 0, tol if conv_tol is None else conv_tol)
    sweeps = ctypes.c_int32(0)
    f64 = torch.float64
    rc = lib().leb_fixed_point_solve(ctypes.byref(dyn), B, N, _dev_ptr(z, "z", f64), _dev_ptr(v, "v", f64),
                                     _dev_ptr(phi, "phi", f64), _host6(e), ctypes.byref(opt),
                                     _dev_ptr(mu, "mu", f64), _dev_ptr(sigma, "sigma", f64),
                                     _dev_ptr(cert, "certified"), ctypes.byref(sweeps), _stream(stream))
    _check(rc)
    return mu, sigma, cert, int(sweeps.value)


def fixed_point_solve_noalloc(dyn: Dynamics, z, v, phi, e, mu, sigma, certified, tol=1e-6, max_sweeps=20, pad=0.0,
                              inflate_abs=1e-12, warm=False, stream=None, conv_tol=None):
    """leb_fixed_point_solve_noalloc: the caller passes every output
    (mu, sigma [B][N][n] float64, certified [B] int32 GPU tensors; mu and sigma
    hold the warm start when warm).  Returns the number of sweeps enqueued."""
    import torch
    B, N = int(z.shape[0]), int(z.shape[1])
    opt = FPOptions(tol, max_sweeps, pad, inflate_abs, 1 if warm else 0, tol if conv_tol is None else conv_tol)
    sweeps = ctypes.c_int32(0)
    f64 = torch.float64
    rc = lib().leb_fixed_point_solve_noalloc(ctypes.byref(dyn), B, N, _dev_ptr(z, "z", f64), _dev_ptr(v, "v", f64),
                                             _dev_ptr(phi, "phi", f64), _host6(e), ctypes.byref(opt),
                                             _dev_ptr(mu, "mu", f64), _dev_ptr(sigma, "sigma", f64),
                                             _dev_ptr(certified, "certified"), ctypes.byref(sweeps), _stream(stream))
    _check(rc)
    return int(sweeps.value)


def fixed_point_learned(dyn: Dynamics, z, v, phi, e, net, sweeps=1, margin=5e-2, tol=1e-6, max_sweeps=200,
                        pad=0.0, inflate_abs=1e-12, stream=None, conv_tol=None):
    """Certified fixed point from a learned initial tube (see leb.h:
    leb_fixed_point_learned).  Returns (mu, sigma, certified, certified sweeps)."""
    import torch
    B, N = int(z.shape[0]), int(z.shape[1])
    n = dyn.nx + dyn.nu
    mu = torch.empty((B, N, n), dtype=torch.float64, device=z.device)
    sigma = torch.empty((B, N, n), dtype=torch.float64, device=z.device)
    cert = _cert_out(B, N, z.device)
    opt = FPOptions(tol, max_sweeps, pad, inflate_abs, 1, tol if conv_tol is None else conv_tol)
    ws = WarmStart(net.handle, int(sweeps), float(margin))
    sw = ctypes.c_int32(0)
    f64 = torch.float64
    rc = lib().leb_fixed_point_learned(ctypes.byref(dyn), B, N, _dev_ptr(z, "z", f64), _dev_ptr(v, "v", f64),
                                       _dev_ptr(phi, "phi", f64), _host6(e), ctypes.byref(opt), ctypes.byref(ws),
                                       _dev_ptr(mu, "mu", f64), _dev_ptr(sigma, "sigma", f64),
                                       _dev_ptr(cert, "certified"), ctypes.byref(sw), _stream(stream))
    _check(rc)
    return mu, sigma, cert, int(sw.value)


def chain_features(dyn: Dynamics, z, v, sigma, mu=None, stream=None):
    """Surrogate inputs [B][N][n_units][32] (float32) of a chain tube."""
    import torch
    B, N = int(z.shape[0]), int(z.shape[1])
    x = torch.empty((B, N, dyn.n_units, CHAIN_FEATURES), dtype=torch.float32, device=z.device)
    f64 = torch.float64
    _check(lib().leb_chain_features(ctypes.byref(dyn), B, N, _dev_ptr(z, "z", f64), _dev_ptr(v, "v", f64),
                                    _dev_ptr(mu, "mu", f64), _dev_ptr(sigma, "sigma", f64),
                                    _dev_ptr(x, "x", torch.float32), _stream(stream)))
    return x


def chain_surrogate_bound(dyn: Dynamics, z, v, sigma, net, mu=None, pad=0.0, stream=None):
    """The surrogate's residual zonotope (c_bar, rho_bar) [B][N][nx] for a
    chain tube (see leb.h: leb_chain_surrogate_bound).  Not certified."""
    import torch
    B, N = int(z.shape[0]), int(z.shape[1])
    f64 = torch.float64
    cb = torch.empty((B, N, dyn.nx), dtype=f64, device=z.device)
    rb = torch.empty_like(cb)
    _check(lib().leb_chain_surrogate_bound(ctypes.byref(dyn), B, N, _dev_ptr(z, "z", f64), _dev_ptr(v, "v", f64),
                                           _dev_ptr(mu, "mu", f64), _dev_ptr(sigma, "sigma", f64), net.handle,
                                           _dev_ptr(cb, "c_bar", f64), _dev_ptr(rb, "rho_bar", f64), float(pad),
                                           _stream(stream)))
    return cb, rb


def chain_targets(dyn: Dynamics, r_lo, r_hi, stream=None):
    """Surrogate targets [B][N][n_units][4] (float32) from a chain bound."""
    import torch
    B, N = int(r_lo.shape[0]), int(r_lo.shape[1])
    t = torch.empty((B, N, dyn.n_units, CHAIN_OUTPUTS), dtype=torch.float32, device=r_lo.device)
    f64 = torch.float64
    _check(lib().leb_chain_targets(ctypes.byref(dyn), B, N, _dev_ptr(r_lo, "r_lo", f64),
                                   _dev_ptr(r_hi, "r_hi", f64), _dev_ptr(t, "t", torch.float32), _stream(stream)))
    return t


def nn_features(z, v, sigma, mu=None, stream=None):
    """NN-surrogate inputs [B][N][2 (nx + nu)] (float32) of the boxes of
    ReLU-MLP dynamics (see leb.h: leb_nn_features)."""
    import torch
    B, N, nx, nu = int(z.shape[0]), int(z.shape[1]), int(z.shape[2]), int(v.shape[2])
    x = torch.empty((B, N, 2 * (nx + nu)), dtype=torch.float32, device=z.device)
    f64 = torch.float64
    _check(lib().leb_nn_features(nx, nu, B, N, _dev_ptr(z, "z", f64), _dev_ptr(v, "v", f64), _dev_ptr(mu, "mu", f64),
                                 _dev_ptr(sigma, "sigma", f64), _dev_ptr(x, "x", torch.float32), _stream(stream)))
    return x


def nn_targets(r_lo, r_hi, stream=None):
    """NN-surrogate targets [B][N][2m] (float32) from a bound [B][N][m]."""
    import torch
    B, N, m = int(r_lo.shape[0]), int(r_lo.shape[1]), int(r_lo.shape[2])
    t = torch.empty((B, N, 2 * m), dtype=torch.float32, device=r_lo.device)
    f64 = torch.float64
    _check(lib().leb_nn_targets(m, B, N, _dev_ptr(r_lo, "r_lo", f64), _dev_ptr(r_hi, "r_hi", f64),
                                _dev_ptr(t, "t", torch.float32), _stream(stream)))
    return t


def nn_surrogate_bound(net, z, v, sigma, mu=None, stream=None):
    """The NN surrogate's predicted (r_lo, r_hi) [B][N][m] (see leb.h:
    leb_nn_surrogate_bound).  Not certified."""
    import torch
    B, N, nx, nu = int(z.shape[0]), int(z.shape[1]), int(z.shape[2]), int(v.shape[2])
    m = net.widths[-1] // 2
    f64 = torch.float64
    lo = torch.empty((B, N, m), dtype=f64, device=z.device)
    hi = torch.empty_like(lo)
    _check(lib().leb_nn_surrogate_bound(net.handle, nx, nu, B, N, _dev_ptr(z, "z", f64), _dev_ptr(v, "v", f64),
                                        _dev_ptr(mu, "mu", f64), _dev_ptr(sigma, "sigma", f64),
                                        _dev_ptr(lo, "r_lo", f64), _dev_ptr(hi, "r_hi", f64), _stream(stream)))
    return lo, hi


class MLP:
    """ReLU MLP uploaded to the device (see leb.h: leb_mlp_create).

    W, b: lists of host float32 arrays ([out][in] and [out]); nx: state
    inputs; residual: dynamics x + g(x, u)."""

    def __init__(self, W, b, nx, residual=True):
        import numpy as np
        self._W = [np.ascontiguousarray(w, dtype=np.float32) for w in W]
        self._b = [np.ascontiguousarray(x, dtype=np.float32) for x in b]
        L = len(self._W)
        widths = [self._W[0].shape[1]] + [w.shape[0] for w in self._W]
        self.widths = widths
        self.nx = int(nx)
        self.m = widths[-1]
        fp = ctypes.POINTER(ctypes.c_float)
        Wp = (fp * L)(*[w.ctypes.data_as(fp) for w in self._W])
        bp = (fp * L)(*[x.ctypes.data_as(fp) for x in self._b])
        wd = (ctypes.c_int32 * (L + 1))(*widths)
        h = ctypes.c_void_p()
        _check(lib().leb_mlp_create(L, wd, Wp, bp, self.nx, 1 if residual else 0, ctypes.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().leb_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def nn_bound(mlp: MLP, z, v, sigma, mu=None, pad: float = 0.0, zonotope: bool = False, stream=None, J=None):
    """CROWN + Theorem 2 bound for ReLU-MLP dynamics (see leb.h: leb_nn_bound).
    z [B][N][nx], v [B][N][nu], sigma (mu) [B][N][nx+nu] float64 GPU tensors;
    J [B][N][m][nx+nu] the linearization's matrix (None: the network's Jacobian)."""
    import torch
    B, N = int(z.shape[0]), int(z.shape[1])
    f64 = torch.float64
    out = {"r_lo": torch.empty((B, N, mlp.m), dtype=f64, device=z.device),
           "r_hi": torch.empty((B, N, mlp.m), dtype=f64, device=z.device),
           "flags": torch.empty((B, N), dtype=torch.int32, device=z.device)}
    if zonotope:
        out["c_bar"] = torch.empty((B, N, mlp.m), dtype=f64, device=z.device)
        out["rho_bar"] = torch.empty((B, N, mlp.m), dtype=f64, device=z.device)
    rc = lib().leb_nn_bound(mlp.handle, B, N, _dev_ptr(z, "z", f64), _dev_ptr(v, "v", f64), _dev_ptr(mu, "mu", f64),
                            _dev_ptr(sigma, "sigma", f64), _dev_ptr(J, "J", f64), _dev_ptr(out["r_lo"], "r_lo", f64),
                            _dev_ptr(out["r_hi"], "r_hi", f64), _dev_ptr(out.get("c_bar"), "c_bar", f64),
                            _dev_ptr(out.get("rho_bar"), "rho_bar", f64), float(pad),
                            _dev_ptr(out["flags"], "flags"), _stream(stream))
    _check(rc)
    return out


def nn_backward(mlp: MLP, z, v, sigma, g_lo, g_hi, mu=None, stream=None):
    """Gradient of sum g_lo r_lo + g_hi r_hi of the MLP bound (see leb.h:
    leb_nn_backward).  Returns {"gz", "gv", "gsigma"} (and "gmu" when mu is
    given), shaped as the inputs."""
    import torch
    f64 = torch.float64
    out = {"gz": torch.empty_like(z), "gv": torch.empty_like(v), "gsigma": torch.empty_like(sigma)}
    if mu is not None:
        out["gmu"] = torch.empty_like(mu)
    B, N = int(z.shape[0]), int(z.shape[1])
    _check(lib().leb_nn_backward(mlp.handle, B, N, _dev_ptr(z, "z", f64), _dev_ptr(v, "v", f64),
                                 _dev_ptr(mu, "mu", f64), _dev_ptr(sigma, "sigma", f64), _dev_ptr(g_lo, "g_lo", f64),
                                 _dev_ptr(g_hi, "g_hi", f64), _dev_ptr(out["gz"], "gz", f64),
                                 _dev_ptr(out["gv"], "gv", f64), _dev_ptr(out.get("gmu"), "gmu", f64),
                                 _dev_ptr(out["gsigma"], "gsigma", f64), _stream(stream)))
    return out


class Surrogate:
    """BF16 MFMA GELU MLP of the learned warm start (see leb.h:
    leb_surrogate_create).  widths [d_0, ..., d_L]; params: flat float32
    host array [W_1, b_1, ..., W_L, b_L] with W_l row-major [d_l][d_{l-1}]."""

    def __init__(self, widths, params):
        import numpy as np
        self.widths = [int(w) for w in widths]
        p = np.ascontiguousarray(params, dtype=np.float32)
        wd = (ctypes.c_int32 * len(self.widths))(*self.widths)
        h = ctypes.c_void_p()
        _check(lib().leb_surrogate_create(len(self.widths) - 1, wd, p.ctypes.data_as(ctypes.c_void_p),
                                          ctypes.byref(h)))
        self.handle = h
        self.n_params = int(lib().leb_surrogate_n_params(h))
        if self.n_params != p.size:
            self.close()
            raise LebError("params has %d values, the widths need %d" % (p.size, self.n_params))

    def params(self):
        import numpy as np
        out = np.empty(self.n_params, dtype=np.float32)
        _check(lib().leb_surrogate_params(self.handle, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def forward(self, x, out=None, stream=None):
        """x [B][d_0] float32 GPU tensor -> y [B][d_L]."""
        import torch
        B = int(x.shape[0])
        y = out if out is not None else torch.empty((B, self.widths[-1]), dtype=torch.float32, device=x.device)
        _check(lib().leb_mlp_fwd_bf16(self.handle, B, _dev_ptr(x, "x", torch.float32),
                                      _dev_ptr(y, "y", torch.float32), _stream(stream)))
        return y

    def backward(self, x, dy, stream=None):
        """Parameter gradient of sum(dy * forward(x)) (flat float32 GPU tensor)."""
        import torch
        g = torch.empty(self.n_params, dtype=torch.float32, device=x.device)
        _check(lib().leb_mlp_bwd_bf16(self.handle, int(x.shape[0]), _dev_ptr(x, "x", torch.float32),
                                      _dev_ptr(dy, "dy", torch.float32), _dev_ptr(g, "grads", torch.float32),
                                      _stream(stream)))
        return g

    def adam(self, grads, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        import torch
        _check(lib().leb_adam_step(self.handle, _dev_ptr(grads, "grads", torch.float32), int(step), float(lr),
                                   float(beta1), float(beta2), float(eps), _stream(stream)))

    def train_step(self, x, t, step, lr, loss=None, stream=None):
        """Forward + MSE + backward + Adam; loss: optional 1-float GPU tensor."""
        import torch
        _check(lib().leb_surrogate_train_step(self.handle, int(x.shape[0]), _dev_ptr(x, "x", torch.float32),
                                              _dev_ptr(t, "t", torch.float32), int(step), float(lr),
                                              _dev_ptr(loss, "loss", torch.float32), _stream(stream)))

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().leb_surrogate_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Uneven problems bounded by one graph launch (see leb.h:
    leb_batch_create).  problems: list of dicts with keys kind ("analytic"
    with dyn, or "nn" with net: MLP), z [N][nx], v [N][nu], sigma [N][n],
    optional mu, and r_lo, r_hi [N][nx] output tensors (float64 GPU,
    contiguous; they must stay alive while the batch exists)."""

    def __init__(self, problems, tune_cache=None):
        import torch
        f64 = torch.float64
        arr = (Problem * len(problems))()
        self._keep = []
        for i, p in enumerate(problems):
            q = arr[i]
            if p["kind"] == "analytic":
                q.type = PROBLEM_ANALYTIC
                d = p["dyn"]
                self._keep.append(d)
                q.dyn = ctypes.pointer(d)
            else:
                q.type = PROBLEM_NN
                q.net = p["net"].handle
                self._keep.append(p["net"])
            q.N = int(p["z"].shape[0])
            q.z = _dev_ptr(p["z"], "z", f64)
            q.v = _dev_ptr(p["v"], "v", f64)
            q.mu = _dev_ptr(p.get("mu"), "mu", f64)
            q.sigma = _dev_ptr(p["sigma"], "sigma", f64)
            q.r_lo = _dev_ptr(p["r_lo"], "r_lo", f64)
            q.r_hi = _dev_ptr(p["r_hi"], "r_hi", f64)
            self._keep.append(p)
        h = ctypes.c_void_p()
        _check(lib().leb_batch_create(arr, len(problems), None if tune_cache is None else str(tune_cache).encode(),
                                      ctypes.byref(h)))
        self.handle = h

    def submit(self, stream=None):
        _check(lib().leb_batch_submit(self.handle, _stream(stream)))

    def info(self):
        buf = ctypes.create_string_buffer(4096)
        _check(lib().leb_batch_info(self.handle, buf, 4096))
        return buf.value.decode()

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().leb_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
