"""FP64 CPU oracle for linearization-error bounds -- TEST INFRASTRUCTURE.

Only the test suite, the package smoke check and the benchmark's CPU
baseline leg may import this package.  It shares no code with the GPU
library.  The C part (`leb_oracle.c`) holds the interval bounds and the
true-remainder sampler; `nn.py` holds the neural-network bounds and
`tube.py` the tube map and fixed point.

Dynamics are described by plain keyword parameters (never by GPU-library
types): `kind` is one of "linear", "quadratic", "sin1d", "sincos2d",
"chain", "satellite", "quad3d"; chain dynamics also take n_units, dt, m, g,
arm, inertia, k_spring, rest_len; the satellite dt and its inertia J; the
3-D quadrotor dt, m, g and J = (Jx, Jy, Jz).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "leb_oracle.c")
_SRC_GRAD = os.path.join(_HERE, "leb_grad.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

KINDS = {"linear": 0, "quadratic": 1, "sin1d": 2, "sincos2d": 3, "chain": 4, "satellite": 5, "quad3d": 6}
MODES = {"path": 0, "expand": 1, "classic": 2}
FLAG_UNBOUNDED, FLAG_BAD_INPUT, FLAG_HULL = 1, 2, 4


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (-O2, OpenMP, no fast-math)."""
    newest = max(os.path.getmtime(_SRC), os.path.getmtime(_SRC_GRAD))
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < newest:
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math",
                               "-o", tmp, _SRC, _SRC_GRAD, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Dyn(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("nx", ctypes.c_int32), ("nu", ctypes.c_int32),
                ("n_units", ctypes.c_int32), ("dt", ctypes.c_double), ("m", ctypes.c_double),
                ("g", ctypes.c_double), ("arm", ctypes.c_double), ("inertia", ctypes.c_double),
                ("k_spring", ctypes.c_double), ("rest_len", ctypes.c_double),
                ("Q", ctypes.POINTER(ctypes.c_double)), ("J", ctypes.c_double * 3)]


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        L.orc_leb.argtypes = [ctypes.POINTER(_Dyn), ctypes.c_int, ctypes.c_long, dp, dp, dp, dp,
                              dp, dp, ctypes.POINTER(ctypes.c_uint32), ctypes.c_int]
        L.orc_remainder.argtypes = [ctypes.POINTER(_Dyn), ctypes.c_long, ctypes.POINTER(ctypes.c_int64),
                                    dp, dp, dp, dp, ctypes.c_int]
        L.orc_hess_entry.argtypes = [ctypes.POINTER(_Dyn), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     dp, dp, dp, dp]
        L.orc_nonlin.argtypes = [ctypes.POINTER(_Dyn), ctypes.c_int, dp, dp, dp]
        L.orc_leb_grad.argtypes = [ctypes.POINTER(_Dyn), ctypes.c_long, dp, dp, dp, dp, dp, dp, dp, dp,
                                   dp, dp, dp, ctypes.c_int]
        L.orc_step.argtypes = [ctypes.POINTER(_Dyn), ctypes.c_long, dp, dp, dp]
        L.orc_jacobian.argtypes = [ctypes.POINTER(_Dyn), ctypes.c_long, dp, dp, dp, dp]
        L.orc_isin.argtypes = [ctypes.c_double, ctypes.c_double, dp]
        L.orc_icos.argtypes = [ctypes.c_double, ctypes.c_double, dp]
        _lib = L
    return _lib


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Dyn:
    """Oracle-side dynamics description (keeps the Q array alive)."""

    def __init__(self, kind: str, nx: int, nu: int = 0, n_units: int = 0, dt=0.05, m=1.0, g=9.81,
                 arm=0.25, inertia=0.01, k_spring=2.0, rest_len=1.0, Q=None, J=(0.0, 0.0, 0.0)):
        self.kind, self.nx, self.nu = kind, nx, nu
        self.n = nx + nu
        self.Q = None if Q is None else np.ascontiguousarray(Q, dtype=np.float64)
        self.c = _Dyn(KINDS[kind], nx, nu, n_units, dt, m, g, arm, inertia, k_spring, rest_len,
                      _ptr(self.Q), (ctypes.c_double * 3)(*J))

    @staticmethod
    def satellite(dt, inertia=(5.0, 2.0, 1.0)):
        """Satellite attitude (quaternion q, rates w; torques v): nx = 7, nu = 3."""
        return Dyn("satellite", 7, 3, 0, dt, J=tuple(inertia))

    @staticmethod
    def quad3d(dt, m, g, J):
        """3-D quadrotor (position, Euler angles, velocity, body rates; thrust, torques): nx = 12, nu = 4."""
        return Dyn("quad3d", 12, 4, 0, dt, m, g, J=tuple(J))

    @staticmethod
    def chain(n_units, dt=0.05, m=1.0, g=9.81, arm=0.25, inertia=0.01, k_spring=2.0, rest_len=1.0):
        return Dyn("chain", 6 * n_units, 2 * n_units, n_units, dt, m, g, arm, inertia, k_spring, rest_len)

    @staticmethod
    def like(obj):
        """Build from any object exposing chain parameters (n_units, dt, m, ...), or
        a satellite / 3-D quadrotor description (kind, dt, m, g, J)."""
        kind = getattr(obj, "kind", "chain")
        if kind == "satellite":
            return Dyn.satellite(obj.dt, obj.J)
        if kind == "quad3d":
            return Dyn.quad3d(obj.dt, obj.m, obj.g, obj.J)
        return Dyn.chain(obj.n_units, obj.dt, obj.m, obj.g, obj.arm, obj.inertia, obj.k_spring,
                         obj.rest_len)


def leb(dyn: Dyn, z, v, sigma, mu=None, mode: str = "path", threads: int = 0):
    """Interval enclosure [lo, hi] of the linearization remainder per unit.

    z [..., nx], v [..., nu], sigma/mu [..., nx+nu] (leading dims are units).
    Returns (lo, hi, flags) with lo/hi shaped [..., nx]."""
    z = np.ascontiguousarray(z, dtype=np.float64)
    lead = z.shape[:-1]
    U = int(np.prod(lead)) if lead else 1
    v = np.ascontiguousarray(v, dtype=np.float64).reshape(U, dyn.nu) if dyn.nu else np.zeros((U, 0))
    sg = np.ascontiguousarray(sigma, dtype=np.float64).reshape(U, dyn.n)
    mu_a = None if mu is None else np.ascontiguousarray(mu, dtype=np.float64).reshape(U, dyn.n)
    lo = np.empty((U, dyn.nx))
    hi = np.empty((U, dyn.nx))
    fl = np.zeros(U, dtype=np.uint32)
    rc = lib().orc_leb(ctypes.byref(dyn.c), MODES[mode], U, _ptr(z.reshape(U, dyn.nx)),
                       _ptr(v) if dyn.nu else _ptr(np.zeros(1)), _ptr(mu_a), _ptr(sg),
                       _ptr(lo), _ptr(hi), fl.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                       int(threads))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return lo.reshape(lead + (dyn.nx,)), hi.reshape(lead + (dyn.nx,)), fl.reshape(lead)


def box(nom, sigma, mu=None):
    """Box of each unit, [a~ + min(mu - sigma, 0), a~ + max(mu + sigma, 0)]
    (hull with the nominal point).  Plain FP64, for sampling."""
    m = 0.0 if mu is None else mu
    return nom + np.minimum(m - sigma, 0.0), nom + np.maximum(m + sigma, 0.0)


def remainder(dyn: Dyn, nom, pts, unit_of, threads: int = 0):
    """True remainder r(a; a~) at sample points, with its FP64 error allowance.

    nom [U][n], pts [S][n], unit_of [S] -> (r [S][nx], eps [S][nx])."""
    nom = np.ascontiguousarray(nom, dtype=np.float64)
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    uo = np.ascontiguousarray(unit_of, dtype=np.int64)
    S = pts.shape[0]
    r = np.empty((S, dyn.nx))
    eps = np.empty((S, dyn.nx))
    lib().orc_remainder(ctypes.byref(dyn.c), S, uo.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                        _ptr(nom), _ptr(pts), _ptr(r), _ptr(eps), int(threads))
    return r, eps


def hess_entry(dyn: Dyn, l, k, j, box_lo, box_hi):
    """Enclosure of one Hessian entry over a given box: (status, lo, hi)."""
    lo = np.array(box_lo, dtype=np.float64)
    hi = np.array(box_hi, dtype=np.float64)
    a = np.zeros(1)
    b = np.zeros(1)
    st = lib().orc_hess_entry(ctypes.byref(dyn.c), int(l), int(k), int(j), _ptr(lo), _ptr(hi),
                              _ptr(a), _ptr(b))
    return st, float(a[0]), float(b[0])


def nonlin(dyn: Dyn, l, point):
    """Nonlinear part N_l of the dynamics and its gradient at a point."""
    p = np.ascontiguousarray(point, dtype=np.float64)
    val = np.zeros(1)
    grad = np.zeros(dyn.n)
    lib().orc_nonlin(ctypes.byref(dyn.c), int(l), _ptr(p), _ptr(val), _ptr(grad))
    return float(val[0]), grad


def step(dyn: Dyn, z, v):
    """Discretised dynamics f(x, u) at points z [..., nx], v [..., nu]."""
    z = np.ascontiguousarray(z, dtype=np.float64)
    lead = z.shape[:-1]
    U = int(np.prod(lead)) if lead else 1
    vv = np.ascontiguousarray(v, dtype=np.float64).reshape(U, dyn.nu) if dyn.nu else np.zeros((U, 1))
    f = np.empty((U, dyn.nx))
    if lib().orc_step(ctypes.byref(dyn.c), U, _ptr(z.reshape(U, dyn.nx)), _ptr(vv), _ptr(f)) != 0:
        raise ValueError("oracle step rejected the arguments")
    return f.reshape(lead + (dyn.nx,))


def jacobian(dyn: Dyn, z, v):
    """Point Jacobians A = df/dx [..., nx, nx], B = df/du [..., nx, nu]
    (eq. linearizations) at the nominal points."""
    z = np.ascontiguousarray(z, dtype=np.float64)
    lead = z.shape[:-1]
    U = int(np.prod(lead)) if lead else 1
    vv = np.ascontiguousarray(v, dtype=np.float64).reshape(U, dyn.nu) if dyn.nu else np.zeros((U, 1))
    A = np.empty((U, dyn.nx, dyn.nx))
    B = np.empty((U, dyn.nx, max(dyn.nu, 1)))
    if lib().orc_jacobian(ctypes.byref(dyn.c), U, _ptr(z.reshape(U, dyn.nx)), _ptr(vv), _ptr(A), _ptr(B)) != 0:
        raise ValueError("oracle jacobian rejected the arguments")
    return A.reshape(lead + (dyn.nx, dyn.nx)), B[..., :dyn.nu].reshape(lead + (dyn.nx, dyn.nu))


def isin(lo, hi):
    out = np.zeros(2)
    lib().orc_isin(lo, hi, _ptr(out))
    return out


def icos(lo, hi):
    out = np.zeros(2)
    lib().orc_icos(lo, hi, _ptr(out))
    return out


def leb_grad(dyn: Dyn, z, v, sigma, g_lo, g_hi, mu=None, threads: int = 0):
    """Gradient of sum(g_lo r_lo + g_hi r_hi) of the path-based bound with
    respect to z, v, sigma (and mu when given), by forward-mode dual
    numbers.  Returns dict gz, gv, gsigma, gmu (or None), margin [units]."""
    z = np.ascontiguousarray(z, dtype=np.float64)
    lead = z.shape[:-1]
    U = int(np.prod(lead))
    v = np.ascontiguousarray(v, dtype=np.float64).reshape(U, dyn.nu)
    sg = np.ascontiguousarray(sigma, dtype=np.float64).reshape(U, dyn.n)
    mu_a = None if mu is None else np.ascontiguousarray(mu, dtype=np.float64).reshape(U, dyn.n)
    gl = np.ascontiguousarray(g_lo, dtype=np.float64).reshape(U, dyn.nx)
    gh = np.ascontiguousarray(g_hi, dtype=np.float64).reshape(U, dyn.nx)
    gz = np.zeros((U, dyn.nx))
    gv = np.zeros((U, dyn.nu))
    gs = np.zeros((U, dyn.n))
    gm = None if mu is None else np.zeros((U, dyn.n))
    mg = np.zeros(U)
    rc = lib().orc_leb_grad(ctypes.byref(dyn.c), U, _ptr(z.reshape(U, dyn.nx)), _ptr(v), _ptr(mu_a), _ptr(sg),
                            _ptr(gl), _ptr(gh), _ptr(gz), _ptr(gv), _ptr(gm), _ptr(gs), _ptr(mg), int(threads))
    if rc != 0:
        raise ValueError("oracle gradient rejected the arguments")
    return {"gz": gz.reshape(lead + (dyn.nx,)), "gv": gv.reshape(lead + (dyn.nu,)),
            "gsigma": gs.reshape(lead + (dyn.n,)), "gmu": None if gm is None else gm.reshape(lead + (dyn.n,)),
            "margin": mg.reshape(lead)}
