"""Seeded synthetic inputs for the linearization-error-bound (LEB) path.

This module holds no part of the bound computation: only random draws,
array shapes, dynamics parameters and the synthetic closed-loop responses
that stand in for a solver's output.  The CPU oracle tests and the GPU
path both take their inputs from here, so neither depends on the other.

Coordinate order (used by every generator and by the path-based bound,
whose result depends on it): the augmented vector is alpha = [x; u].
For a chain of planar quadrotors the state stacks the per-node blocks
(px, pz, theta, vx, vz, omega) node after node, and the input stacks the
per-node pairs (u1, u2) node after node.  Positions are offsets from the
rest lattice (i * rest_len, 0), so the spring between nodes i and i+1 sees
the separation (rest_len + px[i+1] - px[i], pz[i+1] - pz[i]).

The workloads follow the shapes and value ranges of the paper's analytic
and neural systems (planar quadrotor, section "Planar Quadrotor" of the
dynamics appendix; coupled quadrotors up to 168 states; horizon 40).  No
public dataset is involved; all values are drawn here.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

__all__ = [
    "ChainDynamics", "AnalyticBatch", "MLPNet", "NNBatch", "TubeProblem",
    "planar_quad_cfg", "chain_cfg", "nn_cfg", "fixed_point_cfg", "mixed_batch_cfg",
    "chain_batch", "sample_box_points", "rng_for",
]

STATE_PER_NODE = 6      # px, pz, theta, vx, vz, omega
INPUT_PER_NODE = 2      # u1, u2


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


@dataclass(frozen=True)
class ChainDynamics:
    """A chain of planar quadrotors joined by nearest-neighbour springs.

    n_units == 1 is the single planar quadrotor (no spring).  Forward-Euler
    step x+ = x + dt * xdot with xdot of the planar quadrotor plus the
    spring accelerations F/m on (vx, vz).
    """
    n_units: int
    dt: float = 0.05
    m: float = 1.0
    g: float = 9.81
    arm: float = 0.25
    inertia: float = 0.01
    k_spring: float = 2.0
    rest_len: float = 1.0

    @property
    def nx(self) -> int:
        return STATE_PER_NODE * self.n_units

    @property
    def nu(self) -> int:
        return INPUT_PER_NODE * self.n_units

    @property
    def n(self) -> int:
        return self.nx + self.nu


@dataclass(frozen=True)
class SmallDynamics:
    """A small analytic system of the dynamics appendix: kind "satellite"
    (nx = 7, nu = 3, inertia J) or "quad3d" (nx = 12, nu = 4, mass m,
    inertia J)."""
    kind: str
    nx: int
    nu: int
    dt: float
    m: float = 1.0
    g: float = 9.81
    J: tuple = (1.0, 1.0, 1.0)

    @property
    def n(self) -> int:
        return self.nx + self.nu


SATELLITE = SmallDynamics("satellite", 7, 3, dt=0.1, J=(5.0, 2.0, 1.0))
QUAD3D = SmallDynamics("quad3d", 12, 4, dt=0.05, m=1.0, g=9.81, J=(0.01, 0.01, 0.02))


@dataclass
class AnalyticBatch:
    """Boxes ((z_k, v_k) + mu_k) +/- sigma_k for `batch` trajectories of N steps."""
    dyn: ChainDynamics
    z: np.ndarray                 # [batch][N][nx] float64
    v: np.ndarray                 # [batch][N][nu]
    sigma: np.ndarray             # [batch][N][nx+nu]
    mu: Optional[np.ndarray] = None   # [batch][N][nx+nu] or None (= 0)

    @property
    def batch(self) -> int:
        return self.z.shape[0]

    @property
    def N(self) -> int:
        return self.z.shape[1]


@dataclass
class MLPNet:
    """ReLU MLP g: R^n -> R^nx; dynamics f(x, u) = x + g([x; u]) when residual."""
    W: List[np.ndarray]           # float32, W[l] has shape [out][in]
    b: List[np.ndarray]           # float32
    nx: int
    nu: int
    residual: bool = True

    @property
    def widths(self) -> List[int]:
        return [self.W[0].shape[1]] + [w.shape[0] for w in self.W]


@dataclass
class NNBatch:
    net: MLPNet
    z: np.ndarray                 # [batch][N][nx]
    v: np.ndarray                 # [batch][N][nu]
    sigma: np.ndarray             # [batch][N][nx+nu]
    mu: Optional[np.ndarray] = None


@dataclass
class TubeProblem:
    """Tube/LEB fixed point on chain trajectories with a synthetic closed loop.

    phi[d-1] (d = 1..N-1) is the per-node closed-loop response block for a
    lag of d steps: rows 0..5 map a node's state residual into its state
    deviation, rows 6..7 into its input deviation.  Every node and every
    trajectory shares it (decentralised hover controller).  e is the
    per-node disturbance generator magnitude |E| 1.
    """
    batch: AnalyticBatch
    phi: np.ndarray               # [N-1][8][6]
    e: np.ndarray                 # [6]
    K: np.ndarray                 # [2][6] hover LQR gain (for reference)
    A_cl: np.ndarray              # [6][6]


# --------------------------------------------------------------------------
# analytic workloads

def planar_quad_cfg(seed: int = 0, N: int = 20) -> AnalyticBatch:
    """Single planar quadrotor, horizon N, one trajectory."""
    rng = rng_for(seed)
    z = rng.uniform(-1.0, 1.0, (N, 6))
    z[:, 2] = rng.uniform(-0.5, 0.5, N)
    v = rng.uniform(3.0, 7.0, (N, 2))
    sx = rng.uniform(0.01, 0.1, (N, 6))
    su = rng.uniform(0.05, 0.5, (N, 2))
    sigma = np.concatenate([sx, su], axis=1)
    return AnalyticBatch(ChainDynamics(n_units=1), z[None], v[None], sigma[None], None)


def _chain_nominal(rng, shape, n_units, rest_len, min_gap, sigma=None):
    """Nominal states/inputs for chains; spring pairs closer than the margin
    are redrawn node after node so every nominal separation stays clear of
    the singular configuration (zero spring length)."""
    B, N = shape
    U = n_units
    pos_other = rng.uniform(-1.0, 1.0, (B, N, U, 5))       # px, pz, vx, vz, omega
    theta = rng.uniform(-0.5, 0.5, (B, N, U))
    u = rng.uniform(3.0, 7.0, (B, N, U, 2))
    px = pos_other[..., 0].copy()
    pz = pos_other[..., 1].copy()
    for i in range(U - 1):
        while True:
            dx = rest_len + px[..., i + 1] - px[..., i]
            dz = pz[..., i + 1] - pz[..., i]
            dist = np.sqrt(dx * dx + dz * dz)
            need = np.full(dist.shape, min_gap)
            if sigma is not None:
                sx = sigma[..., 6 * i] + sigma[..., 6 * (i + 1)]
                sz = sigma[..., 6 * i + 1] + sigma[..., 6 * (i + 1) + 1]
                need = need + np.sqrt(sx * sx + sz * sz)
            bad = dist < need
            if not bad.any():
                break
            idx = np.nonzero(bad)
            px[idx + (np.full(len(idx[0]), i + 1),)] = rng.uniform(-1.0, 1.0, len(idx[0]))
            pz[idx + (np.full(len(idx[0]), i + 1),)] = rng.uniform(-1.0, 1.0, len(idx[0]))
    z = np.empty((B, N, U, 6))
    z[..., 0] = px
    z[..., 1] = pz
    z[..., 2] = theta
    z[..., 3] = pos_other[..., 2]
    z[..., 4] = pos_other[..., 3]
    z[..., 5] = pos_other[..., 4]
    return z.reshape(B, N, 6 * U), u.reshape(B, N, 2 * U)


def small_nominals(dyn: SmallDynamics, seed: int, count: int) -> tuple:
    """`count` nominal points (z, v) [count][nx], [count][nu] of the state and
    input sets: satellite, a unit quaternion, rates U(-1, 1), torques
    U(-1, 1); 3-D quadrotor, positions and velocities U(-1, 1), roll and
    pitch U(-0.5, 0.5), yaw U(-pi, pi), body rates U(-1, 1), thrust
    U(0.5, 1.5) m g, torques U(-0.05, 0.05)."""
    rng = rng_for(seed)
    if dyn.kind == "satellite":
        q = rng.normal(size=(count, 4))
        q /= np.linalg.norm(q, axis=1, keepdims=True)
        w = rng.uniform(-1.0, 1.0, (count, 3))
        return np.concatenate([q, w], 1), rng.uniform(-1.0, 1.0, (count, 3))
    z = np.empty((count, 12))
    z[:, 0:3] = rng.uniform(-1.0, 1.0, (count, 3))
    z[:, 3:5] = rng.uniform(-0.5, 0.5, (count, 2))
    z[:, 5] = rng.uniform(-np.pi, np.pi, count)
    z[:, 6:9] = rng.uniform(-1.0, 1.0, (count, 3))
    z[:, 9:12] = rng.uniform(-1.0, 1.0, (count, 3))
    v = np.empty((count, 4))
    v[:, 0] = rng.uniform(0.5, 1.5, count) * dyn.m * dyn.g
    v[:, 1:4] = rng.uniform(-0.05, 0.05, (count, 3))
    return z, v


def small_batch(dyn: SmallDynamics, seed: int, count: int, eps: float) -> AnalyticBatch:
    """The local sets of the tightness study: nominal points and the box
    (z, v) + eps [-1, 1]^(nx+nu), as one trajectory of `count` steps."""
    z, v = small_nominals(dyn, seed, count)
    sigma = np.full((count, dyn.n), float(eps))
    return AnalyticBatch(dyn, z[None], v[None], sigma[None], None)


def chain_batch(seed: int, batch: int, N: int, n_units: int,
                sigma_range=(0.01, 0.05), min_gap: float = 0.2) -> AnalyticBatch:
    """`batch` chain trajectories with per-coordinate radii U(sigma_range)."""
    dyn = ChainDynamics(n_units=n_units)
    rng = rng_for(seed)
    sigma = rng.uniform(sigma_range[0], sigma_range[1], (batch, N, dyn.n))
    z, v = _chain_nominal(rng, (batch, N), n_units, dyn.rest_len, min_gap, sigma)
    return AnalyticBatch(dyn, z, v, sigma, None)


def chain_cfg(seed: int = 2, N: int = 40, n_units: int = 28, batch: int = 1) -> AnalyticBatch:
    """28 coupled planar quadrotors (nx=168, nu=56), horizon 40, radii U(0.01, 0.05)."""
    return chain_batch(seed, batch, N, n_units)


# --------------------------------------------------------------------------
# neural-network workload

def mlp_weights(rng, widths) -> tuple:
    W, b = [], []
    for fan_in, fan_out in zip(widths[:-1], widths[1:]):
        W.append(rng.normal(0.0, np.sqrt(2.0 / fan_in), (fan_out, fan_in)).astype(np.float32))
        b.append(rng.uniform(-0.1, 0.1, fan_out).astype(np.float32))
    return W, b


def nn_cfg(seed: int = 1, batch: int = 64, N: int = 50, hidden: int = 256,
           nx: int = 12, nu: int = 4) -> NNBatch:
    """ReLU MLP (nx+nu)-h-h-h-nx, He-normal weights, residual next state."""
    rng = rng_for(seed)
    W, b = mlp_weights(rng, [nx + nu, hidden, hidden, hidden, nx])
    net = MLPNet(W, b, nx, nu, True)
    alpha = rng.uniform(-1.0, 1.0, (batch, N, nx + nu))
    sigma = rng.uniform(0.005, 0.05, (batch, N, nx + nu))
    return NNBatch(net, alpha[..., :nx].copy(), alpha[..., nx:].copy(), sigma, None)


# --------------------------------------------------------------------------
# tube/LEB fixed point

HOVER_Q = (100.0, 100.0, 10.0, 1.0, 1.0, 1.0)
HOVER_R = 0.1


def hover_lqr(dyn: ChainDynamics, Q=HOVER_Q, R=HOVER_R):
    """Hover linearisation of one planar quadrotor (theta=0, u1=u2=mg/2),
    forward-Euler discretised, and its discrete LQR gain for state weights
    diag(Q) and input weight R I2 (position-heavy, so the closed-loop tube
    stays well inside the spring separations)."""
    import scipy.linalg
    dt, m = dyn.dt, dyn.m
    Ac = np.zeros((6, 6))
    Ac[0, 3] = Ac[1, 4] = Ac[2, 5] = 1.0
    Ac[3, 2] = -dyn.g                      # -(u1+u2)/m cos(theta) at hover
    Bc = np.zeros((6, 2))
    Bc[4, 0] = Bc[4, 1] = 1.0 / m
    Bc[5, 0] = dyn.arm / dyn.inertia
    Bc[5, 1] = -dyn.arm / dyn.inertia
    A = np.eye(6) + dt * Ac
    Bm = dt * Bc
    Qm = np.diag(np.asarray(Q, dtype=np.float64))
    Rm = R * np.eye(2)
    P = scipy.linalg.solve_discrete_are(A, Bm, Qm, Rm)
    K = -np.linalg.solve(Rm + Bm.T @ P @ Bm, Bm.T @ P @ A)
    return A, Bm, K


def fixed_point_cfg(seed: int = 4, batch: int = 256, N: int = 40, n_units: int = 28,
                    e_scale: float = 2e-2) -> TubeProblem:
    """256 chain trajectories (nx=168) of horizon 40 with a decentralised
    hover-LQR closed loop and disturbance generator e_scale on (vx, vz) of
    every node.  Tube radii are unknowns of the fixed point, so the nominal
    spring separations keep a fixed margin of 0.6."""
    dyn = ChainDynamics(n_units=n_units)
    rng = rng_for(seed)
    z, v = _chain_nominal(rng, (batch, N), n_units, dyn.rest_len, 0.6, None)
    sigma = np.zeros((batch, N, dyn.n))
    mu = np.zeros((batch, N, dyn.n))
    A, Bm, K = hover_lqr(dyn)
    Acl = A + Bm @ K
    phi = np.zeros((N - 1, 8, 6))
    P = np.eye(6)
    for d in range(1, N):
        phi[d - 1, :6] = P
        phi[d - 1, 6:] = K @ P
        P = Acl @ P
    e = e_scale * np.array([0.0, 0.0, 0.0, 1.0, 1.0, 0.0])
    return TubeProblem(AnalyticBatch(dyn, z, v, sigma, mu), phi, e, K, Acl)


# --------------------------------------------------------------------------
# system-level synthesis layer (closed-loop responses from Riccati recursions)

@dataclass
class SlsProblem:
    """One controller update of chain trajectories: nominal (z, v), the
    diagonal SLS weights per (trajectory, k, j) and the disturbance model
    E(x) = [diag(e) | thrust columns] (nw = nx + n_units)."""
    dyn: ChainDynamics
    z: np.ndarray                 # [batch][N][nx]
    v: np.ndarray                 # [batch][N][nu]
    qx: np.ndarray                # [batch][N+1][N][nx]
    qu: np.ndarray                # [batch][N][N][nu]
    e: np.ndarray                 # [nx]
    thrust: float

    @property
    def batch(self) -> int:
        return self.z.shape[0]

    @property
    def N(self) -> int:
        return self.z.shape[1]


def sls_cfg(seed: int = 5, batch: int = 256, N: int = 40, n_units: int = 1, e_scale: float = 2e-2,
            thrust: float = 0.2, tau_max: float = 1.0) -> SlsProblem:
    """Planar quadrotor chains (the paper's planar quadrotor task has N = 40)
    with nominal states and inputs drawn like the chain workload (spring
    separations kept 0.6 clear of zero).  Weights: the hover tracking
    weights diag(Q~) = HOVER_Q per node and R~ = HOVER_R, plus dual weights
    U(0, tau_max) per (k, j, coordinate) standing in for the constraint
    duals of both faces of box constraints.  Disturbance: e_scale on every
    node's (vx, vz) and a thrust-magnitude disturbance `thrust` (newtons)."""
    dyn = ChainDynamics(n_units=n_units)
    rng = rng_for(seed)
    z, v = _chain_nominal(rng, (batch, N), n_units, dyn.rest_len, 0.6, None)
    qx = np.tile(np.asarray(HOVER_Q, dtype=np.float64), n_units) + \
        rng.uniform(0.0, tau_max, (batch, N + 1, N, dyn.nx))
    qu = HOVER_R + rng.uniform(0.0, tau_max, (batch, N, N, dyn.nu))
    e = np.tile(e_scale * np.array([0.0, 0.0, 0.0, 1.0, 1.0, 0.0]), n_units)
    return SlsProblem(dyn, z, v, qx, qu, e, float(thrust))


def random_ltv(seed: int, batch: int, N: int, nx: int, nu: int, scale: float = 0.1):
    """Random time-varying pairs A_k = I + scale G, B_k = scale H (G, H
    standard normal) [batch][N][nx][nx], [batch][N][nx][nu], and diagonal
    weights qx U(0.5, 2) [batch][N+1][N][nx], qu U(0.05, 0.5) [batch][N][N][nu]."""
    rng = rng_for(seed)
    A = np.eye(nx) + scale * rng.normal(size=(batch, N, nx, nx))
    B = scale * rng.normal(size=(batch, N, nx, nu))
    qx = rng.uniform(0.5, 2.0, (batch, N + 1, N, nx))
    qu = rng.uniform(0.05, 0.5, (batch, N, N, nu))
    return A, B, qx, qu


# --------------------------------------------------------------------------
# uneven batch

@dataclass
class MixedBatch:
    problems: list = field(default_factory=list)   # list of (kind, payload)


def mixed_batch_cfg(seed: int = 3, count: int = 256) -> MixedBatch:
    """Uneven problems: nx drawn from {6, 12, 48, 168}, horizons U{10..80}.
    nx=6 is the planar quadrotor, nx=12 an MLP (one shared net per hidden
    width, widths 128 and 256), nx=48 / 168 chains of 8 / 28 nodes."""
    rng = rng_for(seed)
    nxs = rng.choice([6, 12, 48, 168], size=count)
    Ns = rng.integers(10, 81, size=count)
    widths = rng.choice([128, 256], size=count)
    nets = {}
    for h, s in ((128, 31), (256, 32)):
        W, b = mlp_weights(rng_for(s), [16, h, h, h, 12])
        nets[h] = MLPNet(W, b, 12, 4, True)
    out = MixedBatch()
    for p in range(count):
        nx, N = int(nxs[p]), int(Ns[p])
        sub = int(rng.integers(0, 2**31 - 1))
        if nx == 6:
            out.problems.append(("analytic", planar_quad_cfg(sub, N)))
        elif nx == 12:
            r = rng_for(sub)
            net = nets[int(widths[p])]
            alpha = r.uniform(-1.0, 1.0, (1, N, 16))
            sigma = r.uniform(0.005, 0.05, (1, N, 16))
            out.problems.append(("nn", NNBatch(net, alpha[..., :12].copy(), alpha[..., 12:].copy(), sigma)))
        else:
            out.problems.append(("analytic", chain_batch(sub, 1, N, nx // 6)))
    return out


# --------------------------------------------------------------------------
# sample points inside boxes (violation checks)

def sample_box_points(rng, lo: np.ndarray, hi: np.ndarray, per_box: int) -> np.ndarray:
    """Points inside each box [lo, hi] (shape [U][n]) -> [U][per_box][n]:
    half uniform, a quarter random vertices, a quarter with a random subset
    of coordinates at a bound and the rest uniform."""
    U, n = lo.shape
    out = np.empty((U, per_box, n))
    n_uni = per_box // 2
    n_vert = per_box // 4
    n_mix = per_box - n_uni - n_vert
    w = hi - lo
    out[:, :n_uni] = lo[:, None] + w[:, None] * rng.random((U, n_uni, n))
    pick = rng.random((U, n_vert, n)) < 0.5
    out[:, n_uni:n_uni + n_vert] = np.where(pick, hi[:, None], lo[:, None])
    base = lo[:, None] + w[:, None] * rng.random((U, n_mix, n))
    at_bound = rng.random((U, n_mix, n)) < 0.5
    side = rng.random((U, n_mix, n)) < 0.5
    out[:, n_uni + n_vert:] = np.where(at_bound, np.where(side, hi[:, None], lo[:, None]), base)
    return out
