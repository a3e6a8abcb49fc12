"""Pins of the oracle's discretised dynamics f and point Jacobians
(eq. linearizations): the Jacobian against central differences of f, and
f against physical invariants of the planar-quadrotor chain (hover is an
equilibrium, free fall loses g dt of vertical speed, a thrust difference
spins the body, a spring at rest length exerts no force and a stretched one
pulls the nodes together), which fix the affine part independently of how
it is written."""
import numpy as np
import pytest


def _fd_jacobian(orc, d, z, v, h=1e-6):
    nx, nu = d.nx, d.nu
    A = np.zeros((nx, nx))
    B = np.zeros((nx, nu))
    for k in range(nx):
        e = np.zeros(nx); e[k] = h
        A[:, k] = (orc.step(d, z + e, v) - orc.step(d, z - e, v)) / (2 * h)
    for k in range(nu):
        e = np.zeros(nu); e[k] = h
        B[:, k] = (orc.step(d, z, v + e) - orc.step(d, z, v - e)) / (2 * h)
    return A, B


@pytest.mark.parametrize("kind", ["chain3", "quadratic", "sin1d", "sincos2d"])
def test_jacobian_matches_central_differences(orc, kind):
    rng = np.random.default_rng(5)
    if kind == "chain3":
        d = orc.Dyn.chain(3)
        z = rng.uniform(-1, 1, 18)
        z[6::6] += 1.0 * np.arange(1, 3)          # rest lattice offsets keep the springs non-degenerate
        z[2::6] = rng.uniform(-0.5, 0.5, 3)
        v = rng.uniform(3, 7, 6)
    elif kind == "quadratic":
        Q = rng.normal(size=(3, 5, 5))
        Q = 0.5 * (Q + Q.transpose(0, 2, 1))
        d = orc.Dyn("quadratic", 3, 2, Q=Q)
        z, v = rng.uniform(-1, 1, 3), rng.uniform(-1, 1, 2)
    elif kind == "sin1d":
        d = orc.Dyn("sin1d", 1, 0)
        z, v = rng.uniform(-3, 3, 1), np.zeros(0)
    else:
        d = orc.Dyn("sincos2d", 2, 0)
        z, v = rng.uniform(-3, 3, 2), np.zeros(0)
    A, B = orc.jacobian(d, z, v)
    Af, Bf = _fd_jacobian(orc, d, z, v)
    scale = max(1.0, np.abs(A).max())
    assert np.abs(A - Af).max() <= 1e-7 * scale
    if d.nu:
        assert np.abs(B - Bf).max() <= 1e-7 * scale


def test_chain_hover_is_equilibrium(orc):
    """theta = 0, u1 = u2 = m g / 2, zero velocities, springs at rest
    length: the next state equals the state."""
    d = orc.Dyn.chain(4)
    z = np.zeros(24)                        # positions are offsets from the rest lattice (i L0, 0)
    z[1::6] = 0.25                          # all nodes at one height: every spring at rest length
    v = np.full(8, d.c.m * d.c.g / 2)
    f = orc.step(d, z, v)
    np.testing.assert_allclose(f, z, atol=1e-14)


def test_chain_free_fall_spin_and_velocity_integration(orc):
    d = orc.Dyn.chain(1)
    dt, g, arm, J = d.c.dt, d.c.g, d.c.arm, d.c.inertia
    z = np.array([0.1, 0.2, 0.0, 0.5, -0.3, 0.7])
    f = orc.step(d, z, np.zeros(2))                     # no thrust: free fall
    np.testing.assert_allclose(f, [0.1 + dt * 0.5, 0.2 - dt * 0.3, dt * 0.7, 0.5, -0.3 - dt * g, 0.7], atol=1e-15)
    f2 = orc.step(d, z, np.array([1.0, 0.0]))           # u1 > u2 at theta = 0: pure upward push and spin
    assert f2[5] - f[5] == pytest.approx(dt * arm / J)
    assert f2[4] - f[4] == pytest.approx(dt / d.c.m)
    assert f2[3] == pytest.approx(f[3])


def test_chain_spring_pulls_stretched_nodes_together(orc):
    d = orc.Dyn.chain(2)
    dt, m = d.c.dt, d.c.m
    z = np.zeros(12)
    v = np.full(4, d.c.m * d.c.g / 2)
    f0 = orc.step(d, z, v)                              # at rest length: no force
    np.testing.assert_allclose(f0, z, atol=1e-14)
    z2 = z.copy()
    z2[6] = 0.5                                         # node 1 moved 0.5 along x: stretched by 0.5
    f = orc.step(d, z2, v)
    k = d.c.k_spring
    assert f[3] == pytest.approx(dt * k * 0.5 / m)      # node 0 pulled towards +x
    assert f[9] == pytest.approx(-dt * k * 0.5 / m)     # node 1 pulled towards -x
