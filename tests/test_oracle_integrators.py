"""Pins of the oracle's time integration and boundary conditions.

A collinear two-node bond is an exactly linear spring while intact (s = Delta/L), so
each scheme's recurrence is a 2x2 matrix power; other checks use conservation laws,
time reversibility and closed-form break times.
"""
import numpy as np
import pytest

import pd_inputs as pi

RHO, C, V, L = 2400.0, 1.0e20, 1.0e-9, 1.0e-3


def _pair(oracle_lib, scheme, dt, fixed0=True, s0=10.0, bcs=None, **kw):
    x = np.array([[0.0, 0.0, 0.0], [L, 0.0, 0.0]])
    rp, col = oracle_lib.family(x, 1.5 * L)
    if bcs is None:
        bcs = [pi.BCSpec(np.array([0]), 0b111, pi.BC_DISP, (0.0, 0.0, 0.0), pi.SCHED_CONST)] if fixed0 else []
    return oracle_lib.OracleSim(x, rp, col, c=C, s0=s0, rho=RHO, dt=dt, vol=V, scheme=scheme,
                                bcs=bcs, record_breaks=True, **kw)


def _matrix(scheme, kappa, dt):
    if scheme == "euler_cromer":
        return np.array([[1 - dt * dt * kappa, dt], [-dt * kappa, 1.0]])
    if scheme == "forward_euler":
        return np.array([[1.0, dt], [-dt * kappa, 1.0]])
    h = 1 - dt * dt * kappa / 2
    return np.array([[h, dt], [-dt * kappa * (1 - dt * dt * kappa / 4), h]])


@pytest.mark.parametrize("scheme", ["euler_cromer", "velocity_verlet", "forward_euler"])
def test_linear_spring_recurrence(oracle_lib, scheme):
    kappa = C * V / (RHO * L)                 # F_1 = -c V (Delta / L)
    dt = 0.1 / np.sqrt(kappa)
    nsteps = 400 if scheme != "forward_euler" else 60
    sim = _pair(oracle_lib, scheme, dt)
    d0, v0 = 2e-7, 3e-3
    sim.set_state(u=np.array([[0, 0, 0], [d0, 0, 0]]), v=np.array([[0, 0, 0], [v0, 0, 0]]))
    M = _matrix(scheme, kappa, dt)
    z = np.array([d0, v0])
    for k in range(nsteps):
        sim.run(1)
        z = M @ z
        assert sim.u[1, 0] == pytest.approx(z[0], abs=1e-12 * d0 * (k + 1) ** 0.5)
        assert sim.v[1, 0] == pytest.approx(z[1], abs=1e-12 * v0 * (k + 1) ** 0.5 + 1e-12 * np.sqrt(kappa) * d0)
    assert np.all(sim.u[0] == 0.0) and np.all(sim.v[0] == 0.0)
    assert np.all(sim.u[1, 1:] == 0.0)


def test_free_pair_momentum_exact(oracle_lib):
    sim = _pair(oracle_lib, "euler_cromer", 1e-7, fixed0=False)
    sim.set_state(u=np.array([[0, 0, 0], [1e-7, 2e-8, 0]]))
    sim.run(300)
    assert np.all(sim.v[0] == -sim.v[1])


@pytest.mark.parametrize("scheme", ["euler_cromer", "velocity_verlet"])
def test_free_body_momentum_conserved(oracle_lib, scheme):
    x, _ = pi.lattice((6, 5, 4), 1e-3, 1e-3, seed=8)
    rp, col = oracle_lib.family(x, 3.015e-3)
    sim = oracle_lib.OracleSim(x, rp, col, c=pi.pmb_micromodulus(1.4e10, 3.015e-3), s0=10.0,
                               rho=RHO, dt=1e-7, vol=V, scheme=scheme)
    u0 = np.random.default_rng(2).normal(size=x.shape) * 1e-6
    sim.set_state(u=u0)
    sim.run(200)
    p = sim.v.sum(0)
    assert np.abs(p).max() <= 1e-12 * np.abs(sim.v).sum()


def test_velocity_verlet_time_reversible(oracle_lib):
    x, _ = pi.lattice((5, 5, 5), 1e-3, 1e-3, seed=6)
    rp, col = oracle_lib.family(x, 3.015e-3)
    sim = oracle_lib.OracleSim(x, rp, col, c=pi.pmb_micromodulus(1.4e10, 3.015e-3), s0=10.0,
                               rho=RHO, dt=1e-7, vol=V, scheme="velocity_verlet")
    rng = np.random.default_rng(3)
    u0 = rng.normal(size=x.shape) * 1e-6
    v0 = rng.normal(size=x.shape) * 1e-2
    sim.set_state(u=u0, v=v0)
    sim.run(300)
    umax = np.abs(sim.u).max()
    sim.set_state(v=-sim.v, a_valid=0)
    sim.run(300)
    assert np.abs(sim.u - u0).max() <= 1e-12 * umax
    assert np.abs(sim.v + v0).max() <= 1e-10 * np.abs(v0).max()


def test_forward_euler_unstable_euler_cromer_bounded(oracle_lib):
    """Forward Euler amplifies the stiffest mode every step at dt = 1e-7 s; Euler-Cromer does not."""
    w = pi.workload("block10", dims=(6, 6, 6))
    out = {}
    for scheme in ("forward_euler", "euler_cromer"):
        rp, col = oracle_lib.family(w.coords, w.horizon)
        sim = oracle_lib.OracleSim(w.coords, rp, col, c=w.c, s0=10.0, rho=w.rho, dt=w.dt,
                                   vol=w.volume, scheme=scheme)
        sim.set_state(u=np.random.default_rng(0).normal(size=w.coords.shape) * 1e-9)
        sim.run(400)
        out[scheme] = np.abs(sim.u).max()
    assert out["forward_euler"] > 1e3 * out["euler_cromer"]


def test_displacement_bc_linear_schedule_exact(oracle_lib):
    w = pi.workload("block10", dims=(5, 5, 5))
    rp, col = oracle_lib.family(w.coords, w.horizon)
    sim = oracle_lib.OracleSim(w.coords, rp, col, c=w.c, s0=w.s0, rho=w.rho, dt=w.dt,
                               vol=w.volume, bcs=w.bcs)
    sim.run(37)
    top = pi.face_nodes(w.ijk, 2, 4)
    bot = pi.face_nodes(w.ijk, 2, 0)
    assert np.all(sim.u[top, 2] == 0.1 * (37 * w.dt))
    assert np.all(sim.v[top, 2] == 0.1)
    assert np.all(sim.u[bot] == 0.0) and np.all(sim.v[bot] == 0.0)
    assert np.any(sim.u[top, 0] != 0.0)          # x, y of the top layer stay free


@pytest.mark.parametrize("scheme", ["euler_cromer", "velocity_verlet"])
def test_single_bond_pull_breaks_at_predicted_step(oracle_lib, scheme):
    """Node 1 driven at constant velocity: the bond breaks in the first pass with u/L >= s0."""
    vel, dt, s0 = 0.037, 1e-7, 1e-3
    bcs = [pi.BCSpec(np.array([0]), 0b111, pi.BC_DISP, (0.0, 0.0, 0.0), pi.SCHED_CONST),
           pi.BCSpec(np.array([1]), 0b111, pi.BC_VEL, (vel, 0.0, 0.0), pi.SCHED_CONST)]
    sim = _pair(oracle_lib, scheme, dt, s0=s0, bcs=bcs)
    sim.run(400)
    # displacement after k steps is k*dt*vel; first k with k*dt*vel/L >= s0 is 271
    assert np.all(sim.break_step[:2] == 271)
    assert sim.u[1, 0] == pytest.approx(400 * dt * vel, rel=1e-12)


# ---------------------------------------------------------------- damping (Sec. 2.3)
# The damped equation of motion adds -eta v to the force density.  With gamma = eta/rho and
# kappa = c V/(rho L), node 1 of the fixed-free collinear pair obeys x'' = -kappa x - gamma x'.
# Euler-Cromer takes the drag on the velocity of the start of the step; velocity Verlet
# (Eqs. Velocity_Verlet1-2) takes it on the half-step velocity v + dt a/2, and its first
# acceleration comes from a force pass on the initial state with the drag on v0.

def _damped_ec_matrix(kappa, gamma, dt):
    # v' = (1 - gamma dt) v - kappa dt x;  x' = x + dt v'
    return np.array([[1 - dt * dt * kappa, dt * (1 - gamma * dt)],
                     [-dt * kappa, 1 - gamma * dt]])


def _damped_vv_matrix(kappa, gamma, dt):
    # state (x, v, a):  x' = x + dt v + dt^2/2 a;  a' = -kappa x' - gamma (v + dt/2 a);
    # v' = v + dt/2 (a + a')
    xr = np.array([1.0, dt, dt * dt / 2])
    ar = -kappa * xr - gamma * np.array([0.0, 1.0, dt / 2])
    vr = np.array([0.0, 1.0, dt / 2]) + (dt / 2) * ar
    return np.vstack([xr, vr, ar])


@pytest.mark.parametrize("scheme", ["euler_cromer", "velocity_verlet"])
def test_damped_linear_spring_recurrence(oracle_lib, scheme):
    kappa = C * V / (RHO * L)
    omega = np.sqrt(kappa)
    dt = 0.1 / omega
    gamma = 0.2 * omega                       # under-damped: the amplitude falls by e^-4 in 400 steps
    sim = _pair(oracle_lib, scheme, dt, eta=gamma * RHO)
    d0, v0 = 2e-7, 3e-3
    sim.set_state(u=np.array([[0, 0, 0], [d0, 0, 0]]), v=np.array([[0, 0, 0], [v0, 0, 0]]))
    if scheme == "euler_cromer":
        M, z = _damped_ec_matrix(kappa, gamma, dt), np.array([d0, v0])
    else:
        M, z = _damped_vv_matrix(kappa, gamma, dt), np.array([d0, v0, -kappa * d0 - gamma * v0])
    scale_v = v0 + omega * d0
    for k in range(400):
        sim.run(1)
        z = M @ z
        assert sim.u[1, 0] == pytest.approx(z[0], abs=1e-12 * d0 * (k + 1) ** 0.5)
        assert sim.v[1, 0] == pytest.approx(z[1], abs=1e-12 * scale_v * (k + 1) ** 0.5)
        if scheme == "velocity_verlet":
            assert sim.a[1, 0] == pytest.approx(z[2], abs=1e-12 * omega * scale_v * (k + 1) ** 0.5)
    assert abs(z[0]) < 0.05 * (d0 + v0 / omega)   # the drag has taken the energy out
    assert np.all(sim.u[0] == 0.0) and np.all(sim.u[1, 1:] == 0.0)


@pytest.mark.parametrize("scheme", ["euler_cromer", "velocity_verlet"])
def test_free_node_drag(oracle_lib, scheme):
    """A node without bonds under drag alone: Euler-Cromer gives v_k = v0 (1 - gamma dt)^k
    exactly; velocity Verlet follows its 2x2 recurrence on (v, a) from a0 = -gamma v0; the
    displacement is the sum of the scheme's position updates."""
    x = np.array([[0.0, 0.0, 0.0]])
    rp, col = oracle_lib.family(x, 1e-3)
    gamma, dt = 2.0e5, 1e-7
    sim = oracle_lib.OracleSim(x, rp, col, c=C, s0=1.0, rho=RHO, dt=dt, vol=V, scheme=scheme,
                               eta=gamma * RHO)
    v0 = np.array([1.0e-2, -3.0e-3, 5.0e-4])
    sim.set_state(v=v0[None, :])
    u = np.zeros(3)
    v = v0.copy()
    a = -gamma * v0
    for k in range(1, 301):
        sim.run(1)
        if scheme == "euler_cromer":
            v = v0 * (1 - gamma * dt) ** k
            u = u + dt * v
        else:
            u = u + dt * v + dt * dt / 2 * a
            an = -gamma * (v + dt / 2 * a)
            v, a = v + dt / 2 * (a + an), an
        assert np.allclose(sim.v[0], v, rtol=1e-13, atol=0)
        assert np.allclose(sim.u[0], u, rtol=1e-12, atol=0)
    # both approach the continuous solution v0 exp(-gamma t) to first order in dt
    assert np.allclose(sim.v[0], v0 * np.exp(-gamma * 300 * dt), rtol=300 * (gamma * dt) ** 2)


@pytest.mark.parametrize("scheme", ["euler_cromer", "velocity_verlet"])
def test_damped_pair_converges_to_damped_oscillator(oracle_lib, scheme):
    """Halving dt at least nearly halves the distance to the continuous damped oscillator
    x(t) = exp(-gamma t/2) (d0 cos(w t) + (v0 + gamma d0/2)/w sin(w t)), w^2 = kappa - gamma^2/4
    (a damping sign error or a dropped drag fails this at any dt)."""
    kappa = C * V / (RHO * L)
    omega = np.sqrt(kappa)
    gamma = 0.3 * omega
    wd = np.sqrt(kappa - gamma * gamma / 4)
    d0, v0 = 2e-7, 1e-3
    T = 30.0 / omega

    def exact(t):
        return np.exp(-gamma * t / 2) * (d0 * np.cos(wd * t) + (v0 + gamma * d0 / 2) / wd * np.sin(wd * t))

    errs = []
    for nsteps in (1500, 3000, 6000):
        dt = T / nsteps
        sim = _pair(oracle_lib, scheme, dt, eta=gamma * RHO)
        sim.set_state(u=np.array([[0, 0, 0], [d0, 0, 0]]), v=np.array([[0, 0, 0], [v0, 0, 0]]))
        sim.run(nsteps)
        errs.append(abs(sim.u[1, 0] - exact(T)))
    amp = d0 + v0 / omega
    assert errs[0] < 0.02 * amp
    assert errs[1] < 0.6 * errs[0] and errs[2] < 0.6 * errs[1]
