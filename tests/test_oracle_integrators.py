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
