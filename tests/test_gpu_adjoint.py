"""GPU adjoint (reverse pass of the Euler-Cromer step, frozen break schedule) against the
oracle's reverse-mode gradient, plus the recorded break schedule, state preservation,
argument errors and the torch.autograd path.

Both sides receive the same seed dL/du^T, computed from the oracle's forward run, and
the oracle runs with its own recorded break schedule (bit-identical to the GPU's, which
is checked separately).  Bar: 1e-10 norm-wise relative for the stiffness gradient and
relative for the load gradient.
"""
import dataclasses

import numpy as np
import pytest

import pd_inputs as pi
from parity import TOL_FP64, oracle_run, rel_err, say

pytestmark = pytest.mark.gpu

IMIN, IMAX = np.iinfo(np.int32).min, np.iinfo(np.int32).max


@pytest.fixture(scope="module", autouse=True)
def _lib():
    from paper_2105_04150_amd import _binding as B
    B.load()


def _initial_broken(w, row_ptr, col):
    if w.notch is None:
        return np.zeros(int(row_ptr[-1]), dtype=bool)
    return pi.notch_mask(w.ijk, row_ptr, col, *w.notch).astype(bool)


def _frozen(o, init):
    fr = o.break_step[: o.nnz].copy()
    fr[init] = IMIN
    return fr


def _gpu(w, mapping, lanes):
    from paper_2105_04150_amd import simulation_for
    return simulation_for(w, lanes=lanes, mapping=mapping)


@pytest.mark.parametrize("mapping,lanes", [("sliced", 4), ("staged", 1)])
def test_break_steps_bit_exact(mapping, lanes):
    w = pi.workload("block10", steps=1000)
    o = oracle_run(w, w.steps, record_breaks=True)
    exp = _frozen(o, _initial_broken(w, o.row_ptr, o.col))
    say(f"[run] break steps block10 {mapping}")
    g = _gpu(w, mapping, lanes)
    g.adj_forward(w.steps, 100)
    got = g.break_steps()
    nb = int((exp != IMAX).sum())
    say(f"[adjoint] break steps: {nb} slots broke, mismatched {int((got != exp).sum())}")
    assert nb > 1000
    assert np.array_equal(got, exp)
    assert rel_err(g.u(), o.u) <= TOL_FP64


def test_break_steps_notch_marked_before():
    w = dataclasses.replace(pi.workload("beam3pb", dims=(40, 10, 10), steps=50), scheme="euler_cromer")
    g = _gpu(w, "sliced", 1)
    rp, col = g.family()
    init = _initial_broken(w, rp, col)
    g.adj_forward(w.steps, 16)
    got = g.break_steps()
    assert init.sum() > 0
    assert np.array_equal(got[init], np.full(int(init.sum()), IMIN))
    assert np.all(got[~init] == IMAX)


CASES = [
    # name, overrides, checkpoint interval, mapping, lanes
    ("adjoint_beam", {"dims": (40, 12, 10), "steps": 1500}, 100, "sliced", 4),
    ("adjoint_beam", {"dims": (40, 12, 10), "steps": 1500}, 64, "staged", 1),   # ragged last segment
    ("adjoint_beam", {"dims": (40, 12, 10), "steps": 1500}, 100, "staged", 4),  # four wavefronts per slice
    ("block10", {"steps": 700}, 37, "staged", 2),
    ("block10", {"steps": 700}, 37, "sliced", 16),                              # linear BC schedule
    ("block10", {"steps": 700}, 700, "sliced", 1),                              # one segment
    ("block10", {"dims": (9, 7, 6), "steps": 300}, 1, "staged", 1),             # checkpoint every step
    ("adjoint_beam", {"dims": (30, 10, 8), "steps": 400}, 1, "sliced", 4),      # every level kept
]


@pytest.mark.parametrize("name,over,ckpt,mapping,lanes", CASES)
def test_adjoint_matches_oracle(name, over, ckpt, mapping, lanes):
    w = pi.workload(name, **over)
    o = oracle_run(w, w.steps, record_breaks=True)
    init = _initial_broken(w, o.row_ptr, o.col)
    frozen = _frozen(o, init)
    sensors, target = pi.adjoint_sensors(w, m=50)
    dldu = 2.0 * (o.u[sensors] - target)
    z = np.zeros((w.n, 3))
    gk_o, gA_o = o.adjoint_ec(frozen, w.steps, z, z, 0, sensors, dldu)
    say(f"[run] adjoint {name} {over} ckpt {ckpt} {mapping}-{lanes}")
    g = _gpu(w, mapping, lanes)
    g.adj_forward(w.steps, ckpt)
    gk, gA = g.adj_backward(sensors, dldu)
    ek = rel_err(gk, gk_o)
    eA = abs(gA - gA_o) / abs(gA_o) if gA_o != 0 else abs(gA)
    nbr = int((frozen != IMAX).sum() - init.sum())
    say(f"[adjoint] {name} {mapping}-{lanes} ckpt {ckpt}: grad_k rel {ek:.3e} (max |g| {np.abs(gk_o).max():.3e}), "
        f"grad_A rel {eA:.3e} ({gA_o:.6e}); frozen breaks {nbr}")
    assert np.abs(gk_o).max() > 0
    assert ek <= TOL_FP64
    assert eA <= TOL_FP64
    # a second reverse pass over the same recording gives the same gradients bit for bit
    gk2, gA2 = g.adj_backward(sensors, dldu)
    assert np.array_equal(gk, gk2) and gA == gA2


def test_adjoint_volumes_damping_velocity_bc(oracle_lib):
    """Per-node volumes, damping and a velocity-controlled face (adjoint passes through)."""
    from paper_2105_04150_amd import Simulation
    w = pi.workload("adjoint_beam", dims=(24, 8, 7), steps=400)
    rng = np.random.default_rng(11)
    vols = w.volume * rng.uniform(0.7, 1.3, w.n)
    eta = 3.0e6
    rp, col = oracle_lib.family(w.coords, w.horizon)
    g_field = pi.gaussian_node_field(w.dims, *w.stiffness_field)
    k = pi.slot_stiffness(w.c, g_field, rp, col)
    bhat, bmag = w.body_force
    bcs = w.bcs + [pi.BCSpec(pi.face_nodes(w.ijk, 1, w.dims[1] - 1), 0b010, pi.BC_VEL, (0.0, 0.05, 0.0),
                             pi.SCHED_LINEAR)]
    o = oracle_lib.OracleSim(w.coords, rp, col, c=w.c, s0=w.s0, rho=w.rho, dt=w.dt, vol=vols, eta=eta,
                             kslot=k, bhat=bhat, bmag=bmag, bcs=bcs, record_breaks=True)
    o.run(w.steps)
    frozen = o.break_step[: o.nnz].copy()
    sensors, target = pi.adjoint_sensors(w, m=40)
    dldu = 2.0 * (o.u[sensors] - target)
    z = np.zeros((w.n, 3))
    gk_o, gA_o = o.adjoint_ec(frozen, w.steps, z, z, 0, sensors, dldu)
    for mapping, lanes in (("sliced", 1), ("staged", 1)):
        with Simulation() as g:
            g.set_mapping(mapping, lanes)
            g.build_family(w.coords, w.horizon)
            g.set_integrator("euler_cromer", w.dt)
            g.set_material(w.rho, w.c, w.s0, eta, volumes=vols)
            for bc in bcs:
                g.set_bcs(bc.nodes, bc.comp_mask, bc.kind, bc.value, bc.sched)
            g.set_bond_stiffness(k)
            g.set_body_force(bhat, bmag)
            g.adj_forward(w.steps, 50)
            gk, gA = g.adj_backward(sensors, dldu)
            ek, eA = rel_err(gk, gk_o), abs(gA - gA_o) / abs(gA_o)
            say(f"[adjoint] volumes+damping+vel-bc {mapping}: grad_k rel {ek:.3e} grad_A rel {eA:.3e} "
                f"({gA!r} vs {gA_o!r})")
            assert ek <= TOL_FP64 and eA <= TOL_FP64


def test_backward_leaves_state_unchanged():
    from paper_2105_04150_amd import simulation_for
    w = pi.workload("block10", dims=(10, 9, 8), steps=400)
    sensors, target = pi.adjoint_sensors(w, m=20)
    g = simulation_for(w, lanes=4)
    g.adj_forward(250, 60)
    u1, v1, b1, st1 = g.u(), g.v(), g.broken(), g.step_count
    g.adj_backward(sensors, 2.0 * (u1[sensors] - target))
    assert np.array_equal(g.u(), u1) and np.array_equal(g.v(), v1) and np.array_equal(g.broken(), b1)
    assert g.step_count == st1
    g.step(150)
    ref = simulation_for(w, lanes=4)
    ref.step(400)
    assert np.array_equal(g.u(), ref.u()) and np.array_equal(g.broken(), ref.broken())


def test_adjoint_argument_errors():
    from paper_2105_04150_amd import PD_FP32, PdmiError, Simulation, simulation_for
    w = pi.workload("block10", dims=(6, 6, 6), steps=20)
    g = simulation_for(w, lanes=1)
    sensors, target = pi.adjoint_sensors(w, m=5)
    with pytest.raises(PdmiError):  # nothing recorded yet
        g.adj_backward(sensors, np.zeros((5, 3)))
    assert np.all(g.break_steps() == IMAX)  # intact problem, nothing broken yet
    g.adj_forward(10, 4)
    gk, gA = g.adj_backward(sensors, np.zeros((5, 3)))
    assert not gk.any() and gA == 0.0
    with pytest.raises(PdmiError):
        g.adj_backward(np.array([w.n]), np.zeros((1, 3)))  # sensor out of range
    with pytest.raises(PdmiError):
        g.adj_backward(sensors, np.full((5, 3), np.nan))
    g.step(1)  # the recording is discarded by any further step
    with pytest.raises(PdmiError):
        g.adj_backward(sensors, np.zeros((5, 3)))
    g.set_mapping("staged", 1)
    g.adj_forward(10, 4)
    g.set_mapping("staged", 2)  # another launch shape discards it too
    with pytest.raises(PdmiError):
        g.adj_backward(sensors, np.zeros((5, 3)))
    with pytest.raises(PdmiError):
        g.adj_forward(0, 4)
    with pytest.raises(PdmiError):
        g.adj_forward(10, 0)
    rp, col = g.family()
    k = np.full(rp[-1], w.c)
    k[0] *= 1.5  # one slot of a bond differs from its partner
    g.set_bond_stiffness(k)
    with pytest.raises(PdmiError):
        g.adj_forward(10, 4)
    g.set_bond_stiffness(None)
    g.set_integrator("velocity_verlet", w.dt)
    with pytest.raises(PdmiError):
        g.adj_forward(10, 4)
    with Simulation(precision=PD_FP32) as f:
        f.build_family(w.coords, w.horizon)
        f.set_material(w.rho, w.c, w.s0, 0.0, w.volume)
        with pytest.raises(PdmiError):
            f.adj_forward(10, 4)


def test_autograd_function_and_central_differences():
    """loss.backward() through the autograd Function equals the library's reverse pass; the
    gradient agrees with central differences of the GPU forward run on the largest slots."""
    import torch
    from paper_2105_04150_amd import simulation_for
    from paper_2105_04150_amd.adjoint import AdjointProblem, sensor_displacement
    w = pi.workload("adjoint_beam", dims=(30, 10, 8), steps=300)
    sim = simulation_for(w, lanes=4)
    rp, col = sim.family()
    k0 = pi.slot_stiffness(w.c, pi.gaussian_node_field(w.dims, *w.stiffness_field), rp, col)
    bhat, bmag = w.body_force
    sensors, target = pi.adjoint_sensors(w, m=30)
    prob = AdjointProblem(sim, bhat, sensors, w.steps, ckpt_every=40)
    k = torch.tensor(k0, dtype=torch.float64, requires_grad=True)
    A = torch.tensor(bmag, dtype=torch.float64, requires_grad=True)
    tgt = torch.tensor(target)
    u = sensor_displacement(k, A, prob)
    loss = ((u - tgt) ** 2).sum()
    loss.backward()
    gk, gA = k.grad.numpy(), float(A.grad)
    gk_d, gA_d = sim.adj_backward(sensors, 2.0 * (u.detach().numpy() - target))
    assert np.array_equal(gk, gk_d) and gA == gA_d

    def plain_loss(kk, aa):
        s = simulation_for(w, lanes=4)
        s.set_bond_stiffness(kk)
        s.set_body_force(bhat, aa)
        s.step(w.steps)
        d = s.u()[sensors] - target
        return float((d * d).sum())

    for b in np.argsort(-np.abs(gk))[:3]:
        h = 1e-6 * k0[b]
        kp, km = k0.copy(), k0.copy()
        kp[b] += h
        km[b] -= h
        fd = (plain_loss(kp, bmag) - plain_loss(km, bmag)) / (2 * h)
        say(f"[adjoint] FD slot {b}: adjoint {gk[b]:.6e} FD {fd:.6e} rel {abs(gk[b] - fd) / abs(fd):.2e}")
        assert gk[b] == pytest.approx(fd, rel=1e-5)
    hA = 1e-6 * bmag
    fdA = (plain_loss(k0, bmag + hA) - plain_loss(k0, bmag - hA)) / (2 * hA)
    say(f"[adjoint] FD load: adjoint {gA:.6e} FD {fdA:.6e}")
    assert gA == pytest.approx(fdA, rel=1e-6)


def test_backward_refuses_a_replaced_recording():
    """Each pd_adj_forward hands out a recording id; a backward asked for an earlier
    recording than the one the simulation holds raises instead of returning the later
    run's gradient, through the C ABI and through the autograd Function."""
    import torch
    from paper_2105_04150_amd import PdmiError, simulation_for
    from paper_2105_04150_amd.adjoint import AdjointProblem, sensor_displacement
    w = pi.workload("adjoint_beam", dims=(20, 8, 6), steps=60)
    sim = simulation_for(w, lanes=4)
    rp, col = sim.family()
    k0 = pi.slot_stiffness(w.c, pi.gaussian_node_field(w.dims, *w.stiffness_field), rp, col)
    bhat, bmag = w.body_force
    sensors, target = pi.adjoint_sensors(w, m=10)
    prob = AdjointProblem(sim, bhat, sensors, w.steps, ckpt_every=16)
    prob.reset(k0, bmag)
    r1 = sim.adj_forward(w.steps, 16)
    dl = np.ones((len(sensors), 3))
    g1 = sim.adj_backward(sensors, dl, r1)
    prob.reset(k0 * 1.01, bmag)
    r2 = sim.adj_forward(w.steps, 16)
    assert r1 > 0 and r2 > r1
    with pytest.raises(PdmiError):
        sim.adj_backward(sensors, dl, r1)
    g2 = sim.adj_backward(sensors, dl, r2)
    g0 = sim.adj_backward(sensors, dl)  # 0: the current recording
    assert np.array_equal(g2[0], g0[0]) and not np.array_equal(g1[0], g2[0])
    # two forwards of the autograd Function on one problem, then the first one's backward
    k = torch.tensor(k0, dtype=torch.float64, requires_grad=True)
    A = torch.tensor(bmag, dtype=torch.float64, requires_grad=True)
    u1 = sensor_displacement(k, A, prob)
    u2 = sensor_displacement(k * 1.01, A, prob)
    with pytest.raises(PdmiError):
        u1.sum().backward()
    u2.sum().backward()
    assert k.grad is not None and np.isfinite(k.grad.numpy()).all()
    say("[adjoint] a replaced recording is refused; the current one differentiates")
