"""GPU (HIP library, FP64) against the FP64 CPU oracle on the same seeded inputs.

Bar: bit-identical families and broken-bond sets; displacement within 1e-10
norm-wise relative (largest component error over the largest reference component);
damage within summation rounding.
"""
import numpy as np
import pytest

import pd_inputs as pi
from parity import TOL_FP64, compare, gpu_run, oracle_run, rate_err, rel_err, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    from paper_2105_04150_amd import _binding as B
    B.load()


@pytest.mark.parametrize("name,over", [("block10", {}), ("beam3pb", {"dims": (60, 12, 12)}),
                                       ("cube100", {"dims": (12, 13, 11)}),
                                       ("cube100_wide", {"dims": (13, 12, 14)})])
@pytest.mark.parametrize("order", ["natural", "morton"])
def test_family_bit_exact(oracle_lib, name, over, order):
    from paper_2105_04150_amd import Simulation
    w = pi.workload(name, **over)
    say(f"[family] {name} {over} {order}")
    rp, col = oracle_lib.family(w.coords, w.horizon)
    with Simulation() as sim:
        sim.build_family(w.coords, w.horizon, order)
        grp, gcol = sim.family()
    assert np.array_equal(rp, grp) and np.array_equal(col, gcol)


MAPPINGS = [("sliced", 1), ("sliced", 4), ("sliced", 16), ("sliced", 64), ("staged", 1), ("staged", 2),
            ("staged", 4)]


@pytest.mark.parametrize("mapping,lanes", MAPPINGS)
def test_block10_euler_cromer(oracle_lib, mapping, lanes):
    """1,000-node jittered block, 1,000 Euler-Cromer steps, fractures (about 7.8k slots)."""
    w = pi.workload("block10")
    o = oracle_run(w, w.steps)
    say(f"[run] block10 {mapping} lanes={lanes}")
    g = gpu_run(w, w.steps, lanes=lanes, mapping=mapping)
    eu, ev, mism, ephi = compare(g, o, TOL_FP64, f"block10 {mapping} lanes={lanes}")
    assert o.broken_mask.sum() > 5000
    assert mism == 0
    assert eu <= TOL_FP64 and ev <= TOL_FP64
    assert ephi <= 1e-13


@pytest.mark.parametrize("mapping,lanes", [("sliced", 1), ("sliced", 16), ("staged", 1), ("staged", 4)])
def test_notched_beam_velocity_verlet(oracle_lib, mapping, lanes):
    """Notched three-point-bend beam (reduced length), velocity Verlet, velocity-controlled load."""
    w = pi.workload("beam3pb", dims=(60, 12, 12), steps=1500)
    o = oracle_run(w, w.steps)
    say(f"[run] beam3pb-60 {mapping} lanes={lanes}")
    g = gpu_run(w, w.steps, lanes=lanes, chunks=[1, 700, 799], mapping=mapping)
    eu, ev, mism, ephi = compare(g, o, TOL_FP64, f"beam3pb-60 lanes={lanes}")
    assert mism == 0 and eu <= TOL_FP64 and ev <= TOL_FP64 and ephi <= 1e-13
    assert rate_err(g.a(), o.a, w.dt, o.u, power=2) <= TOL_FP64


@pytest.mark.parametrize("name", ["cube100", "cube100_wide"])
@pytest.mark.parametrize("order,mapping", [("morton", "sliced"), ("natural", "staged"), ("morton", "staged")])
def test_cube(oracle_lib, name, order, mapping):
    """Uniaxial tension of a cube, short and wide horizons, both node orders and mappings."""
    w = pi.workload(name, dims=(24, 20, 18), steps=300)
    o = oracle_run(w, w.steps)
    say(f"[run] {name}-small {order} {mapping}")
    g = gpu_run(w, w.steps, order=order, mapping=mapping)
    eu, ev, mism, ephi = compare(g, o, TOL_FP64, f"{name} 24x20x18 {order} {mapping}")
    assert mism == 0 and eu <= TOL_FP64 and ephi <= 1e-13


@pytest.mark.parametrize("mapping,lanes", [("sliced", 4), ("staged", 1), ("staged", 2)])
def test_stiffness_field_body_force(oracle_lib, mapping, lanes):
    """Per-slot stiffness field c exp(g) and a body-force load (the adjoint workload, reduced)."""
    w = pi.workload("adjoint_beam", dims=(30, 10, 8), steps=400)
    o = oracle_run(w, w.steps)
    say(f"[run] adjoint_beam-30 forward {mapping}")
    g = gpu_run(w, w.steps, lanes=lanes, mapping=mapping)
    eu, ev, mism, ephi = compare(g, o, TOL_FP64, "adjoint_beam 30x10x8")
    assert mism == 0 and eu <= TOL_FP64


@pytest.mark.parametrize("mapping,lanes", [("sliced", 16), ("staged", 1), ("staged", 4)])
def test_nonuniform_volumes_and_damping(oracle_lib, mapping, lanes):
    """Per-node volumes and dynamic-relaxation damping with Euler-Cromer."""
    from paper_2105_04150_amd import Simulation
    w = pi.workload("block10", dims=(9, 8, 7), steps=400)
    rng = np.random.default_rng(5)
    vols = w.volume * rng.uniform(0.7, 1.3, w.n)
    eta = 4.0e6
    rp, col = oracle_lib.family(w.coords, w.horizon)
    o = oracle_lib.OracleSim(w.coords, rp, col, c=w.c, s0=w.s0, rho=w.rho, dt=w.dt, vol=vols,
                             eta=eta, bcs=w.bcs)
    o.run(w.steps)
    say(f"[run] block 9x8x7 volumes + damping {mapping}")
    with Simulation() as g:
        g.set_mapping(mapping, lanes)
        g.build_family(w.coords, w.horizon)
        g.set_integrator("euler_cromer", w.dt)
        g.set_material(w.rho, w.c, w.s0, eta, volumes=vols)
        for bc in w.bcs:
            g.set_bcs(bc.nodes, bc.comp_mask, bc.kind, bc.value, bc.sched)
        g.step(w.steps)
        eu, ev, mism, ephi = compare(g, o, TOL_FP64, "volumes+damping")
    assert mism == 0 and eu <= TOL_FP64 and ephi <= 1e-13


@pytest.mark.parametrize("mapping", ["sliced", "staged"])
def test_batched_instances_match_independent_oracles(oracle_lib, mapping):
    """Three uneven beams advanced together equal three independent oracle runs."""
    from paper_2105_04150_amd import Simulation, apply_workload
    ws = pi.batch_instances(count=3, scale_lo=0.4, scale_hi=0.7, steps=300)
    say(f"[run] batch of 3 ({mapping}): " + ", ".join(str(w.dims) for w in ws))
    with Simulation() as g:
        g.set_mapping(mapping, 4 if mapping == "sliced" else 0)
        g.build_family_batch([w.coords for w in ws], [w.horizon for w in ws])
        g.set_integrator("euler_cromer", ws[0].dt)
        for b, w in enumerate(ws):
            apply_workload(g, w, inst=b)
        g.step(ws[0].steps)
        for b, w in enumerate(ws):
            o = oracle_run(w, w.steps)
            eu, ev, mism, ephi = compare(g, o, TOL_FP64, f"batch inst {b} {w.dims}", inst=b)
            assert mism == 0 and eu <= TOL_FP64 and ephi <= 1e-13


@pytest.mark.parametrize("mapping,lanes", [("sliced", 4), ("staged", 1), ("staged", 4)])
def test_deterministic_and_restartable(mapping, lanes):
    """Bitwise-equal reruns; a 400 + restore + 300 run equals 700 straight steps."""
    from paper_2105_04150_amd import simulation_for
    w = pi.workload("block10", steps=700)
    say(f"[run] determinism + checkpoint {mapping}")
    a = simulation_for(w, lanes=lanes, mapping=mapping)
    a.step(700)
    b = simulation_for(w, lanes=lanes, mapping=mapping)
    b.step(700)
    assert np.array_equal(a.u(), b.u()) and np.array_equal(a.broken(), b.broken())
    c = simulation_for(w, lanes=lanes, mapping=mapping)
    c.step(400)
    u, v, br = c.u(), c.v(), c.broken()
    d = simulation_for(w, lanes=lanes, mapping=mapping)
    d.set_state(u=u, v=v, broken=br)
    d.set_step(400)
    d.step(300)
    assert np.array_equal(d.u(), a.u()) and np.array_equal(d.broken(), a.broken())


def test_mapping_change_keeps_state():
    from paper_2105_04150_amd import simulation_for
    w = pi.workload("block10", steps=600)
    say("[run] relayout mid-run")
    a = simulation_for(w, lanes=1)
    a.step(600)
    b = simulation_for(w, lanes=1)
    b.step(200)
    b.set_lanes_per_node(64)
    b.step(200)
    b.set_mapping("staged")
    b.step(100)
    b.set_mapping("staged", 2)  # same layout, two wavefronts per slice
    b.step(100)
    assert rel_err(b.u(), a.u()) <= 1e-12
    assert np.array_equal(a.broken(), b.broken())


def test_autotune_restores_state(oracle_lib):
    from paper_2105_04150_amd import simulation_for
    w = pi.workload("block10", steps=300)
    say("[run] autotune mid-run")
    o = oracle_run(w, 300)
    g = simulation_for(w)
    g.step(100)
    chosen = g.autotune(trial_steps=5)
    say(f"[autotune] chose {chosen}")
    assert g.step_count == 100
    g.step(200)
    eu, ev, mism, ephi = compare(g, o, TOL_FP64, "after autotune")
    assert mism == 0 and eu <= TOL_FP64


def test_nonfinite_reported():
    """A velocity overflow is flagged and reported by the next synchronising call."""
    from paper_2105_04150_amd import PdmiError, simulation_for
    w = pi.workload("block10", dims=(5, 5, 5))
    say("[run] non-finite detection (overflowing body force)")
    sim = simulation_for(w)
    sim.step(3)
    sim.sync()
    sim.set_body_force(np.ones((w.n, 3)), 1e300)
    sim.set_integrator("euler_cromer", 1e10)
    sim.step(1)
    with pytest.raises(PdmiError) as e:
        sim.sync()
    assert e.value.code == -5
    # a state reset clears the flag
    sim.set_state(u=np.zeros((w.n, 3)), v=np.zeros((w.n, 3)))
    sim.sync()


@pytest.mark.parametrize("n", [1, 2, 65, 130])
def test_small_and_ragged_problems(oracle_lib, n):
    """Single node, a pair, and node counts just past a 64-node slice."""
    from paper_2105_04150_amd import Simulation
    rng = np.random.default_rng(n)
    x = rng.uniform(0, 4e-3, size=(n, 3))
    delta = 1.6e-3
    rp, col = oracle_lib.family(x, delta)
    u0 = rng.normal(size=(n, 3)) * 1e-7
    o = oracle_lib.OracleSim(x, rp, col, c=1e20, s0=2e-3, rho=2400.0, dt=1e-7, vol=1e-9)
    o.set_state(u=u0)
    o.run(50)
    say(f"[run] random cloud n={n} nnz={rp[-1]}")
    for mapping, lanes in (("sliced", 1), ("sliced", 64), ("staged", 1)):
        with Simulation() as g:
            g.set_mapping(mapping, lanes)
            g.build_family(x, delta)
            g.set_material(2400.0, 1e20, 2e-3, 0.0, 1e-9)
            g.set_state(u=u0)
            g.step(50)
            grp, gcol = g.family()
            assert np.array_equal(grp, rp) and np.array_equal(gcol, col)
            assert rel_err(g.u(), o.u) <= TOL_FP64 or np.abs(o.u).max() == 0
            assert np.array_equal(g.broken().astype(bool), o.broken_mask)


def test_argument_errors():
    from paper_2105_04150_amd import PdmiError, Simulation
    with Simulation() as g:
        with pytest.raises(PdmiError) as e:
            g.step(1)
        assert e.value.code == -4
        with pytest.raises(PdmiError):
            g.build_family(np.zeros((3, 3)), -1.0)
        g.build_family(np.eye(3), 1.5)
        with pytest.raises(PdmiError):
            g.set_bcs([5], 1, 1, (0, 0, 0), 0)
        with pytest.raises(PdmiError):
            g.set_integrator("euler_cromer", 0.0)
        with pytest.raises(PdmiError):
            g.set_lanes_per_node(3)


@pytest.mark.parametrize("mapping,lanes", [("sliced", 4), ("staged", 2)])
def test_all_bonds_broken_free_flight(oracle_lib, mapping, lanes):
    """Every bond broken: no bond forces, damage 1 everywhere, and each node follows the
    Euler-Cromer recurrence of a constant body force exactly (v_k = k h b, u_k = h b dt
    k (k + 1) / 2 up to rounding), as the oracle does."""
    from paper_2105_04150_amd import Simulation
    w = pi.workload("block10", dims=(7, 6, 5), steps=50)
    rp, col = oracle_lib.family(w.coords, w.horizon)
    broken = np.ones(rp[-1], dtype=np.uint8)
    bhat = np.tile([0.0, 0.0, -1.0], (w.n, 1))
    bmag = 2.0e6
    o = oracle_lib.OracleSim(w.coords, rp, col, c=w.c, s0=w.s0, rho=w.rho, dt=w.dt, vol=w.volume,
                             bhat=bhat, bmag=bmag, broken=broken)
    o.run(w.steps)
    with Simulation() as g:
        g.set_mapping(mapping, lanes)
        g.build_family(w.coords, w.horizon)
        g.set_integrator("euler_cromer", w.dt)
        g.set_material(w.rho, w.c, w.s0, 0.0, w.volume)
        g.break_bonds(broken)
        g.set_body_force(bhat, bmag)
        g.step(w.steps)
        u = g.u()
        k = w.steps
        uz = (w.dt / w.rho) * bmag * w.dt * k * (k + 1) / 2.0
        assert np.abs(u[:, 2] + uz).max() <= 1e-12 * uz and np.abs(u[:, :2]).max() == 0.0
        assert rel_err(u, o.u) <= TOL_FP64
        assert np.all(g.damage() == 1.0) and np.all(g.broken())


@pytest.mark.parametrize("mapping,lanes,precision,model", [
    ("sliced", 4, "f64", "pmb"), ("staged", 1, "f64", "pmb"), ("staged", 4, "f64", "pmb"),
    ("staged", 1, "f32", "pmb"), ("staged", 1, "f64", "state_based")])
@pytest.mark.parametrize("scheme", ["euler_cromer", "velocity_verlet"])
def test_rest_and_rigid_translation_exact(mapping, lanes, precision, model, scheme):
    """A body at rest under no load stays at rest, and a rigid translation is force-free:
    the stretch depends on the relative displacement only (Eq. simpleBond and the
    state-based dilation), so every bond is unstretched and every node keeps its
    displacement and a zero velocity, bit for bit, in both precisions and models."""
    from paper_2105_04150_amd import PD_FP32, PD_FP64, Simulation
    w = pi.workload("block10", dims=(7, 6, 5), steps=60, model=model)
    # a shift of a fraction of the spacing, exactly representable in single precision
    shift = (np.array([0.37, -0.21, 0.13]) * w.dx).astype(np.float32).astype(np.float64)
    z = np.zeros((w.n, 3))
    with Simulation(precision=PD_FP32 if precision == "f32" else PD_FP64) as g:
        g.set_mapping(mapping, lanes)
        g.build_family(w.coords, w.horizon)
        g.set_integrator(scheme, w.dt)
        g.set_material(w.rho, w.c, w.s0, 0.0, w.volume)
        if model == "state_based":
            g.set_model("state_based", *w.state_based)
        g.step(w.steps)
        assert not g.u().any() and not g.v().any()
        uc = np.tile(shift, (w.n, 1))
        g.set_state(u=uc, v=z, a=z)
        g.step(w.steps)
        assert np.array_equal(g.u(), uc) and not g.v().any()
        assert not g.broken().any()


def test_coincident_nodes_rejected():
    from paper_2105_04150_amd import PdmiError, Simulation
    x = pi.lattice((4, 4, 4), 1.0e-3)[0]
    x[7] = x[3]  # two nodes at one position
    with Simulation() as g:
        with pytest.raises(PdmiError):
            g.build_family(x, 3.015e-3)


@pytest.mark.parametrize("scheme", ["euler_cromer", "velocity_verlet"])
def test_prepare_builds_graphs_without_changing_results(scheme):
    """pd_prepare captures the step graphs up front; the run that follows is bit-identical
    to one that builds them on first use, and preparing twice or after a change is safe."""
    from paper_2105_04150_amd import simulation_for
    w = pi.workload("qs_beam", dims=(35, 10, 10), steps=300)
    w.scheme = scheme
    a = simulation_for(w, lanes=1, mapping="staged")
    a.prepare()
    a.prepare()
    a.step(150)
    a.set_no_fail(None)
    a.prepare()
    a.step(150)
    b = simulation_for(w, lanes=1, mapping="staged")
    b.step(150)
    b.set_no_fail(None)
    b.step(150)
    assert np.array_equal(a.u(), b.u()) and np.array_equal(a.v(), b.v())
    assert np.array_equal(a.broken(), b.broken())
