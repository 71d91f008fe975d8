"""The ordinary state-based linear solid on the GPU against the oracle (Sec. 8.2): two
kernels per step (breaking and dilation, then force and integration) on the staged
layout, every integrator, no-failure zones and the fifth-order ramp, batched instances,
the dilation and force readouts, and the headline cube at full size for a short prefix.
Bars as everywhere: FP64 displacement 1e-10 norm-wise with identical broken sets.
"""
import numpy as np
import pytest

import pd_inputs as pi
from oracle.oracle import OracleSim, from_workload
from parity import TOL_FP32, TOL_FP64, compare, oracle_run, rel_err, say

pytestmark = pytest.mark.gpu

THREADS = 16


@pytest.fixture(scope="module", autouse=True)
def _lib():
    from paper_2105_04150_amd import _binding as B
    B.load()


def _block(steps=800, dims=(12, 10, 9), scheme=None, **kw):
    w = pi.workload("block10", dims=dims, steps=steps, model="state_based", **kw)
    if scheme:
        w.scheme = scheme
    return w


@pytest.fixture(scope="module")
def block_oracle():
    w = _block()
    say(f"[run] oracle block10 state-based {w.dims}, {w.steps} steps")
    return w, oracle_run(w, w.steps)


@pytest.mark.parametrize("split", [1, 2, 4])
def test_block_matches_oracle(block_oracle, split):
    from paper_2105_04150_amd import simulation_for
    w, o = block_oracle
    g = simulation_for(w, lanes=split, mapping="staged")
    g.step(w.steps)
    eu, ev, mism, ephi = compare(g, o, TOL_FP64, f"state-based block staged-{split}")
    assert int(o.broken_mask.sum()) > 100
    assert mism == 0 and eu <= TOL_FP64 and ev <= TOL_FP64 and ephi <= 1e-13


@pytest.mark.parametrize("scheme", ["velocity_verlet", "forward_euler"])
def test_integrators(scheme):
    from paper_2105_04150_amd import simulation_for
    w = _block(steps=500, dims=(11, 9, 8), scheme=scheme)
    o = oracle_run(w, w.steps)
    g = simulation_for(w, mapping="staged")
    for c in (1, 63, 64, 372):  # ragged chunks around the graph length
        g.step(c)
    eu, ev, mism, ephi = compare(g, o, TOL_FP64, f"state-based {scheme}")
    assert mism == 0 and eu <= TOL_FP64


def test_poisson_ratios_change_the_answer():
    """G matters: nu = 0.1 and 0.35 give different runs, each matching its oracle."""
    from paper_2105_04150_amd import simulation_for
    us = []
    for nu in (0.1, 0.35):
        w = _block(steps=300, dims=(10, 8, 8), poisson=nu)
        o = oracle_run(w, w.steps)
        g = simulation_for(w, mapping="staged")
        g.step(w.steps)
        eu, ev, mism, _ = compare(g, o, TOL_FP64, f"state-based nu {nu}")
        assert mism == 0 and eu <= TOL_FP64
        us.append(o.u)
    assert rel_err(us[0], us[1]) > 1e-3


def test_quasistatic_bend_with_zones_and_ramp():
    """The notched three-point bend with no-failure zones, the fifth-order ramp, damping and
    velocity Verlet, on the state-based model."""
    from paper_2105_04150_amd import simulation_for
    w = pi.workload("qs_beam", dims=(35, 10, 10), steps=1600, model="state_based")
    o = oracle_run(w, w.steps)
    for split in (1, 4):
        g = simulation_for(w, lanes=split, mapping="staged")
        g.step(w.steps)
        eu, ev, mism, ephi = compare(g, o, TOL_FP64, f"state-based qs_beam staged-{split}")
        assert mism == 0 and eu <= TOL_FP64 and ephi <= 1e-12
    assert o.broken_mask.sum() > int(w.notch is not None)


def _frozen_copy(o, w):
    """An oracle copy of o's state whose next force evaluation breaks nothing (every slot
    intact now stays intact, every broken one stays broken)."""
    big = np.iinfo(np.int32).max
    frozen = np.where(o.broken_mask, 0, big).astype(np.int32)
    c = OracleSim(o.x, o.row_ptr, o.col, c=w.c, s0=w.s0, rho=w.rho, dt=w.dt, vol=w.volume,
                  frozen=frozen, state_based=w.state_based)
    return c


@pytest.mark.parametrize("split", [1, 4])
def test_fp32_build(block_oracle, split):
    """The FP32 build (single-precision bond arithmetic, f64 master displacement) against
    the FP64 oracle at the FP32 bar, break mismatches counted (at most 1%)."""
    from paper_2105_04150_amd import PD_FP32, simulation_for
    w, o = block_oracle
    g = simulation_for(w, precision=PD_FP32, lanes=split, mapping="staged")
    g.step(w.steps)
    eu, ev, mism, ephi = compare(g, o, TOL_FP32, f"state-based fp32 staged-{split}")
    assert eu <= TOL_FP32 and mism <= 0.01 * int(o.broken_mask.sum())
    th = g.dilation()
    assert np.all(np.isfinite(th))


@pytest.mark.parametrize("precision,split", [("f64", 1), ("f64", 4), ("f32", 1)])
def test_per_node_volumes(precision, split):
    """Uneven node volumes (+-30%): V_j enters the weighted volume, the dilation and the
    force; the library copies the volumes into LDS beside the records."""
    from paper_2105_04150_amd import PD_FP32, PD_FP64, simulation_for
    w = _block(steps=600, dims=(12, 10, 9))
    vols = w.volume * (0.7 + 0.6 * pi.uniform01(55, np.arange(w.n, dtype=np.uint64)))
    o = from_workload(w)
    o = OracleSim(o.x, o.row_ptr, o.col, c=w.c, s0=w.s0, rho=w.rho, dt=w.dt, vol=vols, bcs=w.bcs,
                  state_based=w.state_based)
    o.run(w.steps)
    g = simulation_for(w, precision=PD_FP32 if precision == "f32" else PD_FP64, lanes=split, mapping="staged")
    g.set_material(w.rho, w.c, w.s0, w.eta, volumes=vols)
    g.step(w.steps)
    tol = TOL_FP32 if precision == "f32" else TOL_FP64
    eu, ev, mism, ephi = compare(g, o, tol, f"state-based per-node volumes {precision} staged-{split}")
    assert int(o.broken_mask.sum()) > 100
    assert eu <= tol and mism <= (0.01 * int(o.broken_mask.sum()) if precision == "f32" else 0)


def test_dilation_and_force_readouts(block_oracle):
    from paper_2105_04150_amd import simulation_for
    w, o = block_oracle
    g = simulation_for(w, mapping="staged")
    g.step(w.steps)
    c = _frozen_copy(o, w)
    F = c.force(o.u, o.step)
    th = g.dilation()
    eth = rel_err(th, c.theta)
    eF = rel_err(g.force(), F)
    say(f"[state-based] dilation rel {eth:.2e}, force rel {eF:.2e}")
    assert eth <= 1e-9 and eF <= 1e-9
    # the readouts break nothing and leave the run unchanged
    g.step(0)
    assert np.array_equal(g.broken().astype(bool), o.broken_mask)


def test_uniform_expansion_on_the_device():
    """u = lambda x: the dilation is 3 lambda at every node."""
    from paper_2105_04150_amd import simulation_for
    w = _block(steps=10, dims=(9, 8, 7))
    g = simulation_for(w, mapping="staged", lanes=2)
    lam = 1e-3
    g.set_state(u=lam * w.coords)
    th = g.dilation()
    assert np.allclose(th, 3 * lam, rtol=1e-12, atol=0)


def test_batched_instances():
    """Two state-based instances with different moduli and sizes in one launch."""
    from paper_2105_04150_amd import Simulation, apply_workload
    wa = _block(steps=400, dims=(12, 10, 9), poisson=0.15)
    wb = _block(steps=400, dims=(9, 9, 7), poisson=0.3)
    with Simulation() as g:
        g.set_mapping("staged", 2)
        g.build_family_batch([wa.coords, wb.coords], [wa.horizon, wb.horizon])
        g.set_integrator("euler_cromer", wa.dt)
        apply_workload(g, wa, inst=0)
        apply_workload(g, wb, inst=1)
        g.step(400)
        for b, w in enumerate((wa, wb)):
            o = oracle_run(w, 400)
            eu, ev, mism, ephi = compare(g, o, TOL_FP64, f"state-based batch inst {b}", inst=b)
            assert mism == 0 and eu <= TOL_FP64


def test_model_switch_and_errors():
    from paper_2105_04150_amd import PdmiError, simulation_for
    w = _block(steps=50, dims=(8, 7, 6))
    g = simulation_for(w, mapping="staged")
    with pytest.raises(PdmiError):
        g.set_mapping("sliced", 4)
    g.set_damage_law(0, [1e-3, 2e-3], [1.0, 0.0])
    with pytest.raises(PdmiError):  # no damage laws on the state-based model
        g.step(1)
    g.clear_damage_laws()
    with pytest.raises(PdmiError):
        g.adj_forward(5, 5)
    with pytest.raises(PdmiError):
        g.set_model("state_based", -1.0, 1.0)
    with pytest.raises(ValueError):
        g.set_model("cubic")
    # back to the PMB: the bond-based kernels' results bit for bit
    g.set_model("pmb")
    g.step(50)
    wp = pi.workload("block10", dims=(8, 7, 6), steps=50)
    ref = simulation_for(wp, mapping="staged")
    ref.step(50)
    assert np.array_equal(g.u(), ref.u())
    with pytest.raises(PdmiError):
        g.dilation()
    # the sliced mapping refuses the model
    s = simulation_for(wp, lanes=4)
    with pytest.raises(PdmiError):
        s.set_model("state_based", *w.state_based)


def test_prepare_and_graph_replays():
    """Steps through captured graphs (chunks of 64) equal steps launched one by one."""
    from paper_2105_04150_amd import simulation_for
    w = _block(steps=256, dims=(10, 9, 8))
    a = simulation_for(w, mapping="staged")
    a.prepare()
    a.step(256)
    b = simulation_for(w, mapping="staged")
    for _ in range(256):
        b.step(1)
    assert np.array_equal(a.u(), b.u()) and np.array_equal(a.broken(), b.broken())


def test_velocity_verlet_graphs_and_autotune():
    """Velocity Verlet through captured graphs (two kernels per step, the drift of a
    restart) equals single launches bit for bit; the autotuner keeps to the staged
    layout and its choice matches the oracle."""
    from paper_2105_04150_amd import simulation_for
    w = pi.workload("qs_beam", dims=(30, 9, 9), steps=300, model="state_based")
    a = simulation_for(w, mapping="staged")
    a.prepare()
    a.step(150)
    a.u()  # a readout between chunks
    a.step(150)
    b = simulation_for(w, mapping="staged")
    for _ in range(300):
        b.step(1)
    assert np.array_equal(a.u(), b.u()) and np.array_equal(a.v(), b.v())
    o = oracle_run(w, w.steps)
    t = simulation_for(w, mapping="staged")
    chosen = t.autotune(trial_steps=3)
    assert chosen < 0  # a staged choice (negative: wavefronts per slice)
    t.step(w.steps)
    eu, ev, mism, ephi = compare(t, o, TOL_FP64, f"state-based after autotune ({chosen})")
    assert mism == 0 and eu <= TOL_FP64


def test_cube100_full_size():
    """The headline cube (1M nodes) on the state-based model, in the launch configurations
    the benchmark times (staged, one wavefront per slice, natural order; FP64 and FP32),
    for a short prefix the oracle can follow."""
    from paper_2105_04150_amd import PD_FP32, simulation_for
    w = pi.workload("cube100", steps=8, model="state_based")
    w.order = "natural"
    say(f"[run] oracle cube100 state-based, {w.steps} steps, {THREADS} threads")
    o = oracle_run(w, w.steps, nthreads=THREADS)
    g = simulation_for(w, mapping="staged", order="natural")
    g.step(w.steps)
    eu, ev, mism, ephi = compare(g, o, TOL_FP64, "state-based cube100 full size")
    assert np.abs(o.u).max() > 0 and mism == 0 and eu <= TOL_FP64
    g.close()
    g = simulation_for(w, precision=PD_FP32, mapping="staged", order="natural")
    g.step(w.steps)
    eu, ev, mism, ephi = compare(g, o, TOL_FP32, "state-based cube100 full size fp32")
    assert eu <= TOL_FP32 and mism == 0


@pytest.mark.parametrize("n", [1, 2, 65, 130])
def test_small_and_ragged_problems(n):
    """A single node (no bonds: m = 0, no dilation, no force), a pair, and node counts just
    past a 64-node slice, with 1 and 4 wavefronts per slice."""
    from paper_2105_04150_amd import Simulation
    rng = np.random.default_rng(100 + n)
    x = rng.uniform(0, 4e-3, size=(n, 3))
    delta = 1.6e-3
    K, G = 1.4e10, pi.shear_modulus(1.4e10, 0.2)
    from oracle.oracle import family
    rp, col = family(x, delta)
    u0 = rng.normal(size=(n, 3)) * 1e-7
    o = OracleSim(x, rp, col, c=0.0, s0=2e-3, rho=2400.0, dt=1e-7, vol=1e-9, state_based=(K, G))
    o.set_state(u=u0)
    o.run(50)
    say(f"[run] state-based random cloud n={n} nnz={rp[-1]} broken {int(o.broken_mask.sum())}")
    for split in (1, 4):
        with Simulation() as g:
            g.set_mapping("staged", split)
            g.build_family(x, delta)
            g.set_material(2400.0, 0.0, 2e-3, 0.0, 1e-9)
            g.set_model("state_based", K, G)
            g.set_state(u=u0)
            g.step(50)
            assert rel_err(g.u(), o.u) <= TOL_FP64 or np.abs(o.u - u0).max() == 0
            assert np.array_equal(g.broken().astype(bool), o.broken_mask)
            if n == 1:
                assert np.array_equal(g.u(), u0) and g.dilation()[0] == 0.0
