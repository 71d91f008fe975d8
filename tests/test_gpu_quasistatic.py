"""Quasi-static loading tools on the GPU against the oracle: the fifth-order displacement
ramp, no-failure zones, dynamic-relaxation damping (Secs. 2.3, 6, 7) and the force readout
(bond force density and the resultant of a node set, the measured load of Sec. 6).

Bars as everywhere: FP64 displacement 1e-10 norm-wise with identical broken sets, FP32
1e-5 with counted break mismatches.  Force readouts are compared at the same state
(the oracle's displacement and broken set loaded into the library), FP64 within 1e-12 of
the largest force component.
"""
import numpy as np
import pytest

import pd_inputs as pi
from oracle.oracle import from_workload
from parity import TOL_FP32, TOL_FP64, compare, oracle_run, rel_err, say

pytestmark = pytest.mark.gpu

SMALL = dict(dims=(35, 10, 10), steps=2000)
MAPPINGS = [("sliced", 4), ("sliced", 1), ("staged", 1), ("staged", 4)]


@pytest.fixture(scope="module", autouse=True)
def _lib():
    from paper_2105_04150_amd import _binding as B
    B.load()


def _zone_mask(w, row_ptr, col):
    flag = np.zeros(w.n, dtype=bool)
    flag[w.nofail] = True
    rows = np.repeat(np.arange(w.n), np.diff(row_ptr))
    return flag[rows] | flag[col]


@pytest.fixture(scope="module")
def qs_oracle():
    w = pi.workload("qs_beam", **SMALL)
    say(f"[run] oracle qs_beam {w.dims}, {w.steps} steps")
    return w, oracle_run(w, w.steps)


@pytest.mark.parametrize("mapping,lanes", MAPPINGS)
def test_qs_beam_matches_oracle(qs_oracle, mapping, lanes):
    """Notched three-point bend, velocity Verlet with damping, ramped load, no-failure zones."""
    from paper_2105_04150_amd import simulation_for
    w, o = qs_oracle
    g = simulation_for(w, lanes=lanes, mapping=mapping)
    g.step(w.steps)
    eu, ev, mism, ephi = compare(g, o, TOL_FP64, f"qs_beam {mapping}-{lanes}")
    zone = _zone_mask(w, o.row_ptr, o.col)
    nb = int(o.broken_mask.sum())
    assert nb > 1000 and not (o.broken_mask & zone).any()
    assert mism == 0 and eu <= TOL_FP64 and ev <= TOL_FP64 and ephi <= 1e-13


def test_qs_beam_fp32(qs_oracle):
    from paper_2105_04150_amd import PD_FP32, simulation_for
    w, o = qs_oracle
    g = simulation_for(w, precision=PD_FP32, mapping="staged")
    g.step(w.steps)
    eu, ev, mism, ephi = compare(g, o, TOL_FP32, "qs_beam fp32")
    zone = _zone_mask(w, o.row_ptr, o.col)
    assert not (g.broken().astype(bool) & zone).any()
    assert eu <= TOL_FP32 and mism <= 0.01 * int(o.broken_mask.sum())


@pytest.mark.parametrize("mapping,lanes", [("sliced", 4), ("staged", 1)])
def test_qs_beam_euler_cromer_without_zones(mapping, lanes):
    """The same loading with Euler-Cromer and no zones: bonds at the supports break too."""
    from paper_2105_04150_amd import simulation_for
    w = pi.workload("qs_beam", **SMALL)
    w.scheme = "euler_cromer"
    zones = w.nofail
    w.nofail = None
    o = oracle_run(w, w.steps)
    w.nofail = zones
    assert (o.broken_mask & _zone_mask(w, o.row_ptr, o.col)).any()
    w.nofail = None
    g = simulation_for(w, lanes=lanes, mapping=mapping)
    g.step(w.steps)
    eu, ev, mism, ephi = compare(g, o, TOL_FP64, f"qs_beam EC no zones {mapping}-{lanes}")
    assert mism == 0 and eu <= TOL_FP64


@pytest.mark.parametrize("kind", [pi.BC_DISP, pi.BC_VEL])
@pytest.mark.parametrize("scheme", ["euler_cromer", "velocity_verlet"])
def test_ramp_schedule(kind, scheme):
    """A face driven by the ramp (both kinds), past the end of the ramp, against the oracle
    every 25 steps; the driven face reaches its end value.  (Amplitudes keep u/dx above
    ~1e-6 from the first check on: below that the oracle's printed-form stretch,
    |y| - |xi|, loses more digits than the 1e-10 bar allows.)"""
    from paper_2105_04150_amd import simulation_for
    w = pi.workload("block10", dims=(8, 7, 6), steps=300)
    w.scheme = scheme
    amp = 3.0e-6 if kind == pi.BC_DISP else 0.5
    top = pi.face_nodes(w.ijk, 2, w.dims[2] - 1)
    w.bcs = [w.bcs[0], pi.BCSpec(top, 0b101, kind, (0.5 * amp, 0.0, amp), pi.SCHED_RAMP5)]
    w.ramp_T = 200 * w.dt
    o = from_workload(w)
    g = simulation_for(w, lanes=4)
    for k in range(12):
        o.run(25)
        g.step(25)
        eu = rel_err(g.u(), o.u)
        assert eu <= TOL_FP64, (k, eu)
    if kind == pi.BC_DISP:
        assert np.allclose(g.u()[top, 2], amp, rtol=0, atol=1e-15 * amp)
        assert np.abs(g.v()[top][:, [0, 2]]).max() == 0.0 or scheme == "velocity_verlet"
    say(f"[ramp] kind {kind} {scheme}: u rel {eu:.2e}")


def _same_state(w, o, mapping, lanes, precision=None):
    """A library simulation of w holding the oracle's displacement and broken set."""
    from paper_2105_04150_amd import PD_FP64, simulation_for
    g = simulation_for(w, lanes=lanes, mapping=mapping, precision=PD_FP64 if precision is None else precision)
    g.set_state(u=o.u, broken=o.broken_mask.astype(np.uint8))
    return g


def _oracle_force(w, u, broken):
    fr = np.where(broken, np.iinfo(np.int32).min, np.iinfo(np.int32).max).astype(np.int32)
    return from_workload(w, frozen=fr).force(u=u, k=0)


@pytest.mark.parametrize("mapping,lanes", MAPPINGS)
def test_force_readout(qs_oracle, mapping, lanes):
    """Bond force density at a cracked state; breaking does not happen in the readout."""
    w, o = qs_oracle
    g = _same_state(w, o, mapping, lanes)
    F_ref = _oracle_force(w, o.u, o.broken_mask)
    F = g.force()
    e = float(np.abs(F - F_ref).max() / np.abs(F_ref).max())
    say(f"[force] {mapping}-{lanes}: rel {e:.2e}")
    assert e <= 1e-12
    assert np.array_equal(g.broken().astype(bool), o.broken_mask)  # nothing broke
    assert np.array_equal(g.u(), o.u)                             # state untouched


def test_force_readout_fp32(qs_oracle):
    from paper_2105_04150_amd import PD_FP32
    w, o = qs_oracle
    g = _same_state(w, o, "staged", 1, precision=PD_FP32)
    F_ref = _oracle_force(w, o.u, o.broken_mask)
    e = float(np.abs(g.force() - F_ref).max() / np.abs(F_ref).max())
    say(f"[force] fp32: rel {e:.2e}")
    assert e <= TOL_FP32


@pytest.mark.parametrize("mapping,lanes", [("sliced", 16), ("staged", 2)])
def test_force_readout_after_verlet_steps(mapping, lanes):
    """After velocity-Verlet steps the library keeps the next level in flight; the readout
    must use the current one (the level the displacement readout returns)."""
    from paper_2105_04150_amd import simulation_for
    w = pi.workload("qs_beam", dims=(35, 10, 10), steps=700)
    g = simulation_for(w, lanes=lanes, mapping=mapping)
    g.step(w.steps)
    u, br = g.u(), g.broken().astype(bool)
    F_ref = _oracle_force(w, u, br)
    e = float(np.abs(g.force() - F_ref).max() / np.abs(F_ref).max())
    assert e <= 1e-12
    g.step(1)  # stepping goes on from the same state
    o = oracle_run(w, w.steps + 1)
    assert rel_err(g.u(), o.u) <= TOL_FP64


def test_resultant(qs_oracle):
    """Load on the driven set (sum of V_i F_i) and the balance of all internal forces."""
    from paper_2105_04150_amd import simulation_for
    w, o = qs_oracle
    g = _same_state(w, o, "staged", 1)
    F_ref = _oracle_force(w, o.u, o.broken_mask)
    _, _, load = pi.qs_beam_sets(w.ijk, w.dims)
    R = g.resultant(load)
    R_ref = (w.volume * F_ref[load]).sum(0)
    scale = (w.volume * np.abs(F_ref[load])).sum()
    say(f"[resultant] load set: {R} (oracle {R_ref})")
    assert np.abs(R - R_ref).max() <= 1e-12 * scale
    assert R[2] > 0.0  # the bonds pull the pushed-down load nodes back up
    allR = g.resultant(np.arange(w.n))
    assert np.abs(allR).max() <= 1e-12 * (w.volume * np.abs(F_ref)).sum()
    g2 = simulation_for(w, lanes=4)
    g2.set_state(u=o.u, broken=o.broken_mask.astype(np.uint8))
    assert np.abs(g2.resultant(load) - R_ref).max() <= 1e-12 * scale


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_mean_displacement(qs_oracle, precision):
    """Mid-span deflection: the mean u of the top nodes at mid-span (and of the load set)
    after the run, against the oracle's displacement."""
    from paper_2105_04150_amd import PD_FP32, PD_FP64, simulation_for
    w, o = qs_oracle
    g = simulation_for(w, mapping="staged", precision=PD_FP64 if precision == "f64" else PD_FP32)
    g.step(w.steps)
    mid = np.nonzero((w.ijk[:, 0] == w.dims[0] // 2) & (w.ijk[:, 2] == w.dims[2] - 1))[0]
    _, _, load = pi.qs_beam_sets(w.ijk, w.dims)
    tol = TOL_FP64 if precision == "f64" else TOL_FP32
    scale = np.abs(o.u).max()
    for nodes in (mid, load, np.arange(w.n)):
        got = g.mean_displacement(nodes)
        want = o.u[nodes].mean(0)
        assert np.abs(got - want).max() <= tol * scale, (len(nodes), got, want)
    # the ramp holds the load set exactly at its end value
    assert g.mean_displacement(load)[2] == pytest.approx(-1.15e-7 * w.dims[0], rel=1e-14)


def test_zone_changes_keep_state_and_break_steps():
    """Removing a zone mid-run keeps the broken set and the recorded break steps, and the
    run goes on as the oracle's with the same history (zone for 1200 steps, none after)."""
    from paper_2105_04150_amd import simulation_for
    w = pi.workload("qs_beam", dims=(35, 10, 10), steps=1500)
    g = simulation_for(w, lanes=1, mapping="staged")
    g.step(1200)
    bs, br, u = g.break_steps(), g.broken(), g.u()
    assert (bs < np.iinfo(np.int32).max).sum() > 100
    g.set_no_fail(None)
    assert np.array_equal(g.break_steps(), bs) and np.array_equal(g.broken(), br)
    assert np.array_equal(g.u(), u)
    g.step(300)
    o = from_workload(w)
    o.run(1200)
    o.P.nofail = None  # the oracle's zone removed at the same step
    o.run(300)
    zone = _zone_mask(w, o.row_ptr, o.col)
    assert (o.broken_mask & zone).any()  # bonds of the former zone break afterwards
    eu, ev, mism, ephi = compare(g, o, TOL_FP64, "zone removed at step 1200")
    assert mism == 0 and eu <= TOL_FP64


def test_arguments():
    from paper_2105_04150_amd import PdmiError, simulation_for
    w = pi.workload("qs_beam", dims=(20, 6, 6), steps=10)
    g = simulation_for(w, lanes=4)
    for bad in (0.0, -1.0, np.nan, np.inf):
        with pytest.raises(PdmiError):
            g.set_bc_ramp(bad)
    with pytest.raises(PdmiError):
        g.set_no_fail([w.n])
    with pytest.raises(PdmiError):
        g.set_no_fail([-1])
    with pytest.raises(PdmiError):
        g.set_bcs([0], 0b1, pi.BC_DISP, (0.0, 0.0, 0.0), 3)
    with pytest.raises(PdmiError):
        g.resultant([])
    with pytest.raises(PdmiError):
        g.resultant([w.n])
    with pytest.raises(PdmiError):
        g.mean_displacement([])
    with pytest.raises(PdmiError):
        g.mean_displacement([-3])
    g.step(10)


def test_batched_instances_with_and_without_zones():
    """Two instances in one context, a zone on one of them only: each matches its oracle."""
    from paper_2105_04150_amd import Simulation, apply_workload
    wa = pi.workload("qs_beam", dims=(35, 10, 10), steps=1500)
    wb = pi.workload("qs_beam", dims=(30, 9, 9), steps=1500)
    wb.nofail = None
    for mapping, lanes in (("sliced", 4), ("staged", 1)):
        with Simulation() as g:
            g.set_mapping(mapping, lanes)
            g.build_family_batch([wa.coords, wb.coords], [wa.horizon, wb.horizon])
            g.set_integrator(wa.scheme, wa.dt)
            apply_workload(g, wa, inst=0)
            apply_workload(g, wb, inst=1)
            g.step(1500)
            for b, w in enumerate((wa, wb)):
                o = oracle_run(w, w.steps)
                eu, ev, mism, ephi = compare(g, o, TOL_FP64, f"zones batch {mapping} inst {b}", inst=b)
                assert mism == 0 and eu <= TOL_FP64


@pytest.mark.parametrize("mapping,lanes", [("sliced", 4), ("staged", 4)])
def test_adjoint_with_zone(mapping, lanes):
    """The adjoint's forward recording and recompute run the zone-aware kernels: gradients
    match the oracle adjoint of a run with a no-failure zone next to the clamp (without
    the zone, most breaks of this run fall inside it)."""
    from paper_2105_04150_amd import simulation_for
    w = pi.workload("adjoint_beam", dims=(30, 10, 8), steps=1200)
    w.nofail = np.concatenate([pi.face_nodes(w.ijk, 0, 1), pi.face_nodes(w.ijk, 0, 2)])
    o = oracle_run(w, w.steps, record_breaks=True)
    frozen = o.break_step[: o.nnz].copy()
    assert (frozen < np.iinfo(np.int32).max).sum() > 300
    assert not (o.broken_mask & _zone_mask(w, o.row_ptr, o.col)).any()
    sensors, target = pi.adjoint_sensors(w, m=40)
    dldu = 2.0 * (o.u[sensors] - target)
    z = np.zeros((w.n, 3))
    gk_o, gA_o = o.adjoint_ec(frozen, w.steps, z, z, 0, sensors, dldu)
    g = simulation_for(w, lanes=lanes, mapping=mapping)
    g.adj_forward(w.steps, 100)
    assert np.array_equal(g.break_steps(), frozen)
    gk, gA = g.adj_backward(sensors, dldu)
    ek, eA = rel_err(gk, gk_o), abs(gA - gA_o) / abs(gA_o)
    say(f"[adjoint] zone {mapping}-{lanes}: grad_k rel {ek:.3e} grad_A rel {eA:.3e}")
    assert ek <= TOL_FP64 and eA <= TOL_FP64
