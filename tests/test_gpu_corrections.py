"""Stiffness corrections on the GPU against the oracle (Secs. 2.2, 2.3 and 2.5): conical
micromodulus, partial volumes, volume-method surface correction, alone and together, on
top of uniform, per-slot and per-node stiffness.  The oracle forms its factors itself;
the library folds them into the per-slot stiffness on the host.  Bars as everywhere:
FP64 displacement 1e-10 with identical broken sets, FP32 1e-5 with counted mismatches.
"""
import copy

import numpy as np
import pytest

import pd_inputs as pi
from parity import TOL_FP32, TOL_FP64, compare, oracle_run, rel_err, say

pytestmark = pytest.mark.gpu

M = 3.015


@pytest.fixture(scope="module", autouse=True)
def _lib():
    from paper_2105_04150_amd import _binding as B
    B.load()


def _block(corr, partial=False, steps=800):
    w = pi.workload("block10", dims=(12, 10, 9), steps=steps)
    w = copy.copy(w)
    if partial:  # family out to delta + dx/2 so the cut cells take part
        w.horizon = (M + 0.5) * pi.DX
    w.corrections = dict(corr, delta=M * pi.DX, dx=pi.DX)
    return w


CASES = {
    "conical": dict(micro="conical"),
    "surface": dict(surface=True),
    "partial": dict(partial_volumes=True),
    "all": dict(micro="conical", partial_volumes=True, surface=True),
}


@pytest.mark.parametrize("mapping,lanes", [("sliced", 4), ("staged", 1)])
@pytest.mark.parametrize("case", list(CASES))
def test_corrections_match_oracle(case, mapping, lanes):
    from paper_2105_04150_amd import simulation_for
    corr = CASES[case]
    w = _block(corr, partial=corr.get("partial_volumes", False))
    if corr.get("micro") == "conical":
        w.c = 5.0 * w.c  # peak value for the same bulk stiffness
    o = oracle_run(w, w.steps)
    g = simulation_for(w, lanes=lanes, mapping=mapping)
    g.step(w.steps)
    eu, ev, mism, ephi = compare(g, o, TOL_FP64, f"corrections {case} {mapping}-{lanes}")
    assert int(o.broken_mask.sum()) > 100
    assert mism == 0 and eu <= TOL_FP64 and ephi <= 1e-13


def test_corrections_change_the_answer():
    """Each correction changes the run (against the uncorrected oracle)."""
    base = oracle_run(pi.workload("block10", dims=(12, 10, 9), steps=400), 400)
    for case, corr in CASES.items():
        w = _block(corr, partial=corr.get("partial_volumes", False), steps=400)
        o = oracle_run(w, 400)
        diff = np.abs(o.u - base.u).max() / np.abs(base.u).max()
        say(f"[corrections] {case}: changes u by {diff:.2e}")
        assert diff > 1e-4


@pytest.mark.parametrize("lanes", [1, 4])
def test_corrections_with_zones_and_ramp(lanes):
    """The notched bend with no-failure zones, the ramp and damping, plus the conical
    profile and the surface correction: the zone-aware kernels with per-slot corrections."""
    from paper_2105_04150_amd import simulation_for
    w = pi.workload("qs_beam", dims=(35, 10, 10), steps=1200)
    w.c = 5.0 * w.c
    w.corrections = dict(micro="conical", surface=True, delta=w.horizon, dx=pi.DX)
    o = oracle_run(w, w.steps)
    g = simulation_for(w, lanes=lanes, mapping="staged")
    g.step(w.steps)
    eu, ev, mism, ephi = compare(g, o, TOL_FP64, f"corrections with zones staged-{lanes}")
    assert int(o.broken_mask.sum()) > 0
    assert mism == 0 and eu <= TOL_FP64 and ephi <= 1e-12


def test_switch_between_kernel_and_stream_forms():
    """Per-node volumes turn the per-slot corrections into the folded stiffness stream
    and back; every stage matches the oracle of the same problem."""
    from paper_2105_04150_amd import simulation_for
    w = _block(CASES["all"], partial=True, steps=300)
    w.c = 5.0 * w.c
    o = oracle_run(w, 300)
    g = simulation_for(w, lanes=1, mapping="staged")
    g.step(100)
    # same volumes given per node: the library folds the corrections into the stream
    g.set_material(w.rho, w.c, w.s0, w.eta, volumes=np.full(w.n, w.volume))
    g.step(100)
    g.set_material(w.rho, w.c, w.s0, w.eta, w.volume)
    g.step(100)
    eu, ev, mism, ephi = compare(g, o, TOL_FP64, "corrections kernel -> stream -> kernel")
    assert mism == 0 and eu <= TOL_FP64


def test_corrections_fp32():
    from paper_2105_04150_amd import PD_FP32, simulation_for
    w = _block(CASES["all"], partial=True)
    w.c = 5.0 * w.c
    o = oracle_run(w, w.steps)
    g = simulation_for(w, precision=PD_FP32, mapping="staged")
    g.step(w.steps)
    eu, ev, mism, ephi = compare(g, o, TOL_FP32, "corrections all fp32")
    assert eu <= TOL_FP32 and mism <= 0.01 * int(o.broken_mask.sum())


@pytest.mark.parametrize("stiffness", ["slot", "node"])
def test_corrections_on_stiffness_fields(stiffness):
    """Surface correction and conical profile on top of a log-normal stiffness field given
    per slot or per node (a node field is expanded into slots once corrections apply)."""
    from paper_2105_04150_amd import simulation_for
    w = pi.workload("adjoint_beam", dims=(30, 10, 8), steps=600)
    w.corrections = dict(micro="conical", surface=True, delta=M * pi.DX, dx=pi.DX)
    o = oracle_run(w, w.steps)
    g = simulation_for(w, lanes=4, stiffness=stiffness)
    g.step(w.steps)
    eu, ev, mism, ephi = compare(g, o, TOL_FP64, f"corrections on a {stiffness} field")
    assert mism == 0 and eu <= TOL_FP64


def test_batched_and_removal():
    """Two instances, corrections on one: both match their oracles; removing the
    corrections gives the uncorrected kernels' results bit for bit."""
    from paper_2105_04150_amd import Simulation, apply_workload, simulation_for
    wa = _block(CASES["all"], partial=True, steps=500)
    wb = pi.workload("block10", dims=(11, 9, 8), steps=500)
    with Simulation() as g:
        g.set_mapping("staged", 1)
        g.build_family_batch([wa.coords, wb.coords], [wa.horizon, wb.horizon])
        g.set_integrator("euler_cromer", wa.dt)
        apply_workload(g, wa, inst=0)
        apply_workload(g, wb, inst=1)
        g.step(500)
        for b, w in enumerate((wa, wb)):
            o = oracle_run(w, 500)
            eu, ev, mism, ephi = compare(g, o, TOL_FP64, f"batched corrections inst {b}", inst=b)
            assert mism == 0 and eu <= TOL_FP64
    w = pi.workload("block10", dims=(12, 10, 9), steps=300)
    g = simulation_for(w, lanes=1, mapping="staged")
    g.set_corrections(dict(micro="conical", surface=True, delta=M * pi.DX))
    g.set_corrections(None)
    g.step(300)
    ref = simulation_for(w, lanes=1, mapping="staged")
    ref.step(300)
    assert np.array_equal(g.u(), ref.u())


def test_correction_arguments():
    from paper_2105_04150_amd import PdmiError, simulation_for
    w = pi.workload("block10", dims=(8, 7, 6), steps=10)
    w.scheme = "euler_cromer"
    g = simulation_for(w, lanes=4)
    with pytest.raises(ValueError):
        g.set_corrections(dict(micro="cubic"))
    for bad in (dict(micro="conical"), dict(micro="conical", delta=-1.0), dict(partial_volumes=True, delta=1e-3),
                dict(partial_volumes=True, delta=1e-3, dx=0.0)):
        with pytest.raises(PdmiError):
            g.set_corrections(bad)
    g.set_corrections(dict(surface=True))
    with pytest.raises(PdmiError):
        g.adj_forward(5, 5)
    g.set_corrections(None)
    g.step(10)


@pytest.mark.parametrize("n", [1, 2, 65, 130])
def test_small_and_ragged_problems(oracle_lib, n):
    """A single node (no bonds, family volume 0), a pair, and node counts just past a
    64-node slice, with every correction, per slot (staged) and folded (sliced)."""
    from paper_2105_04150_amd import Simulation
    rng = np.random.default_rng(200 + n)
    x = rng.uniform(0, 4e-3, size=(n, 3))
    delta, dx = 1.6e-3, 1e-3
    corr = dict(micro="conical", partial_volumes=True, surface=True, delta=delta - 0.5 * dx, dx=dx)
    rp, col = oracle_lib.family(x, delta)
    u0 = rng.normal(size=(n, 3)) * 1e-7
    o = oracle_lib.OracleSim(x, rp, col, c=5e20, s0=2e-3, rho=2400.0, dt=1e-7, vol=1e-9, corrections=corr)
    o.set_state(u=u0)
    o.run(50)
    for mapping, lanes in (("staged", 1), ("staged", 4), ("sliced", 4)):
        with Simulation() as g:
            g.set_mapping(mapping, lanes)
            g.build_family(x, delta)
            g.set_material(2400.0, 5e20, 2e-3, 0.0, 1e-9)
            g.set_corrections(corr)
            g.set_state(u=u0)
            g.step(50)
            assert np.all(np.isfinite(g.u()))
            if n == 1:
                assert np.array_equal(g.u(), u0)
            else:
                assert rel_err(g.u(), o.u) <= TOL_FP64
            assert np.array_equal(g.broken().astype(bool), o.broken_mask)
