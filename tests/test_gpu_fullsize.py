"""Parity at the benchmark's full sizes, in the launch configurations bench.py times.

The oracle cannot follow these problems for the benchmark's step counts, so each case
runs a short prefix (every node and every slot still takes part in every step) or, for
the 64-beam batch, checks two of the instances (the smallest and the largest) against
their own oracle runs.  Bars as everywhere: FP64 displacement 1e-10 norm-wise with
identical broken sets, FP32 1e-5, adjoint gradients 1e-10.
"""
import os

import numpy as np
import pytest

import pd_inputs as pi
from parity import TOL_FP32, TOL_FP64, compare, oracle_run, rel_err, say

pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module", autouse=True)
def _lib():
    from paper_2105_04150_amd import _binding as B
    B.load()


@pytest.fixture(scope="module")
def cube_oracle():
    w = pi.workload("cube100", steps=20)
    w.order = "natural"
    say(f"[run] oracle cube100 1M nodes, {w.steps} steps, {THREADS} threads")
    return w, oracle_run(w, w.steps, nthreads=THREADS)


@pytest.mark.parametrize("split", [1, 4])
def test_cube100_full_size(cube_oracle, split):
    """The headline workload (1M nodes, 117.8M slots) with the staged mapping."""
    from paper_2105_04150_amd import simulation_for
    w, o = cube_oracle
    g = simulation_for(w, lanes=split, mapping="staged", order="natural")
    g.step(w.steps)
    eu, ev, mism, ephi = compare(g, o, TOL_FP64, f"cube100 full size staged-{split}")
    assert np.abs(o.u).max() > 0
    assert mism == 0 and eu <= TOL_FP64 and ephi <= 1e-13


def test_cube100_full_size_fp32(cube_oracle):
    from paper_2105_04150_amd import PD_FP32, simulation_for
    w, o = cube_oracle
    g = simulation_for(w, precision=PD_FP32, mapping="staged", order="natural")
    g.step(w.steps)
    eu, ev, mism, ephi = compare(g, o, TOL_FP32, "cube100 full size fp32")
    assert eu <= TOL_FP32 and mism <= 0.01 * max(int(o.broken_mask.sum()), 1)


@pytest.fixture(scope="module")
def beam_adjoint_oracle():
    w = pi.workload("adjoint_beam", steps=100)
    o = oracle_run(w, w.steps, nthreads=THREADS, record_breaks=True)
    sensors, target = pi.adjoint_sensors(w)
    dldu = 2.0 * (o.u[sensors] - target)
    z = np.zeros((w.n, 3))
    say(f"[run] oracle adjoint, full-size beam, {w.steps} steps")
    gk_o, gA_o = o.adjoint_ec(o.break_step[: o.nnz].copy(), w.steps, z, z, 0, sensors, dldu)
    return w, sensors, dldu, gk_o, gA_o


@pytest.mark.parametrize("mapping,lanes", [("staged", 4), ("sliced", 16)])
def test_adjoint_beam_full_size(beam_adjoint_oracle, mapping, lanes):
    """The adjoint workload at full size (100x25x20, 200 sensors), a 100-step prefix with
    a ragged checkpoint interval."""
    from paper_2105_04150_amd import simulation_for
    w, sensors, dldu, gk_o, gA_o = beam_adjoint_oracle
    g = simulation_for(w, lanes=lanes, mapping=mapping)
    g.adj_forward(w.steps, 30)
    gk, gA = g.adj_backward(sensors, dldu)
    ek, eA = rel_err(gk, gk_o), abs(gA - gA_o) / abs(gA_o)
    say(f"[adjoint] full-size beam {mapping}-{lanes}: grad_k rel {ek:.3e} grad_A rel {eA:.3e}")
    assert np.abs(gk_o).max() > 0
    assert ek <= TOL_FP64 and eA <= TOL_FP64


def test_batch64_full_size_sampled():
    """The 64 uneven beams (5.15M nodes, 564M slots) with node stiffness fields, advanced
    together; the smallest and the largest instance against their own oracle runs."""
    from paper_2105_04150_amd import Simulation, apply_workload
    steps = 20
    ws = pi.batch_instances(count=64, steps=steps)
    with Simulation() as g:
        g.set_mapping("staged", 1)
        g.build_family_batch([w.coords for w in ws], [w.horizon for w in ws])
        g.set_integrator("euler_cromer", ws[0].dt)
        for b, w in enumerate(ws):
            apply_workload(g, w, inst=b, stiffness="node")
        say(f"[run] batch of 64 built: {g.info()['n_slots']} slots")
        g.step(steps)
        for b in (0, 63):
            o = oracle_run(ws[b], steps, nthreads=THREADS)
            eu, ev, mism, ephi = compare(g, o, TOL_FP64, f"batch64 inst {b} {ws[b].dims}", inst=b)
            assert np.abs(o.u).max() > 0
            assert mism == 0 and eu <= TOL_FP64


@pytest.mark.parametrize("law,lanes", [("brittle", 2), ("trilinear", 4)])
def test_qs_beam_full_size(law, lanes):
    """The quasi-static bend at the benchmark's size (175 x 50 x 50, 437,500 nodes, 50.6M
    slots) with zones, damping and velocity Verlet, in the launch configurations of the
    quasistatic and damage_law lines; a 60-step prefix with the ramp compressed into it so
    that the load moves the beam by a resolvable amount."""
    from paper_2105_04150_amd import simulation_for
    w = pi.workload("qs_beam", steps=60, law=law)
    say(f"[run] oracle qs_beam {law} full size, {w.steps} steps, {THREADS} threads")
    o = oracle_run(w, w.steps, nthreads=THREADS)
    g = simulation_for(w, lanes=lanes, mapping="staged", order="natural")
    g.step(w.steps)
    eu, ev, mism, ephi = compare(g, o, TOL_FP64, f"qs_beam {law} full size staged-{lanes}")
    assert np.abs(o.u).max() > 0
    assert mism == 0 and eu <= TOL_FP64 and ephi <= 1e-12
    if law != "brittle":
        assert np.array_equal(g.max_stretch() > 0, o.smax[: o.nnz] > 0)


def test_cube100_corrections_full_size():
    """The corrections line's problem (the 1M-node cube, conical profile at 5c, surface
    correction, formed per slot in the kernel) over a short prefix."""
    from paper_2105_04150_amd import simulation_for
    w = pi.workload("cube100", steps=8)
    w.order = "natural"
    w.c = 5.0 * w.c
    w.corrections = dict(micro="conical", surface=True, delta=w.horizon, dx=w.dx)
    say(f"[run] oracle cube100 with corrections, {w.steps} steps, {THREADS} threads")
    o = oracle_run(w, w.steps, nthreads=THREADS)
    g = simulation_for(w, mapping="staged", order="natural")
    g.step(w.steps)
    eu, ev, mism, ephi = compare(g, o, TOL_FP64, "cube100 corrections full size")
    assert np.abs(o.u).max() > 0 and mism == 0 and eu <= TOL_FP64
