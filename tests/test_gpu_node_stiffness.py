"""Per-node stiffness (bond value sqrt(k_i k_j)) against the oracle's per-slot field.

The workloads' log-normal fields give per-slot c exp((g_i + g_j)/2), which the oracle
receives slot by slot; the library receives the node values c exp(g_i) and forms
sqrt(k_i) sqrt(k_j) on the device.  Bars as for every FP64 case: displacement 1e-10,
identical broken sets; FP32 1e-5 with counted break mismatches.
"""
import numpy as np
import pytest

import pd_inputs as pi
from parity import TOL_FP32, TOL_FP64, compare, oracle_run, rel_err, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    from paper_2105_04150_amd import _binding as B
    B.load()


@pytest.mark.parametrize("mapping,lanes", [("sliced", 4), ("sliced", 1), ("staged", 1)])
def test_node_field_matches_oracle(mapping, lanes):
    from paper_2105_04150_amd import simulation_for
    w = pi.workload("adjoint_beam", dims=(40, 12, 10), steps=1500)
    o = oracle_run(w, w.steps)
    say(f"[run] node stiffness {mapping}-{lanes}")
    g = simulation_for(w, lanes=lanes, mapping=mapping, stiffness="node")
    g.step(w.steps)
    eu, ev, mism, ephi = compare(g, o, TOL_FP64, f"node stiffness {mapping}-{lanes}")
    assert int(o.broken_mask.sum()) > 1000
    assert mism == 0 and eu <= TOL_FP64 and ephi <= 1e-13


def test_node_field_fp32():
    from paper_2105_04150_amd import PD_FP32, simulation_for
    w = pi.workload("adjoint_beam", dims=(40, 12, 10), steps=1500)
    o = oracle_run(w, w.steps)
    g = simulation_for(w, precision=PD_FP32, mapping="staged", stiffness="node")
    g.step(w.steps)
    eu, ev, mism, ephi = compare(g, o, TOL_FP32, "node stiffness fp32")
    nb = max(int(o.broken_mask.sum()), 1)
    say(f"[fp32] node stiffness: broken-bond mismatches {mism} of {nb}")
    assert eu <= TOL_FP32 and mism <= 0.01 * nb


@pytest.mark.parametrize("mapping", ["sliced", "staged"])
def test_batched_node_fields(mapping):
    """Three uneven beams with node fields advanced together equal independent oracles."""
    from paper_2105_04150_amd import Simulation, apply_workload
    ws = pi.batch_instances(count=3, scale_lo=0.4, scale_hi=0.7, steps=300)
    with Simulation() as g:
        g.set_mapping(mapping, 4 if mapping == "sliced" else 0)
        g.build_family_batch([w.coords for w in ws], [w.horizon for w in ws])
        g.set_integrator("euler_cromer", ws[0].dt)
        for b, w in enumerate(ws):
            apply_workload(g, w, inst=b, stiffness="node")
        assert g.info()["model_bytes_per_step"] > 0
        g.step(ws[0].steps)
        for b, w in enumerate(ws):
            o = oracle_run(w, w.steps)
            eu, ev, mism, ephi = compare(g, o, TOL_FP64, f"batch node field inst {b}", inst=b)
            assert mism == 0 and eu <= TOL_FP64


def test_mixed_slot_and_node_instances():
    """One instance with a per-slot field, one with a node field: the node field is
    expanded to slots, both match their oracles."""
    from paper_2105_04150_amd import Simulation, apply_workload
    ws = pi.batch_instances(count=2, scale_lo=0.4, scale_hi=0.5, steps=300)
    with Simulation() as g:
        g.set_mapping("staged")
        g.build_family_batch([w.coords for w in ws], [w.horizon for w in ws])
        g.set_integrator("euler_cromer", ws[0].dt)
        apply_workload(g, ws[0], inst=0, stiffness="slot")
        apply_workload(g, ws[1], inst=1, stiffness="node")
        g.step(300)
        for b, w in enumerate(ws):
            o = oracle_run(w, w.steps)
            eu, ev, mism, ephi = compare(g, o, TOL_FP64, f"mixed inst {b}", inst=b)
            assert mism == 0 and eu <= TOL_FP64
        # removing the per-slot field switches the context to node factors; the state is kept
        u_before = g.u(1)
        g.set_bond_stiffness(None, inst=0)
        assert np.array_equal(g.u(1), u_before)


@pytest.mark.parametrize("mapping,lanes", [("sliced", 4), ("staged", 1), ("staged", 4)])
def test_adjoint_with_node_field(oracle_lib, mapping, lanes):
    from paper_2105_04150_amd import simulation_for
    w = pi.workload("adjoint_beam", dims=(30, 10, 8), steps=400)
    o = oracle_run(w, w.steps, record_breaks=True)
    frozen = o.break_step[: o.nnz].copy()
    sensors, target = pi.adjoint_sensors(w, m=40)
    dldu = 2.0 * (o.u[sensors] - target)
    z = np.zeros((w.n, 3))
    gk_o, gA_o = o.adjoint_ec(frozen, w.steps, z, z, 0, sensors, dldu)
    g = simulation_for(w, lanes=lanes, mapping=mapping, stiffness="node")
    g.adj_forward(w.steps, 50)
    gk, gA = g.adj_backward(sensors, dldu)
    ek, eA = rel_err(gk, gk_o), abs(gA - gA_o) / abs(gA_o)
    say(f"[adjoint] node field {mapping}-{lanes}: grad_k rel {ek:.3e} grad_A rel {eA:.3e}")
    assert ek <= TOL_FP64 and eA <= TOL_FP64


def test_node_stiffness_arguments_and_removal():
    from paper_2105_04150_amd import PdmiError, simulation_for
    w = pi.workload("block10", dims=(8, 7, 6), steps=100)
    g = simulation_for(w, lanes=4)
    n = w.n
    with pytest.raises(PdmiError):
        g.set_node_stiffness(np.full(n, -1.0))
    bad = np.full(n, w.c)
    bad[3] = np.nan
    with pytest.raises(PdmiError):
        g.set_node_stiffness(bad)
    g.set_node_stiffness(np.full(n, 2.0 * w.c))
    g.set_node_stiffness(None)  # back to the uniform micromodulus
    g.step(w.steps)
    ref = simulation_for(w, lanes=4)
    ref.step(w.steps)
    assert np.array_equal(g.u(), ref.u())
