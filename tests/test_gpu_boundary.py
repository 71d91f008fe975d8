"""Boundary calls around the step: a problem on a family the caller supplies
(pd_set_family) and readouts into device memory (pd_get_*_dev into torch tensors).
Bars: bit-identical to the host-built family and to the host readouts; a caller's
family against the oracle on the same CSR at the FP64 bar; malformed families and
non-device buffers rejected before any kernel runs."""
import numpy as np
import pytest

import pd_inputs as pi
from oracle.oracle import OracleSim, family
from parity import TOL_FP64, compare, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    from paper_2105_04150_amd import _binding as B
    B.load()


def _setup(g, w):
    from paper_2105_04150_amd import apply_workload
    g.set_integrator(w.scheme, w.dt)
    apply_workload(g, w)


@pytest.mark.parametrize("mapping,lanes", [("sliced", 4), ("staged", 1)])
def test_imported_family_equals_built_family(mapping, lanes):
    """The family pd_build_family finds, handed back through pd_set_family, gives the
    same run bit for bit."""
    from paper_2105_04150_amd import Simulation
    w = pi.workload("block10", dims=(12, 10, 9), steps=400)
    with Simulation() as a, Simulation() as b:
        for g in (a, b):
            g.set_mapping(mapping, lanes)
        a.build_family(w.coords, w.horizon)
        rp, col = a.family()
        b.set_family(w.coords, rp, col)
        rp2, col2 = b.family()
        assert np.array_equal(rp, rp2) and np.array_equal(col, col2)
        for g in (a, b):
            _setup(g, w)
            g.step(w.steps)
        assert np.array_equal(a.u(), b.u()) and np.array_equal(a.broken(), b.broken())


def test_custom_family_matches_oracle():
    """A neighbourhood that no horizon produces (the delta family with a symmetric random
    tenth of its bonds removed) against the oracle on the same CSR."""
    from paper_2105_04150_amd import Simulation
    w = pi.workload("block10", dims=(11, 10, 9), steps=500)
    rp, col = family(w.coords, w.horizon)
    n = w.n
    rows = np.repeat(np.arange(n), np.diff(rp))
    key = np.minimum(rows, col).astype(np.uint64) * np.uint64(n) + np.maximum(rows, col).astype(np.uint64)
    keep = pi.uniform01(31, key) >= 0.1
    rp2 = np.zeros(n + 1, dtype=np.int64)
    rp2[1:] = np.cumsum(np.bincount(rows[keep], minlength=n))
    col2 = col[keep]
    o = OracleSim(w.coords, rp2, col2, c=w.c, s0=w.s0, rho=w.rho, dt=w.dt, vol=w.volume, bcs=w.bcs)
    o.run(w.steps)
    with Simulation() as g:
        g.set_mapping("staged", 2)
        g.set_family(w.coords, rp2, col2)
        _setup(g, w)
        g.step(w.steps)
        eu, ev, mism, ephi = compare(g, o, TOL_FP64, "caller's family (10% of bonds removed)")
        assert int(o.broken_mask.sum()) > 50
        assert mism == 0 and eu <= TOL_FP64 and ephi <= 1e-13


def test_malformed_families_rejected():
    from paper_2105_04150_amd import PdmiError, Simulation
    x = np.array([[0.0, 0.0, 0.0], [1e-3, 0.0, 0.0], [2e-3, 0.0, 0.0]])
    good_rp, good_col = np.array([0, 1, 3, 4]), np.array([1, 0, 2, 1])
    bad = [
        (np.array([0, 1, 2, 3]), np.array([1, 0, 1])),        # 2 -> 1 without 1 -> 2
        (np.array([0, 1, 3, 4]), np.array([1, 2, 0, 1])),     # row 1 not ascending
        (np.array([0, 1, 3, 4]), np.array([0, 0, 2, 1])),     # self bond
        (np.array([0, 1, 3, 4]), np.array([1, 0, 5, 1])),     # out of range
        (np.array([1, 1, 3, 4]), np.array([1, 0, 2, 1])),     # row_ptr[0] != 0
        (np.array([0, 2, 1, 4]), np.array([1, 0, 2, 1])),     # decreasing row_ptr
    ]
    with Simulation() as g:
        g.set_family(x, good_rp, good_col)
        assert g.size() == (3, 4)
        for rp, col in bad:
            with pytest.raises(PdmiError):
                g.set_family(x, rp, col)
        same = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 0.0], [2e-3, 0.0, 0.0]])
        with pytest.raises(PdmiError):
            g.set_family(same, good_rp, good_col)
        assert g.size() == (3, 4)  # all-or-nothing: the good problem is still there


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_device_readouts_equal_host_readouts(precision):
    import torch
    from paper_2105_04150_amd import PD_FP32, PD_FP64, simulation_for
    w = pi.workload("block10", dims=(12, 10, 9), steps=800)  # long enough to break bonds
    g = simulation_for(w, precision=PD_FP32 if precision == "f32" else PD_FP64, mapping="staged")
    g.step(w.steps)
    u = torch.full((w.n, 3), float("nan"), dtype=torch.float64, device="cuda")
    v = torch.full((w.n, 3), float("nan"), dtype=torch.float64, device="cuda")
    phi = torch.full((w.n,), float("nan"), dtype=torch.float64, device="cuda")
    g.u_dev(u)
    g.v_dev(v)
    g.damage_dev(phi)
    g.sync()
    assert np.array_equal(u.cpu().numpy(), g.u())
    assert np.array_equal(v.cpu().numpy(), g.v())
    assert np.array_equal(phi.cpu().numpy(), g.damage())
    assert g.damage().max() > 0
    say(f"[boundary] device readouts ({precision}) equal the host readouts")


def test_device_readouts_of_a_batch_and_bad_buffers():
    import torch
    from paper_2105_04150_amd import PdmiError, Simulation, apply_workload
    from paper_2105_04150_amd import _binding as B
    wa = pi.workload("block10", dims=(9, 8, 7), steps=100)
    wb = pi.workload("block10", dims=(7, 7, 6), steps=100)
    with Simulation() as g:
        g.set_mapping("sliced", 4)
        g.build_family_batch([wa.coords, wb.coords], [wa.horizon, wb.horizon])
        g.set_integrator("euler_cromer", wa.dt)
        apply_workload(g, wa, inst=0)
        apply_workload(g, wb, inst=1)
        g.step(100)
        for b, w in enumerate((wa, wb)):
            u = torch.empty((w.n, 3), dtype=torch.float64, device="cuda")
            g.u_dev(u, inst=b)
            g.sync()
            assert np.array_equal(u.cpu().numpy(), g.u(b))
        # host memory and a short tensor never reach a kernel
        host = np.zeros((wa.n, 3))
        with pytest.raises(PdmiError):
            B._check(g.ctx, B.load().pd_get_u_dev(g.ctx, 0, host.ctypes.data))
        with pytest.raises(ValueError):
            g.u_dev(torch.empty((wa.n - 1, 3), dtype=torch.float64, device="cuda"))
        with pytest.raises(ValueError):
            g.u_dev(torch.empty((wa.n, 3), dtype=torch.float64))
