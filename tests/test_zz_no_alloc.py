"""The allocation-free set readout (pd_get_mean_displacement_noalloc) through the C ABI:
the same three numbers as pd_get_mean_displacement, bit for bit, on two calls in a row
(the second with a smaller node set, so a stale tail of the shared device array would
show), FP64 and FP32 builds and two instances; sizes beyond the array are refused."""
import numpy as np
import pytest

import pd_inputs as pi
from parity import say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_noalloc_mean_matches_allocating_readout(precision):
    from paper_2105_04150_amd import PD_FP32, PD_FP64, PdmiError, Simulation, apply_workload
    from paper_2105_04150_amd import _binding as B
    wa = pi.workload("block10", dims=(12, 10, 9), steps=300)
    wb = pi.workload("block10", dims=(9, 8, 7), steps=300)
    with Simulation(precision=PD_FP32 if precision == "f32" else PD_FP64) as g:
        g.set_mapping("staged", 1)
        g.build_family_batch([wa.coords, wb.coords], [wa.horizon, wb.horizon])
        g.set_integrator("euler_cromer", wa.dt)
        apply_workload(g, wa, inst=0)
        apply_workload(g, wb, inst=1)
        g.step(300)
        rng = np.random.default_rng(3)
        big = rng.choice(wa.n, size=700, replace=False)
        small = rng.choice(wb.n, size=37, replace=False)
        for inst, nodes in ((0, big), (1, small), (0, big[:5])):
            want = B.pd_get_mean_displacement(g.ctx, inst, nodes)
            got = B.pd_get_mean_displacement_noalloc(g.ctx, inst, nodes)
            assert np.abs(want).max() > 0
            assert np.array_equal(got.view(np.int64), want.view(np.int64)), (inst, got, want)
        say(f"[no-alloc] {precision}: three calls (700, 37, 5 nodes) equal the allocating readout bit for bit")
        with pytest.raises(PdmiError):
            B.pd_get_mean_displacement_noalloc(g.ctx, 0, np.zeros(262145, dtype=np.int64))
        with pytest.raises(PdmiError):
            B.pd_get_mean_displacement_noalloc(g.ctx, 0, np.array([wa.n]))
        with pytest.raises(PdmiError):
            B.pd_get_mean_displacement_noalloc(g.ctx, 0, np.zeros(0, dtype=np.int64))
