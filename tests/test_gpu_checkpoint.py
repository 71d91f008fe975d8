"""Checkpoint and restart through pd_get_state / pd_load_state (Sec. 3.6: a run may
continue from a saved intermediate state).

Bar: a run of N steps, exported, loaded into a fresh context holding the same problem
and continued for M steps equals the uninterrupted N + M step run bit for bit:
displacement, velocity, acceleration, broken set, break steps, stretch state and damage.
Euler-Cromer and velocity Verlet (whose restart re-forms the displacement of the next
level from the saved acceleration), both mappings, the FP32 build and a damage law.
"""
import numpy as np
import pytest

import pd_inputs as pi
from parity import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    from paper_2105_04150_amd import _binding as B
    B.load()


def _make(w, mapping, precision, law):
    from paper_2105_04150_amd import PD_FP32, PD_FP64, simulation_for
    g = simulation_for(w, precision=PD_FP32 if precision == "f32" else PD_FP64, mapping=mapping)
    if law:
        g.set_damage_law(0, [6e-4, 8e-4, 1.5e-3], [1.0, 0.25, 0.0])
    return g


@pytest.mark.parametrize("scheme", ["euler_cromer", "velocity_verlet"])
@pytest.mark.parametrize("mapping,precision,law", [("staged", "f64", False), ("sliced", "f64", False),
                                                   ("staged", "f32", False), ("staged", "f64", True)])
def test_restart_is_bitwise(scheme, mapping, precision, law):
    w = pi.workload("block10", dims=(10, 9, 8), steps=1000)
    w.scheme = scheme
    n1, n2 = 500, 500
    ref = _make(w, mapping, precision, law)
    ref.step(n1 + n2)
    want = ref.get_state()
    phi = ref.damage()
    a = _make(w, mapping, precision, law)
    a.step(n1)
    saved = a.get_state()
    a.close()
    assert saved["step"] == n1
    b = _make(w, mapping, precision, law)
    b.load_state(saved)
    assert b.step_count == n1
    b.step(n2)
    got = b.get_state()
    say(f"[checkpoint] {scheme} {mapping} {precision} law={law}: broken {int(want['broken'].sum())}, "
        f"softened {int((want['max_stretch'] > 0).sum())}, step {got['step']}")
    assert int(want["broken"].sum()) + int((want["max_stretch"] > 0).sum()) > 100
    for key in ("u", "v", "a", "broken", "break_step", "max_stretch"):
        assert np.array_equal(got[key], want[key]), key
    assert got["step"] == want["step"] == n1 + n2
    assert np.array_equal(b.damage(), phi)
    if law:
        assert (want["max_stretch"] > 0).sum() > 0
    for g in (ref, b):
        g.close()


def test_load_state_checks_its_input():
    from paper_2105_04150_amd import PdmiError
    w = pi.workload("block10", dims=(6, 6, 6), steps=10)
    g = _make(w, "staged", "f64", False)
    s = g.get_state()
    bad = dict(s)
    bad["u"] = s["u"].copy()
    bad["u"][0, 0] = np.nan
    with pytest.raises(PdmiError):
        g.load_state(bad)
    g.load_state({"max_stretch": s["max_stretch"], "step": 0})  # all zeros: ignored without laws
    with pytest.raises(PdmiError):  # a stretch state without damage laws
        g.load_state({"max_stretch": s["max_stretch"] + 1e-4, "step": 0})
    with pytest.raises(PdmiError):
        g.load_state({"step": -1})
    g.load_state({"step": 7})  # every array kept, the counter set
    assert g.step_count == 7 and np.array_equal(g.u(), s["u"])
    g.close()
