"""n-linear damage laws and bond classes on the GPU against the oracle (Secs. 3.6, 6, 7).

The notched three-point bend with the trilinear law of Sec. 6 (and a composite variant:
trilinear matrix bonds and bilinear fibre bonds mixed at random, fibre bonds twice as
stiff) softens thousands of bonds and breaks thousands more.  Bars as everywhere: FP64
displacement 1e-10 norm-wise with identical broken sets; here also identical softened
sets.  The stretch state is a difference of displacements over a bond length, so it is
held to the displacement bar in displacement units: max |s_gpu - s_ref| dx / (2 |u|_max)
<= 1e-10 over the slots softened on both sides.  Damage, 1 - secant ratio, moves with the
stretch state at up to s_0 |rho'| / s (about 60 for the trilinear law): 1e-9 absolute.
FP32: 1e-5 with counted mismatches.
"""
import numpy as np
import pytest

import pd_inputs as pi
from oracle.oracle import from_workload
from parity import TOL_FP32, TOL_FP64, compare, oracle_run, rel_err, say

pytestmark = pytest.mark.gpu

SMALL = dict(dims=(35, 10, 10), steps=1600)
MAPPINGS = [("sliced", 4), ("sliced", 1), ("staged", 1), ("staged", 4)]


@pytest.fixture(scope="module", autouse=True)
def _lib():
    from paper_2105_04150_amd import _binding as B
    B.load()


def _workload(law, **kw):
    w = pi.workload("qs_beam", law=law, **dict(SMALL, **kw))
    return w


def _sim(w, mapping, lanes, precision=None):
    from paper_2105_04150_amd import PD_FP64, simulation_for
    g = simulation_for(w, lanes=lanes, mapping=mapping, precision=PD_FP64 if precision is None else precision)
    if w.class_spec is not None:  # fibre bonds twice as stiff (per-slot stiffness by class)
        rp, col = g.family()
        cls = pi.bond_classes(rp, col, *w.class_spec)
        g.set_bond_stiffness(np.where(cls == 1, 2.0 * w.c, w.c))
    return g


def _oracle(w, steps, class_stiffness=True):
    o = from_workload(w)
    if w.class_spec is not None and class_stiffness:
        cls = pi.bond_classes(o.row_ptr, o.col, *w.class_spec)
        o.kslot = np.ascontiguousarray(np.where(cls == 1, 2.0 * w.c, w.c))
        o.P.kslot = o.kslot.ctypes.data
    o.run(steps)
    return o


@pytest.fixture(scope="module", params=["trilinear", "composite"])
def law_oracle(request):
    w = _workload(request.param)
    say(f"[run] oracle qs_beam {request.param} {w.dims}, {w.steps} steps")
    return w, _oracle(w, w.steps)


def _oracle_spread(w, steps, o, class_stiffness):
    """Conditioning of a softening run: the relative displacement difference between the
    oracle's run and the same run with every coordinate moved by one ulp.  A softening
    branch is a negative-stiffness region, where rounding-level differences (the oracle's
    printed-form stretch |y| - |xi| alone carries about 1e-16/s relative) grow with time."""
    import copy
    w2 = copy.copy(w)
    w2.coords = np.nextafter(w.coords, np.inf)
    o2 = _oracle(w2, steps, class_stiffness)
    return rel_err(o2.u, o.u)


def _stretch_err(sg, so, u_ref):
    """Stretch-state error in displacement units over the slots softened on both sides."""
    both = (sg > 0) & (so > 0)
    return float(np.abs(sg - so)[both].max() * pi.DX / (2.0 * np.abs(u_ref).max())) if both.any() else 0.0


def _compare_state(g, o, tol, what, inst=0):
    eu, ev, mism, ephi = compare(g, o, tol, what, inst=inst)
    sg, so = g.max_stretch(inst), o.smax[: o.nnz]
    soft_mism = int(((sg > 0) != (so > 0)).sum())
    es = _stretch_err(sg, so, o.u)
    say(f"[laws] {what}: softened {int((so > 0).sum())} (mismatched {soft_mism}), stretch state (displacement units) {es:.2e}")
    return eu, ev, mism, ephi, soft_mism, es


@pytest.mark.parametrize("mapping,lanes", MAPPINGS)
def test_laws_match_oracle(law_oracle, mapping, lanes):
    w, o = law_oracle
    g = _sim(w, mapping, lanes)
    g.step(w.steps)
    eu, ev, mism, ephi, smism, es = _compare_state(g, o, TOL_FP64, f"{w.class_spec and 'composite' or 'trilinear'} "
                                                                  f"{mapping}-{lanes}")
    nb0 = int(pi.notch_mask(w.ijk, o.row_ptr, o.col, *w.notch).sum())
    assert int(o.broken_mask.sum()) - nb0 > 100 and int((o.smax[: o.nnz] > 0).sum()) > 1000
    assert mism == 0 and smism == 0
    assert eu <= TOL_FP64 and ev <= TOL_FP64 and es <= TOL_FP64 and ephi <= 1e-9


# FP32 with a softening law: the records carry f32 displacements, so a bond's stretch
# has a relative error near 6e-8 |u| / (s L), and the secant ratio amplifies relative
# stretch errors by |s rho'/rho - 1|, up to about 60 on the steep first branch of the
# trilinear law (rho drops from 1 to 1/4 between s = 2.3e-4 and 2.42e-4); the bar is
# therefore 5e-5 instead of the 1e-5 of the brittle law.
TOL_FP32_SOFTENING = 5e-5


def test_laws_fp32(law_oracle):
    """The trilinear beam is held to TOL_FP32_SOFTENING (measured 1.9e-5); the composite,
    whose bonds mostly sit on gentler branches, meets the brittle law's 1e-5 (measured
    1.5e-6)."""
    from paper_2105_04150_amd import PD_FP32
    w, o = law_oracle
    bar = TOL_FP32 if w.class_spec is not None else TOL_FP32_SOFTENING
    g = _sim(w, "staged", 1, precision=PD_FP32)
    g.step(w.steps)
    eu, ev, mism, ephi, smism, es = _compare_state(g, o, bar, "fp32")
    nsoft = int((o.smax[: o.nnz] > 0).sum())
    assert eu <= bar and mism <= 0.01 * int(o.broken_mask.sum()) and smism <= 0.01 * nsoft


def test_force_readout_with_softened_bonds(law_oracle):
    """The readout at the library's own state against the oracle's force at that state
    (same displacement, broken set and stretch state, nothing updated)."""
    w, o = law_oracle
    g = _sim(w, "staged", 1)
    g.step(w.steps)
    u, br, sm = g.u(), g.broken().astype(bool), g.max_stretch()
    fr = np.where(br, np.iinfo(np.int32).min, np.iinfo(np.int32).max).astype(np.int32)
    ref = from_workload(w, frozen=fr)
    ref.smax[: ref.nnz] = sm
    if w.class_spec is not None:
        cls = pi.bond_classes(ref.row_ptr, ref.col, *w.class_spec)
        ref.kslot = np.ascontiguousarray(np.where(cls == 1, 2.0 * w.c, w.c))
        ref.P.kslot = ref.kslot.ctypes.data
    F_ref = ref.force(u=u, k=0)
    e = float(np.abs(g.force() - F_ref).max() / np.abs(F_ref).max())
    say(f"[laws] force readout rel {e:.2e}")
    assert e <= 1e-12
    assert np.array_equal(g.max_stretch(), sm)  # the readout changed nothing


def test_checkpoint_restart_and_layout_change():
    """Stop, save (u, v, a, broken, stretch state), restore into a fresh simulation with the
    other mapping, continue: equal to the oracle's uninterrupted run."""
    w = _workload("trilinear")
    o = _oracle(w, w.steps)
    g = _sim(w, "staged", 1)
    g.step(900)
    state = dict(u=g.u(), v=g.v(), a=g.a(), broken=g.broken())
    sm = g.max_stretch()
    assert (sm > 0).sum() > 100
    h = _sim(w, "sliced", 4)
    h.set_state(**state)
    h.set_max_stretch(sm)
    h.set_step(900)
    assert np.array_equal(h.max_stretch(), sm)
    h.step(w.steps - 900)
    eu, ev, mism, ephi, smism, es = _compare_state(h, o, TOL_FP64, "restarted")
    assert mism == 0 and smism == 0 and eu <= TOL_FP64 and es <= TOL_FP64
    # a mapping change rebuilds the layout and keeps the stretch state
    g.set_mapping("sliced", 16)
    assert np.array_equal(g.max_stretch(), sm)
    g.step(w.steps - 900)
    eu, ev, mism, ephi, smism, es = _compare_state(g, o, TOL_FP64, "after a layout change")
    assert mism == 0 and smism == 0 and eu <= TOL_FP64


# The batched case runs 1,200 steps with the loads ramped over that run: there the oracle's
# own rounding spread (every coordinate moved by one ulp) is 1.3e-10 for the trilinear beam
# and 4.8e-11 for the 30 x 9 x 9 composite; at 1,600 steps the composites soften into an
# ill-conditioned regime (spreads 2.6e-10 to 6.5e-9), which no fixed bar can hold.
BATCH_STEPS = 1200
SPREAD_MAX = 2.5e-10   # the case must be this well conditioned ...
BAR_CAP = 1e-9         # ... so the bar, four times the spread, never exceeds this


def test_batched_mixed_laws():
    """One instance with the trilinear law, one brittle, one composite: each matches its
    oracle (laws are per instance; the kernels see all three in one launch)."""
    from paper_2105_04150_amd import Simulation, apply_workload
    n = BATCH_STEPS
    ws = [_workload("trilinear", steps=n), _workload("brittle", dims=(30, 9, 9), steps=n),
          _workload("composite", dims=(30, 9, 9), steps=n)]
    with Simulation() as g:
        g.set_mapping("staged", 1)
        g.build_family_batch([w.coords for w in ws], [w.horizon for w in ws])
        g.set_integrator(ws[0].scheme, ws[0].dt)
        for b, w in enumerate(ws):
            apply_workload(g, w, inst=b)
        g.step(n)
        for b, w in enumerate(ws):
            o = from_workload(w)
            o.run(n)
            # the bar: 1e-10, or four times the run's own rounding spread where softening
            # has grown it beyond that, never above BAR_CAP
            bar = TOL_FP64
            if w.laws:
                spread = _oracle_spread(w, n, o, class_stiffness=False)
                say(f"[laws] inst {b}: oracle spread under one-ulp coordinates {spread:.2e}")
                assert spread <= SPREAD_MAX, "the case is not conditioned well enough for a fixed bar"
                bar = min(BAR_CAP, max(TOL_FP64, 4.0 * spread))
                eu, ev, mism, ephi, smism, es = _compare_state(g, o, bar, f"mixed laws inst {b}", inst=b)
                assert smism == 0 and es <= bar
                assert int((o.smax[: o.nnz] > 0).sum()) > 1000
            else:
                eu, ev, mism, ephi = compare(g, o, TOL_FP64, f"mixed laws inst {b}", inst=b)
            assert mism == 0 and eu <= bar <= BAR_CAP


def test_law_arguments_and_reset():
    from paper_2105_04150_amd import PdmiError, simulation_for
    w = _workload("trilinear", dims=(20, 6, 6), steps=10)
    w.scheme = "euler_cromer"
    g = simulation_for(w, lanes=4)
    bad = [(2, [1e-3], [1.0]),                          # class out of order (one defined)
           (0, [2e-3, 1e-3], [1.0, 0.0]),               # decreasing breakpoints
           (0, [1e-3, 2e-3], [0.5, 0.0]),               # does not start at ratio 1
           (0, [1e-3, 2e-3], [1.0, 0.1]),               # does not end at ratio 0
           (0, [-1e-3], [1.0]),                         # negative stretch
           (0, [1e-3] * 9, [1.0] * 9),                  # too many breakpoints
           (8, [1e-3], [1.0])]                          # class out of range
    for cls, sb, rb in bad:
        with pytest.raises(PdmiError):
            g.set_damage_law(cls, sb, rb)
    rp, col = g.family()
    asym = np.zeros(rp[-1], dtype=np.uint8)
    asym[0] = 1
    g.set_damage_law(1, [4e-4, 1e-3], [1.0, 0.0])
    with pytest.raises(PdmiError):
        g.set_bond_classes(asym)                        # asymmetric
    with pytest.raises(PdmiError):
        g.set_bond_classes(np.full(rp[-1], 2, dtype=np.uint8))  # class without a law
    with pytest.raises(PdmiError):
        g.adj_forward(10, 5)                            # the adjoint takes brittle laws only
    g.step(10)
    g.clear_damage_laws()
    with pytest.raises(PdmiError):
        g.set_max_stretch(np.zeros(rp[-1]))              # no laws any more
    g.step(10)


def test_one_breakpoint_law_matches_brittle_oracle():
    """A single-breakpoint law runs the bond-model branch and reproduces the brittle law."""
    from paper_2105_04150_amd import simulation_for
    w = pi.workload("block10", dims=(10, 8, 8), steps=600)
    o = oracle_run(w, w.steps)
    for mapping, lanes in (("sliced", 4), ("staged", 1)):
        g = simulation_for(w, lanes=lanes, mapping=mapping)
        g.set_damage_law(0, [w.s0], [1.0])
        g.step(w.steps)
        eu, ev, mism, ephi = compare(g, o, TOL_FP64, f"one-breakpoint law {mapping}-{lanes}")
        assert int(o.broken_mask.sum()) > 500
        assert mism == 0 and eu <= TOL_FP64
