"""Break decisions equal to the oracle's by construction (FP64 build).

The paper's rule (Eq. mu, Algorithm 2) keeps a bond only while s < s0, with
s = (|y| - |xi|)/|xi|.  The kernels decide on a fast q-form almost always, and on
the oracle's exact sequence of operations inside a narrow margin around every
threshold.  These tests read the same x and u on both sides and require the same
decision slot for slot, with thresholds placed -2, -1, 0, +1 and +2 ulp from the
oracle's own stretch of each bond:
- the device's exact stretch agrees bit for bit with an IEEE host evaluation (correctly
  rounded square root and division on the device);
- two-node bonds, both mappings, the plain kernels and the bond-model kernels (a
  no-failure zone elsewhere, a one-breakpoint law, the trilinear law's elastic limit and
  last breakpoint, whose stored stretch must equal the oracle's bit for bit);
- a jittered lattice under a uniform dilation with s0 at the median of the bonds' own
  stretches (about half the slots break on rounding alone), bond-based and state-based.
"""
import numpy as np
import pytest

import pd_inputs as pi
from parity import say

pytestmark = pytest.mark.gpu

OFFSETS = (-2, -1, 0, 1, 2)  # threshold minus the bond's stretch, in ulps of the stretch


@pytest.fixture(scope="module", autouse=True)
def _lib():
    from paper_2105_04150_amd import _binding as B
    B.load()


def host_stretch(xi, y):
    """The oracle's stretch, evaluated with numpy (element-wise IEEE operations)."""
    r = np.sqrt((y[:, 0] * y[:, 0] + y[:, 1] * y[:, 1]) + y[:, 2] * y[:, 2])
    L = np.sqrt((xi[:, 0] * xi[:, 0] + xi[:, 1] * xi[:, 1]) + xi[:, 2] * xi[:, 2])
    return (r - L) / L


def ulps(s, k):
    """s moved by k ulps (k may be negative)."""
    out = np.asarray(s, dtype=np.float64).copy()
    for _ in range(abs(k)):
        out = np.nextafter(out, np.inf if k > 0 else -np.inf)
    return out


def test_device_exact_stretch_is_ieee():
    from paper_2105_04150_amd import _binding as B
    rng = np.random.default_rng(11)
    m = 400_000
    n = rng.normal(size=(m, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    scale = 10.0 ** rng.uniform(-4, 1, size=(m, 1))  # bond lengths from 1e-4 to 10
    xi = n * scale * (1.0 + 1e-3 * rng.uniform(-1, 1, size=(m, 1)))
    # stretches from 1e-14 to 0.3, both signs, plus a transverse part (rotation)
    s = np.sign(rng.uniform(-1, 1, size=(m, 1))) * 10.0 ** rng.uniform(-14, -0.5, size=(m, 1))
    t = rng.normal(size=(m, 3)) * scale * 10.0 ** rng.uniform(-12, -2, size=(m, 1))
    y = xi * (1.0 + s) + t
    # hard cases: y a one-ulp neighbour of xi, and unstretched bonds (y == xi)
    y[:2000] = np.nextafter(xi[:2000], np.inf)
    y[2000:4000] = xi[2000:4000]
    want = host_stretch(xi, y)
    got = B.pd_stretch_exact(xi, y)
    bad = np.nonzero(got.view(np.int64) != want.view(np.int64))[0]
    say(f"[exact stretch] {m} bonds, {bad.size} differ from the host")
    assert bad.size == 0, (xi[bad[:3]], y[bad[:3]], got[bad[:3]], want[bad[:3]])


def two_node_cases(count, seed, s_target=1e-3):
    """Bonds of length about 1 mm in random directions stretched to about s_target, with
    a small transverse displacement; per case: coords (3 x 3, the third node far from
    the pair), u (3 x 3) and the oracle's stretch of the bond."""
    rng = np.random.default_rng(seed)
    cases = []
    for _ in range(count):
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        L = 1e-3 * (1.0 + 1e-3 * rng.uniform(-1, 1))
        x0 = rng.uniform(-1e-6, 1e-6, size=3)
        x = np.array([x0, x0 + L * n, x0 + 20.0 * L * np.array([1.0, 0.0, 0.0])])
        u0 = rng.uniform(-1e-6, 1e-6, size=3)
        tr = np.cross(n, rng.normal(size=3)) * 1e-8
        u = np.array([u0, u0 + s_target * (1.0 + 0.1 * rng.uniform(-1, 1)) * L * n + tr, np.zeros(3)])
        xi = (x[1] - x[0])[None]
        y = xi + (u[1] - u[0])[None]
        cases.append((x, u, float(host_stretch(xi, y)[0])))
    return cases


def run_pairs(cases, thresholds, mapping, law=None, zone=False, steps=1):
    """One problem of len(cases) * len(OFFSETS) two-node instances advanced `steps`
    Euler-Cromer steps from the given displacements; law(s_o, k) gives each instance's
    damage law (breakpoints, ratios) or None for the brittle s0 = thresholds[c][k].
    Returns, per instance, the GPU's and the oracle's broken flags and stored stretches."""
    from oracle.oracle import OracleSim, family
    from paper_2105_04150_amd import Simulation
    L0 = 1e-3
    horizon = 1.5 * L0
    K = 1.4e10
    c = pi.pmb_micromodulus(K, horizon)
    rho, dt, vol = 2400.0, 1e-8, L0 ** 3
    inst = [(ci, k) for ci in range(len(cases)) for k in range(len(OFFSETS))]
    sim = Simulation()
    sim.set_mapping(mapping, 1)
    sim.build_family_batch([cases[ci][0] for ci, _ in inst], [horizon] * len(inst))
    sim.set_integrator("euler_cromer", dt)
    out = []
    for b, (ci, k) in enumerate(inst):
        x, u, s_o = cases[ci]
        s0 = thresholds[ci][k]
        lw = law(s_o, OFFSETS[k]) if law else None
        sim.set_material(rho, c, 1.0 if lw else s0, volume=vol, inst=b)
        if lw:
            sim.set_damage_law(0, lw[0], lw[1], inst=b)
        if zone:
            sim.set_no_fail([2], inst=b)  # the far node: the pair stays breakable
        sim.set_state(u=u, v=np.zeros((3, 3)), inst=b)
    sim.step(steps)
    sim.sync()
    for b, (ci, k) in enumerate(inst):
        x, u, s_o = cases[ci]
        rp, col = family(x, horizon)
        assert int(rp[-1]) == 2
        o = OracleSim(x, rp, col, c=c, s0=1.0 if law else thresholds[ci][k], rho=rho, dt=dt, vol=vol,
                      laws=[law(s_o, OFFSETS[k])] if law else None,
                      nofail=np.array([0, 0, 1], dtype=np.uint8) if zone else None)
        o.set_state(u=u)
        assert o.run(steps) == 0
        gsm = sim.max_stretch(b) if law else np.zeros(2)
        osm = o.smax[:2] if law else np.zeros(2)
        out.append((sim.broken(b).astype(bool), o.broken_mask.copy(), gsm, osm))
    sim.close()
    return out


@pytest.mark.parametrize("mapping", ["staged", "sliced"])
@pytest.mark.parametrize("variant", ["plain", "zone", "brittle_law"])
def test_two_node_brittle_threshold_ulps(oracle_lib, mapping, variant):
    cases = two_node_cases(12, seed=3)
    thr = [[float(ulps(s_o, k)) for k in OFFSETS] for _, _, s_o in cases]
    law = (lambda s_o, k: ([float(ulps(s_o, k))], [0.0])) if variant == "brittle_law" else None
    res = run_pairs(cases, thr, mapping, law=law, zone=variant == "zone")
    want = np.array([[k <= 0] for _ in cases for k in OFFSETS]).ravel()  # s_o >= s0 breaks
    got = np.array([g[0] for g, _, _, _ in res])
    orc = np.array([o[0] for _, o, _, _ in res])
    say(f"[break ulps] {mapping} {variant}: {int(got.sum())} of {got.size} broken "
        f"(oracle {int(orc.sum())}, rule {int(want.sum())})")
    assert np.array_equal(orc, want)
    for g, o, _, _ in res:
        assert np.array_equal(g, o)


@pytest.mark.parametrize("mapping", ["staged", "sliced"])
@pytest.mark.parametrize("which", ["elastic_limit", "last_breakpoint"])
def test_two_node_trilinear_threshold_ulps(oracle_lib, mapping, which):
    """Softening starts when the stretch exceeds the elastic limit s_0 (strictly); the
    bond breaks when it reaches the last breakpoint.  The stored stretch of a softened
    slot is the oracle's, bit for bit."""
    cases = two_node_cases(10, seed=5)
    thr = [[0.0] * len(OFFSETS) for _ in cases]
    if which == "elastic_limit":
        def law(s_o, k):
            s1 = float(ulps(s_o, k))
            return ([s1, 4.0 * s_o, 10.0 * s_o], [1.0, 0.25, 0.0])
        want = np.array([k < 0 for _ in cases for k in OFFSETS])   # softened iff s_o > s_1
    else:
        def law(s_o, k):
            return ([0.25 * s_o, 0.5 * s_o, float(ulps(s_o, k))], [1.0, 0.25, 0.0])
        want = np.array([k <= 0 for _ in cases for k in OFFSETS])  # broken iff s_o >= s_last
    res = run_pairs(cases, thr, mapping, law=law)
    for i, (g, o, gsm, osm) in enumerate(res):
        assert np.array_equal(g, o), i
        assert np.array_equal(gsm.view(np.int64), osm.view(np.int64)), (i, gsm, osm)
    if which == "elastic_limit":
        soft = np.array([gsm[0] > 0 for _, _, gsm, _ in res])
        say(f"[trilinear ulps] {mapping} elastic limit: {int(soft.sum())} of {soft.size} softened")
        assert np.array_equal(soft, want)
    else:
        brk = np.array([g[0] for g, _, _, _ in res])
        say(f"[trilinear ulps] {mapping} last breakpoint: {int(brk.sum())} of {brk.size} broken")
        assert np.array_equal(brk, want)


def dilated_lattice(dims=(8, 8, 8), eps=1e-3):
    """Jittered lattice under u = eps x: every bond's stretch is eps up to rounding."""
    dx = 1e-3
    x, _ = pi.lattice(dims, dx, jitter=1e-3, seed=21)
    return x, eps * x, dx


@pytest.mark.parametrize("mapping,model", [("staged", "pmb"), ("sliced", "pmb"), ("staged", "state_based"),
                                           ("staged", "pmb_zone")])
def test_lattice_median_threshold(oracle_lib, mapping, model):
    from oracle.oracle import OracleSim, family
    from paper_2105_04150_amd import Simulation
    x, u, dx = dilated_lattice()
    horizon = 3.015 * dx
    rp, col = family(x, horizon)
    i = np.repeat(np.arange(x.shape[0]), np.diff(rp))
    xi = x[col] - x[i]
    y = xi + (u[col] - u[i])
    s = host_stretch(xi, y)
    s0 = float(np.median(s))
    K = 1.4e10
    c = pi.pmb_micromodulus(K, horizon)
    state_based = (K, 0.75 * K) if model == "state_based" else None  # G for Poisson ratio 0.2
    zone = np.zeros(x.shape[0], dtype=np.uint8)
    if model == "pmb_zone":
        zone[0] = 1  # a corner node: its bonds never break (the bond-model kernels run)
    o = OracleSim(x, rp, col, c=c, s0=s0, rho=2400.0, dt=1e-8, vol=dx ** 3, state_based=state_based,
                  nofail=zone if model == "pmb_zone" else None)
    o.set_state(u=u)
    assert o.run(1) == 0
    with Simulation() as sim:
        sim.set_mapping(mapping, 1)
        sim.build_family(x, horizon)
        sim.set_integrator("euler_cromer", 1e-8)
        sim.set_material(2400.0, c, s0, volume=dx ** 3)
        if state_based:
            sim.set_model("state_based", *state_based)
        if model == "pmb_zone":
            sim.set_no_fail([0])
        sim.set_state(u=u, v=np.zeros_like(u))
        sim.step(1)
        sim.sync()
        g = sim.broken().astype(bool)
    ob = o.broken_mask
    near = np.abs(s / s0 - 1.0) < 1e-12
    say(f"[lattice median] {mapping} {model}: {ob.size} slots, {int(near.sum())} within 1e-12 of s0, "
        f"oracle broke {int(ob.sum())}, mismatched {int((g != ob).sum())}")
    assert 0.3 * ob.size < ob.sum() < 0.7 * ob.size
    assert np.array_equal(g, ob)
