"""Pins of the oracle's n-linear damage laws and bond classes (Secs. 3.7, 6, 7).

A law is given by stretch breakpoints s_0 < ... < s_last and force ratios r_0 = 1, ...,
r_last = 0: a monotonic pull follows c s up to s_0, then c s_0 times the interpolated
ratio, and the bond is broken from s_last on; a softened bond unloads and reloads along
the secant to the origin.  The checks: the force-stretch curve of a single bond at the
breakpoints, between them, under unloading and reloading and past s_last; the work to
break a bond equals the area under the law (for the bilinear law of Sec. 7 the ratio of
the two fracture energies equals s_c/s_0, the relation the paper uses to set it); the
one-breakpoint law is the brittle law bit for bit; uniform dilation gives the closed-form
damage of every node, with one class and with two classes mixed at random; softening is
irreversible and symmetric in a fracturing run; no-failure zones never soften.
"""
import numpy as np
import pytest

import pd_inputs as pi

RHO, C, V, L = 2400.0, 1.0e20, 1.0e-9, 1.0e-3
# Table of optimised trilinear parameters (Sec. 6), point estimate 1, kink ratio 1/4
TRI = ([2.3e-4, 2.42e-4, 1.45e-3], [1.0, 0.25, 0.0])
BI = ([1.0e-4, 2.5e-3], [1.0, 0.0])   # bilinear, k_r = s_c / s_0 = 25


def _bond(oracle_lib, law):
    x = np.array([[0.0, 0.0, 0.0], [L, 0.0, 0.0]])
    rp, col = oracle_lib.family(x, 1.5 * L)
    return oracle_lib.OracleSim(x, rp, col, c=C, s0=1.0, rho=RHO, dt=1e-7, vol=V, laws=[law])


def _pull(sim, s_list):
    """Force on node 0 (x component, per c V) for each stretch of node 1, in order."""
    out = []
    for k, s in enumerate(s_list):
        u = np.zeros((2, 3))
        u[1, 0] = s * L
        out.append(sim.force(u=u, k=k)[0, 0] / (C * V))
    return np.array(out)


def _envelope(law, s):
    sb, rb = law
    if s <= sb[0]:
        return s
    if s >= sb[-1]:
        return 0.0
    return sb[0] * np.interp(s, sb, rb)


@pytest.mark.parametrize("law", [TRI, BI])
def test_single_bond_follows_the_law(oracle_lib, law):
    sb, rb = law
    sim = _bond(oracle_lib, law)
    # loading through every breakpoint and between them
    pts = sorted(set([0.5 * sb[0], sb[0]] + [0.5 * (a + b) for a, b in zip(sb, sb[1:])] + list(sb[1:-1])))
    f = _pull(sim, pts)
    for s, fs in zip(pts, f):
        assert fs == pytest.approx(_envelope(law, s), rel=1e-11), s
    assert f[pts.index(sb[0])] == pytest.approx(sb[0], rel=1e-12)        # peak c s_0
    for k in range(1, len(sb) - 1):
        assert f[pts.index(sb[k])] == pytest.approx(sb[0] * rb[k], rel=1e-11)


def test_unload_and_reload_along_the_secant(oracle_lib):
    sim = _bond(oracle_lib, TRI)
    sa = 0.5 * (TRI[0][1] + TRI[0][2])        # on the second softening branch
    secant = _envelope(TRI, sa) / sa
    path = [1e-4, 2e-4, sa, 0.6 * sa, 0.1 * sa, -0.3 * sa, 0.8 * sa, sa]
    f = _pull(sim, path)
    for s, fs in zip(path[3:], f[3:]):
        assert fs == pytest.approx(secant * s, rel=1e-10), s   # compression included
    sm_before = sim.smax[0]
    assert sm_before == pytest.approx(sa, rel=1e-12)
    # reloading past the previous maximum rejoins the law
    f2 = _pull(sim, [1.1 * sa])
    assert f2[0] == pytest.approx(_envelope(TRI, 1.1 * sa), rel=1e-11)
    assert sim.smax[0] > sm_before
    # past s_last the bond is broken for good: no force in tension or compression
    f3 = _pull(sim, [TRI[0][2], 0.5 * sa, -sa])
    assert np.all(f3 == 0.0) and sim.broken[0] == 1


@pytest.mark.parametrize("law", [TRI, BI])
def test_work_to_break_is_the_area_under_the_law(oracle_lib, law):
    """Quasi-static pull: the trapezoid sum of f ds over fine steps equals the area of the
    law's polygon; for the bilinear law the fracture energies G_f (to break) and G_0 (to
    the elastic limit) stand in the ratio s_c / s_0."""
    sb, rb = law
    sim = _bond(oracle_lib, law)
    s = np.linspace(0.0, sb[-1] * (1 + 1e-9), 20001)
    f = _pull(sim, s)
    work = float(np.sum(0.5 * (f[1:] + f[:-1]) * np.diff(s)))
    area = 0.5 * sb[0] ** 2 + sum(sb[0] * 0.5 * (rb[k] + rb[k + 1]) * (sb[k + 1] - sb[k])
                                  for k in range(len(sb) - 1))
    assert work == pytest.approx(area, rel=2e-4)
    if len(sb) == 2:
        g0 = 0.5 * sb[0] ** 2
        assert work / g0 == pytest.approx(sb[1] / sb[0], rel=2e-4)


def _block(oracle_lib, dims=(6, 5, 5), jitter=1e-3):
    x, ijk = pi.lattice(dims, 1e-3, jitter, seed=5)
    rp, col = oracle_lib.family(x, 3.015e-3)
    return x, rp, col, dict(c=pi.pmb_micromodulus(1.4e10, 3.015e-3), rho=RHO, dt=1e-8, vol=V)


def test_one_breakpoint_law_is_the_brittle_law(oracle_lib):
    x, rp, col, kw = _block(oracle_lib, (8, 5, 5))
    n = x.shape[0]
    ijk = np.rint(x / 1e-3).astype(int)
    bcs = [pi.BCSpec(pi.face_nodes(ijk, 0, 0), 0b111, pi.BC_DISP, (0.0, 0.0, 0.0), pi.SCHED_CONST),
           pi.BCSpec(pi.face_nodes(ijk, 0, 7), 0b001, pi.BC_DISP, (5.0, 0.0, 0.0), pi.SCHED_LINEAR)]
    s0 = 1.0e-3
    a = oracle_lib.OracleSim(x, rp, col, s0=s0, bcs=bcs, **kw)
    b = oracle_lib.OracleSim(x, rp, col, s0=123.0, bcs=bcs, laws=[([s0], [1.0])], **kw)
    a.run(400)
    b.run(400)
    assert a.broken_mask.any()
    assert np.array_equal(a.u, b.u) and np.array_equal(a.v, b.v)
    assert np.array_equal(a.broken_mask, b.broken_mask)
    assert np.array_equal(a.damage(), b.damage())
    assert n > 0


def test_uniform_dilation_damage_closed_form(oracle_lib):
    """u = lam x on an exact lattice stretches every bond by lam: one pass softens every
    bond to 1 - s_0 rho(lam)/lam, the damage of every node; with two classes mixed at
    random (symmetric per bond), node i's damage is the class-weighted mean."""
    x, rp, col, kw = _block(oracle_lib, jitter=0.0)
    n = x.shape[0]
    lam = 0.5 * (TRI[0][1] + TRI[0][2])
    d_tri = 1.0 - _envelope(TRI, lam) / lam
    sim = oracle_lib.OracleSim(x, rp, col, s0=1.0, laws=[TRI], **kw)
    sim.force(u=lam * x, k=0)
    assert np.allclose(sim.damage(), d_tri, rtol=1e-10, atol=0)
    # two classes: TRI and an elastic-until-later bilinear law
    law2 = ([2.0 * lam, 4.0 * lam], [1.0, 0.0])
    rows = np.repeat(np.arange(n), np.diff(rp))
    key = np.minimum(rows, col).astype(np.uint64) * np.uint64(n) + np.maximum(rows, col).astype(np.uint64)
    cls = (pi.uniform01(77, key) < 0.4).astype(np.uint8)
    sim2 = oracle_lib.OracleSim(x, rp, col, s0=1.0, laws=[TRI, law2], slot_cls=cls, **kw)
    sim2.force(u=lam * x, k=0)
    want = np.zeros(n)
    for i in range(n):
        sl = slice(rp[i], rp[i + 1])
        want[i] = np.mean(np.where(cls[sl] == 0, d_tri, 0.0))
    assert np.allclose(sim2.damage(), want, rtol=1e-10, atol=1e-15)
    assert 0.0 < want.min() and want.max() < d_tri


def test_softening_irreversible_and_symmetric(oracle_lib):
    w = pi.workload("qs_beam", dims=(35, 10, 10), steps=1600)
    from oracle.oracle import from_workload
    o = from_workload(w)
    o2 = oracle_lib.OracleSim(o.x, o.row_ptr, o.col, c=w.c, s0=1.0, rho=w.rho, dt=w.dt, vol=w.volume,
                              scheme=w.scheme, eta=w.eta, bcs=w.bcs, ramp_T=w.ramp_T,
                              nofail=o.nofail, broken=o.broken[: o.nnz].copy(), laws=[TRI])
    rows = np.repeat(np.arange(w.n), np.diff(o2.row_ptr))
    order = np.lexsort((rows, o2.col))          # slot of (j, i) for every (i, j): sort by (col, row)
    rev = np.empty(o2.nnz, dtype=np.int64)
    rev[np.lexsort((o2.col, rows))] = order
    prev = np.zeros(o2.nnz)
    for _ in range(8):
        o2.run(200)
        sm = o2.smax[: o2.nnz]
        assert np.all(sm >= prev)
        prev = sm.copy()
    assert (sm > 0).sum() > 100 and o2.broken_mask.any()
    assert np.array_equal(sm, sm[rev]) and np.array_equal(o2.broken_mask, o2.broken_mask[rev])
    zone = np.zeros(w.n, bool)
    zone[w.nofail] = True
    touch = zone[rows] | zone[o2.col]
    assert not (sm[touch] > 0).any() and not o2.broken_mask[touch & ~o.broken_mask].any()


@pytest.mark.parametrize("law", [TRI, BI])
def test_zone_on_a_softened_bond_keeps_its_secant(oracle_lib, law):
    """A bond softened to s_m and then made a no-failure zone (Secs. 5.1, 6, 7: the zones
    keep the loaded and supported nodes' bonds from failing) keeps its damage state as it
    stands: at any later stretch s, unloading, reloading past s_m or stretched far beyond
    s_last, it carries the secant force (envelope(s_m)/s_m) s and neither softens further
    nor breaks.  The expected force is formed here from the law's breakpoints."""
    sb, rb = law
    x = np.array([[0.0, 0.0, 0.0], [L, 0.0, 0.0]])
    rp, col = oracle_lib.family(x, 1.5 * L)
    sim = oracle_lib.OracleSim(x, rp, col, c=C, s0=1.0, rho=RHO, dt=1e-7, vol=V, laws=[law],
                               nofail=np.zeros(2, dtype=np.uint8))
    s_m = 0.5 * (sb[0] + sb[1])                       # on the first softening branch
    f = _pull(sim, [0.5 * s_m, s_m])
    assert f[1] == pytest.approx(_envelope(law, s_m), rel=1e-11)
    secant = _envelope(law, s_m) / s_m
    stored = sim.smax[:2].copy()
    assert stored == pytest.approx([s_m, s_m], rel=1e-11)
    sim.nofail[1] = 1                                 # node 1 joins a zone
    later = [0.25 * s_m, s_m, 1.5 * s_m, 0.5 * (sb[-2] + sb[-1]), 3.0 * sb[-1], 0.5 * s_m]
    for k, s in enumerate(later):
        u = np.zeros((2, 3))
        u[1, 0] = s * L
        fs = sim.force(u=u, k=2 + k)[0, 0] / (C * V)
        assert fs == pytest.approx(secant * s, rel=1e-11), s
    assert not sim.broken[:2].any()
    assert np.all(sim.smax[:2] == stored)             # the stored stretch did not move
    sim.nofail[1] = 0                                 # zone removed: the law applies again
    u = np.zeros((2, 3))
    u[1, 0] = 3.0 * sb[-1] * L
    assert sim.force(u=u, k=10)[0, 0] == 0.0
    assert sim.broken[:2].all()
