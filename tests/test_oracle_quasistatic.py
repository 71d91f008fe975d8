"""Pins of the oracle's quasi-static loading tools: the fifth-order displacement ramp and
no-failure zones (Secs. 5.1, 6 and 7).

The ramp g(tau) = 10 tau^3 - 15 tau^4 + 6 tau^5 is fixed by its boundary behaviour: it
goes from 0 to 1 over [0, T] with zero first and second derivatives at both ends.  The
checks below use properties that any mistake in its coefficients or its derivative
breaks: exact values at tau = 1/2 and tau >= 1, the point symmetry g(tau) + g(1 - tau) = 1,
the peak slope 15/(8T), the cubic/quadratic onset of displacement/velocity, agreement of
g' with a central difference of g, and the exact Euler-Maclaurin sum of the ramp (the
sum of g(k/N) over k = 1..N is (N + 1)/2 for this polynomial, because every odd
derivative that the correction terms need is equal at both ends).
"""
import numpy as np
import pytest

import pd_inputs as pi

RHO, C, V, L = 2400.0, 1.0e20, 1.0e-9, 1.0e-3
SCHED_RAMP5 = pi.SCHED_RAMP5


def _pair(oracle_lib, scheme, dt, ramp_T, kind=pi.BC_DISP, amp=1.0e-5, **kw):
    """Node 0 fixed, node 1 driven in x by the ramp (a constrained component ignores forces)."""
    x = np.array([[0.0, 0.0, 0.0], [L, 0.0, 0.0]])
    rp, col = oracle_lib.family(x, 1.5 * L)
    bcs = [pi.BCSpec(np.array([0]), 0b111, pi.BC_DISP, (0.0, 0.0, 0.0), pi.SCHED_CONST),
           pi.BCSpec(np.array([1]), 0b001, kind, (amp, 0.0, 0.0), SCHED_RAMP5)]
    return oracle_lib.OracleSim(x, rp, col, c=C, s0=10.0, rho=RHO, dt=dt, vol=V, scheme=scheme,
                                bcs=bcs, ramp_T=ramp_T, **kw)


def _trace(sim, nsteps):
    u, v = [0.0], [0.0]
    for _ in range(nsteps):
        sim.run(1)
        u.append(sim.u[1, 0])
        v.append(sim.v[1, 0])
    return np.array(u), np.array(v)


@pytest.mark.parametrize("scheme", ["euler_cromer", "velocity_verlet", "forward_euler"])
def test_ramp_values(oracle_lib, scheme):
    dt, N, A = 1.0e-7, 200, 1.0e-5
    T = N * dt
    u, v = _trace(_pair(oracle_lib, scheme, dt, T, amp=A), N + 20)
    assert u[N // 2] == 0.5 * A                     # g(1/2) = 1/2 exactly
    assert np.all(u[N:] == A)                       # g = 1 from T on
    if scheme != "velocity_verlet":                 # (Verlet reports v one level behind u)
        assert np.all(v[N:] == 0.0)                 # g' = 0 from T on
        assert v[N // 2] == pytest.approx(15.0 / 8.0 * A / T, rel=1e-14)  # peak slope
        assert v.max() == v[N // 2]
        # g' agrees with a central difference of g (error ~ 5 (dt/T)^2 of the peak)
        cd = (u[2:N] - u[: N - 2]) / (2 * dt)
        assert np.abs(cd - v[1: N - 1]).max() <= 2e-4 * v.max()
        # onset: velocity ~ tau^2
        assert v[2] / v[1] == pytest.approx(4.0, rel=0.02)
    # symmetry g(tau) + g(1 - tau) = 1, monotone rise, cubic onset
    k = np.arange(0, N + 1)
    assert np.abs(u[k] + u[N - k] - A).max() <= 4e-15 * A  # a few ulps
    assert np.all(np.diff(u[: N + 1]) >= 0.0)
    assert u[2] / u[1] == pytest.approx(8.0, rel=0.02)


def test_ramp_velocity_kind_exact_sum(oracle_lib):
    """A velocity-controlled component under the ramp: u(N dt) = dt A sum g(k/N) = A (T + dt)/2."""
    dt, N, A = 1.0e-7, 160, 2.0e-2
    T = N * dt
    u, v = _trace(_pair(oracle_lib, "euler_cromer", dt, T, kind=pi.BC_VEL, amp=A), N + 10)
    assert u[N] == pytest.approx(A * (T + dt) / 2.0, rel=1e-13)
    assert np.all(v[N:] == A)
    assert u[N + 10] == pytest.approx(A * (T + dt) / 2.0 + 10 * dt * A, rel=1e-13)


def _block(oracle_lib, dims=(5, 4, 4), s0=1.0e-3, seed=4, **kw):
    x, _ = pi.lattice(dims, 1e-3, 1e-3, seed=seed)
    rp, col = oracle_lib.family(x, 3.015e-3)
    c = pi.pmb_micromodulus(1.4e10, 3.015e-3)
    return x, rp, col, dict(c=c, s0=s0, rho=RHO, dt=1e-8, vol=V, **kw)


def test_nofail_breaks_exactly_the_unflagged_bonds(oracle_lib):
    """Uniform expansion u = lam x stretches every bond by lam > s0: one pass must break
    exactly the bonds with neither end flagged (brute force over the slots)."""
    x, rp, col, kw = _block(oracle_lib)
    n = x.shape[0]
    flag = (np.random.default_rng(11).random(n) < 0.3).astype(np.uint8)
    sim = oracle_lib.OracleSim(x, rp, col, nofail=flag, **kw)
    sim.force(u=2.0 * kw["s0"] * x, k=0)
    want = np.zeros(int(rp[-1]), dtype=bool)
    for i in range(n):
        for b in range(rp[i], rp[i + 1]):
            want[b] = not (flag[i] or flag[col[b]])
    assert want.any() and not want.all()
    assert np.array_equal(sim.broken_mask, want)


def test_nofail_everywhere_is_unbreakable(oracle_lib):
    """Every node flagged: the run equals the same run with an unreachable critical stretch,
    bit for bit, and nothing breaks."""
    x, rp, col, kw = _block(oracle_lib)
    n = x.shape[0]
    bcs = [pi.BCSpec(np.arange(n)[x[:, 0] < 0.5e-3], 0b111, pi.BC_DISP, (0.0, 0.0, 0.0), pi.SCHED_CONST),
           pi.BCSpec(np.arange(n)[x[:, 0] > 3.5e-3], 0b001, pi.BC_DISP, (2.0e-5, 0.0, 0.0), SCHED_RAMP5)]
    a = oracle_lib.OracleSim(x, rp, col, bcs=bcs, ramp_T=2e-6, nofail=np.ones(n, np.uint8), **kw)
    kw_inf = dict(kw, s0=1.0e30)
    b = oracle_lib.OracleSim(x, rp, col, bcs=bcs, ramp_T=2e-6, **kw_inf)
    c = oracle_lib.OracleSim(x, rp, col, bcs=bcs, ramp_T=2e-6, **kw)
    for s in (a, b, c):
        s.run(300)
    assert not a.broken_mask.any()
    assert np.array_equal(a.u, b.u) and np.array_equal(a.v, b.v)
    assert c.broken_mask.any()  # without the zone the same loading breaks bonds


def test_nofail_keeps_bonds_broken_before(oracle_lib):
    """A no-failure zone stops new breaks; bonds broken as an initial condition stay broken."""
    x, rp, col, kw = _block(oracle_lib)
    n = x.shape[0]
    pre = np.zeros(int(rp[-1]), dtype=np.uint8)
    pre[::7] = 1
    sym = pre.copy()  # keep the initial broken set symmetric
    rows = np.repeat(np.arange(n), np.diff(rp))
    for b in np.flatnonzero(pre):
        i, j = rows[b], col[b]
        sym[rp[j] + np.flatnonzero(col[rp[j]:rp[j + 1]] == i)] = 1
    sim = oracle_lib.OracleSim(x, rp, col, nofail=np.ones(n, np.uint8), broken=sym, **kw)
    sim.force(u=2.0 * kw["s0"] * x, k=0)
    assert np.array_equal(sim.broken_mask, sym.astype(bool))
