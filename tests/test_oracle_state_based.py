"""Pins of the oracle's ordinary state-based linear solid (Sec. 8.2): weighted volume,
dilation, scalar force state and the two-pass force.

Fixed by mathematics rather than by the oracle's formulas: the force of a single bond in
closed form (the shear modulus drops out); the dilation of a uniform expansion (exactly 3
lambda at every node, surface nodes and uneven volumes included) and of a small linear
strain (its trace, at nodes whose family has the lattice's cubic symmetry); invariance
under a rigid motion; the force as the negative gradient of the model's elastic energy
(finite differences of an energy written here from the energy density, not from the
force), and that energy against classical elasticity (bulk part exact, shear part
converging with the horizon to the continuum value through a sphere average); balance of
linear momentum with bonds breaking; irreversible, symmetric breaking at s0 and no
breaking in no-failure zones.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import pd_inputs as pi
from lattice_math import family_offsets

DX = 1.0e-3
M = 3.015
K = 1.4e10
G = pi.shear_modulus(K, 0.2)


def _sim(oracle_lib, x, vol, *, s0=np.inf, K=K, G=G, m=M, **kw):
    rp, col = oracle_lib.family(x, m * DX)
    return oracle_lib.OracleSim(x, rp, col, c=0.0, s0=s0, rho=2400.0, dt=1e-7, vol=vol,
                                state_based=(K, G), **kw), rp, col


def _energy(x, u, rp, col, vol, K, G):
    """Elastic energy sum_i V_i W_i of the linear solid: W_i = K theta_i^2 / 2 +
    (15 G / 2 m_i) sum_j (e^d_ij)^2 V_j with e^d = e - theta |xi| / 3 (influence 1)."""
    n = x.shape[0]
    rows = np.repeat(np.arange(n), np.diff(rp))
    cols = col.astype(np.int64)
    xi = x[cols] - x[rows]
    L = np.linalg.norm(xi, axis=1)
    e = np.linalg.norm(xi + u[cols] - u[rows], axis=1) - L
    vj = vol[cols]
    m = np.bincount(rows, L * L * vj, minlength=n)
    theta = 3.0 / m * np.bincount(rows, L * e * vj, minlength=n)
    ed = e - theta[rows] * L / 3.0
    W = 0.5 * K * theta ** 2 + 15.0 * G / (2.0 * m) * np.bincount(rows, ed * ed * vj, minlength=n)
    return float((vol * W).sum())


def test_single_bond_closed_form(oracle_lib):
    """Two nodes: m_0 = L^2 V_1, theta_0 = 3 e / L, the deviatoric extension vanishes, and
    F_0 = 9 K e / L^2 (1 + V_1 / V_0) along the bond, whatever G is."""
    L = 0.9 * DX
    x = np.array([[0.0, 0.0, 0.0], [L * 0.6, L * 0.0, L * 0.8]])
    vol = np.array([1.0e-9, 1.7e-9])
    u = np.array([[1e-7, -2e-7, 0.5e-7], [4e-7, 1e-7, -3e-7]])
    y = x[1] + u[1] - x[0] - u[0]
    e = np.linalg.norm(y) - L
    want = 9.0 * K * e / L ** 2 * (1.0 + vol[1] / vol[0]) * y / np.linalg.norm(y)
    for g in (0.0, G, 5.0 * G):
        sim, _, _ = _sim(oracle_lib, x, vol, G=g)
        F = sim.force(u, 0)
        assert np.allclose(F[0], want, rtol=1e-9, atol=0)
        assert np.allclose(F[1] * vol[1], -F[0] * vol[0], rtol=1e-12, atol=0)
        assert sim.theta[0] == pytest.approx(3.0 * e / L, rel=1e-9)


def test_uniform_expansion_dilation_is_three_lambda(oracle_lib):
    """u = lambda x stretches every bond by lambda, so theta_i = 3 lambda at every node
    (any family, any volumes); bulk nodes of an exact lattice feel no force."""
    lam = 1.0e-3
    x, ijk = pi.lattice((9, 8, 8), DX, 1e-2, seed=3)
    vol = DX ** 3 * (1.0 + 0.3 * pi.uniform01(9, np.arange(x.shape[0], dtype=np.uint64)))
    sim, _, _ = _sim(oracle_lib, x, vol)
    sim.force(lam * x, 0)
    assert np.allclose(sim.theta, 3.0 * lam, rtol=1e-12, atol=0)
    xe, ijk = pi.lattice((16, 16, 16), DX)
    sim, rp, col = _sim(oracle_lib, xe, DX ** 3)
    F = sim.force(lam * xe, 0)
    full = np.diff(rp) == np.diff(rp).max()
    inner = full & np.array([full[col[rp[i]:rp[i + 1]]].all() for i in range(xe.shape[0])])
    assert inner.sum() > 8
    scale = 9.0 * K * lam / DX  # one bond's force density scale
    assert np.abs(F[inner]).max() <= 1e-9 * scale
    assert np.abs(F[~full]).max() > 1e-2 * scale


def test_linear_strain_dilation_is_the_trace(oracle_lib):
    """For a small strain eps the dilation of a node with a complete (cubic-symmetric)
    family is tr(eps) up to second order: the family's second moment is isotropic."""
    x, ijk = pi.lattice((12, 12, 12), DX)
    rng = np.random.default_rng(11)
    A = rng.normal(size=(3, 3)) * 1e-7
    eps = 0.5 * (A + A.T)
    sim, rp, col = _sim(oracle_lib, x, DX ** 3)
    sim.force(x @ eps.T, 0)
    full = np.diff(rp) == np.diff(rp).max()
    assert np.allclose(sim.theta[full], np.trace(eps), rtol=1e-5, atol=1e-6 * np.abs(eps).max())


def test_rigid_motion_gives_no_force(oracle_lib):
    x, _ = pi.lattice((7, 6, 6), DX, 1e-2, seed=4)
    a = 0.3
    R = np.array([[math.cos(a), -math.sin(a), 0.0], [math.sin(a), math.cos(a), 0.0], [0.0, 0.0, 1.0]])
    u = x @ R.T - x + np.array([2e-4, -1e-4, 3e-4])
    sim, _, _ = _sim(oracle_lib, x, DX ** 3)
    F = sim.force(u, 0)
    assert np.abs(sim.theta).max() < 1e-12
    assert np.abs(F).max() <= 1e-9 * 9.0 * K * 1e-3 / DX


@pytest.mark.parametrize("g", [0.0, G])
def test_force_is_the_energy_gradient(oracle_lib, g):
    """V_i F_i = -dE/du_i by central differences of the energy, on a jittered block with
    uneven volumes (the t_ji term and the placement of V_i, V_j included)."""
    x, _ = pi.lattice((5, 5, 4), DX, 5e-2, seed=8)
    n = x.shape[0]
    vol = DX ** 3 * (1.0 + 0.4 * pi.uniform01(21, np.arange(n, dtype=np.uint64)))
    u = np.random.default_rng(2).normal(size=(n, 3)) * 1e-6
    sim, rp, col = _sim(oracle_lib, x, vol, G=g)
    F = sim.force(u, 0)
    h = 1e-10
    for i in (0, 7, 31, 55, n - 1):
        for d in range(3):
            up, um = u.copy(), u.copy()
            up[i, d] += h
            um[i, d] -= h
            dE = (_energy(x, up, rp, col, vol, K, g) - _energy(x, um, rp, col, vol, K, g)) / (2 * h)
            assert -dE / vol[i] == pytest.approx(F[i, d], rel=2e-6, abs=2e-7 * np.abs(F).max())


def test_energy_against_classical_elasticity():
    """The energy of a homogeneous strain at a node with a complete family: the bulk part
    K (tr eps)^2 / 2 exactly; the shear part of a pure shear (eps_xy = g/2) tends to the
    classical G g^2 / 2 as the horizon grows, the continuum limit being the sphere average
    <n_x^2 n_y^2> = 1/15."""
    avg, _ = integrate.dblquad(lambda t, p: (math.sin(t) * math.cos(p)) ** 2 * (math.sin(t) * math.sin(p)) ** 2
                               * math.sin(t), 0.0, 2 * math.pi, 0.0, math.pi)
    assert avg / (4 * math.pi) == pytest.approx(1.0 / 15.0, rel=1e-10)
    for m, tol in ((3.015, 0.15), (6.015, 0.05), (9.015, 0.02)):
        O = family_offsets(m).astype(float)
        r2 = (O ** 2).sum(1)
        # e = g o_x o_y / |o|, theta = 0: W / (G g^2 / 2) = 15 / m sum (o_x o_y)^2 / |o|^2
        ratio = 15.0 / r2.sum() * ((O[:, 0] * O[:, 1]) ** 2 / r2).sum()
        assert abs(ratio - 1.0) < tol, (m, ratio)


def test_breaking_symmetric_irreversible_and_momentum(oracle_lib):
    """A pulled block breaks bonds at s0 on both slots in the same pass, never heals, and
    the internal forces balance (sum V_i F_i = 0) with broken bonds present; no-failure
    nodes keep every bond."""
    w = pi.workload("block10", dims=(9, 7, 7), steps=600, model="state_based")
    from oracle.oracle import from_workload
    o = from_workload(w)
    rows = np.repeat(np.arange(w.n), np.diff(o.row_ptr))
    order = np.lexsort((rows, o.col))
    rev = np.empty(o.nnz, dtype=np.int64)
    rev[np.lexsort((o.col, rows))] = order
    prev = o.broken_mask.copy()
    for _ in range(3):
        o.run(200)
        b = o.broken_mask
        assert np.all(b >= prev) and np.array_equal(b, b[rev])
        prev = b.copy()
    assert b.sum() > 50
    F = o.force(o.u, o.step)
    Vf = (w.volume * F).sum(0)
    assert np.abs(Vf).max() <= 1e-12 * np.abs(w.volume * F).sum()
    # no-failure zone: the same run with the top layers flagged keeps their bonds
    top = np.flatnonzero(w.ijk[:, 2] >= w.dims[2] - 3)
    flags = np.zeros(w.n, np.uint8)
    flags[top] = 1
    o2 = oracle_lib.OracleSim(w.coords, o.row_ptr, o.col, c=0.0, s0=w.s0, rho=w.rho, dt=w.dt, vol=w.volume,
                              bcs=w.bcs, nofail=flags, state_based=w.state_based)
    o2.run(600)
    touch = flags[rows].astype(bool) | flags[o.col].astype(bool)
    assert not o2.broken_mask[touch].any() and o2.broken_mask.any()


def test_single_bond_breaks_at_s0(oracle_lib):
    L = DX
    x = np.array([[0.0, 0.0, 0.0], [L, 0.0, 0.0]])
    s0 = 1e-3
    for s, broken in ((0.999 * s0, False), (1.001 * s0, True)):
        sim, _, _ = _sim(oracle_lib, x, DX ** 3, s0=s0)
        u = np.array([[0.0, 0.0, 0.0], [s * L, 0.0, 0.0]])
        F = sim.force(u, 0)
        assert sim.broken_mask.all() == broken and sim.broken_mask.any() == broken
        assert (np.abs(F).max() == 0.0) == broken
        if broken:  # irreversible: released, the bond stays broken
            assert np.abs(sim.force(0 * u, 1)).max() == 0.0 and sim.broken_mask.all()


def test_workload_moduli():
    """Isotropic elasticity: G = 3K(1 - 2 nu)/(2(1 + nu)); at nu = 1/4 (the PMB's fixed
    Poisson ratio) G = 3K/5, and E = 9KG/(3K + G) returns 2G(1 + nu)."""
    assert pi.shear_modulus(K, 0.25) == pytest.approx(0.6 * K, rel=1e-15)
    for nu in (0.1, 0.2, 0.3, 0.45):
        g = pi.shear_modulus(K, nu)
        assert 9 * K * g / (3 * K + g) == pytest.approx(2 * g * (1 + nu), rel=1e-13)
    w = pi.workload("block10", dims=(5, 5, 5), steps=10, model="state_based", poisson=0.3)
    assert w.state_based == (pi.K_CONCRETE, pi.shear_modulus(pi.K_CONCRETE, 0.3))
    assert pi.workload("block10", dims=(5, 5, 5), steps=10).state_based is None
    with pytest.raises(KeyError):
        pi.workload("block10", model="cubic")
