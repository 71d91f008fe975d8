"""Pins of the oracle's bond force, breaking rule and node sum.

Each check is fixed by mathematics, not by the oracle's own formula: rigid motions,
the energy the force derives from (complex-step derivative of the micropotential
sum), Newton's third law, and closed-form lattice sums under affine stretches.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import pd_inputs as pi
from lattice_math import family_offsets

DX = 1e-3


def _sim(oracle_lib, x, m, **kw):
    rp, col = oracle_lib.family(x, m * DX)
    args = dict(c=1.0e20, s0=10.0, rho=2400.0, dt=1e-7, vol=DX ** 3)
    args.update(kw)
    return oracle_lib.OracleSim(x, rp, col, **args)


def test_micromodulus_matches_continuum_dilation_energy():
    """c = 18K/(pi delta^4) makes the bulk PD energy under dilation eps equal 9/2 K eps^2."""
    K, delta, eps = 1.4e10, 3.015e-3, 1e-4
    c = pi.pmb_micromodulus(K, delta)
    # W = 1/2 int_H w dV, w = c s^2 |xi| / 2, s = eps for every bond
    I, _ = integrate.quad(lambda r: 4.0 * math.pi * r * r * r, 0.0, delta, epsabs=0, epsrel=1e-13)
    W = 0.5 * (0.5 * c * eps * eps) * I
    assert W == pytest.approx(4.5 * K * eps * eps, rel=1e-12)


def test_rigid_translation_gives_zero_force_bitwise(oracle_lib):
    x, _ = pi.lattice((6, 6, 6), DX, 1e-3, seed=2)
    sim = _sim(oracle_lib, x, 3.015)
    u = np.tile(np.array([3e-6, -1e-6, 2.5e-6]), (x.shape[0], 1))
    F = sim.force(u, 0)
    assert np.all(F == 0.0)


def test_finite_rigid_rotation_gives_negligible_force(oracle_lib):
    x, _ = pi.lattice((6, 6, 6), DX, 1e-3, seed=2)
    sim = _sim(oracle_lib, x, 3.015, c=1e20, s0=1e-3)
    a = 0.3
    R = np.array([[math.cos(a), -math.sin(a), 0.0], [math.sin(a), math.cos(a), 0.0], [0, 0, 1.0]])
    xc = x - x.mean(0)
    u = xc @ R.T - xc
    F = sim.force(u, 0)
    bound = 1e-12 * 1e20 * 1e-3 * DX ** 3 * 122
    assert np.abs(F).max() <= bound
    assert not sim.broken_mask.any()


def _energy(x, rows, cols, k, vol, u):
    """Total bond energy sum_b 1/4 k_b s_b^2 |xi_b| V_i V_j (micropotential w = c s^2 |xi| / 2)."""
    xi = x[cols] - x[rows]
    y = xi + (u[cols] - u[rows])
    r = np.sqrt((y * y).sum(1))
    L = np.sqrt((xi * xi).sum(1))
    s = (r - L) / L
    return np.sum(0.25 * k * s * s * L * vol[rows] * vol[cols])


def test_force_is_minus_energy_gradient_complex_step(oracle_lib):
    """F_i = -(1/V_i) dE/du_i, with non-uniform volumes and a symmetric stiffness field."""
    x, _ = pi.lattice((4, 4, 3), DX, 0.2, seed=4)
    n = x.shape[0]
    rng = np.random.default_rng(7)
    vol = DX ** 3 * rng.uniform(0.5, 1.5, n)
    rp, col = oracle_lib.family(x, 2.2 * DX)
    rows = np.repeat(np.arange(n), np.diff(rp))
    g = rng.normal(size=n) * 0.3
    k = 1e20 * np.exp(0.5 * (g[rows] + g[col]))
    u = rng.normal(size=(n, 3)) * 1e-6
    sim = oracle_lib.OracleSim(x, rp, col, c=0.0, s0=10.0, rho=1.0, dt=1.0, vol=vol, kslot=k)
    F = sim.force(u, 0)
    h = 1e-30
    grad = np.zeros((n, 3))
    for i in range(n):
        for d in range(3):
            up = u.astype(complex)
            up[i, d] += 1j * h
            grad[i, d] = _energy(x, rows, col, k, vol, up).imag / h
    want = -grad / vol[:, None]
    scale = np.abs(want).max()
    assert np.abs(F - want).max() <= 1e-11 * scale


def test_third_law_and_torque_balance(oracle_lib):
    x, _ = pi.lattice((7, 6, 5), DX, 1e-3, seed=3)
    n = x.shape[0]
    rng = np.random.default_rng(1)
    vol = DX ** 3 * rng.uniform(0.8, 1.2, n)
    rp, col = oracle_lib.family(x, 3.015 * DX)
    rows = np.repeat(np.arange(n), np.diff(rp))
    g = rng.normal(size=n) * 0.2
    k = 1e20 * np.exp(0.5 * (g[rows] + g[col]))
    sim = oracle_lib.OracleSim(x, rp, col, c=0.0, s0=10.0, rho=1.0, dt=1.0, vol=vol, kslot=k)
    u = rng.normal(size=(n, 3)) * 1e-6
    F = sim.force(u, 0)
    VF = vol[:, None] * F
    assert np.abs(VF.sum(0)).max() <= 1e-12 * np.abs(VF).sum()
    p = x + u
    torque = np.cross(p, VF).sum(0)
    assert np.abs(torque).max() <= 1e-12 * (np.linalg.norm(p, axis=1)[:, None] * np.abs(VF)).sum()


def test_isotropic_dilation_closed_form(oracle_lib):
    """u = eps (x - x0) stretches every bond by exactly eps: F_i = c eps V sum_j o_ij/|o_ij|."""
    dims = (6, 7, 5)
    x, ijk = pi.lattice(dims, DX)
    eps, c = 1e-4, 1e20
    sim = _sim(oracle_lib, x, 3.015, c=c)
    u = eps * (x - x.mean(0))
    F = sim.force(u, 0)
    want = np.zeros_like(F)
    O = family_offsets(3.015)
    unit = O / np.linalg.norm(O, axis=1)[:, None]
    for i in range(x.shape[0]):
        nb = ijk[i] + O
        ok = np.all((nb >= 0) & (nb < np.array(dims)), axis=1)
        want[i] = c * eps * DX ** 3 * unit[ok].sum(0)
    scale = c * eps * DX ** 3 * len(O)
    assert np.abs(F - want).max() <= 1e-9 * scale
    # bulk nodes feel nothing; surface nodes are pulled inwards
    assert np.abs(F).max() > 1e-3 * scale


def test_uniaxial_stretch_closed_form(oracle_lib):
    """u_z = eps z: a bond of direction n has s = sqrt(1 + (2 eps + eps^2) n_z^2) - 1."""
    dims = (5, 5, 6)
    x, ijk = pi.lattice(dims, DX)
    eps, c = 2e-4, 1e20
    sim = _sim(oracle_lib, x, 3.015, c=c)
    u = np.zeros_like(x)
    u[:, 2] = eps * x[:, 2]
    F = sim.force(u, 0)
    O = family_offsets(3.015)
    nz = O[:, 2] / np.linalg.norm(O, axis=1)
    s = np.sqrt(1.0 + (2 * eps + eps * eps) * nz * nz) - 1.0
    ydir = O * np.array([1.0, 1.0, 1.0 + eps])
    ydir = ydir / np.linalg.norm(ydir, axis=1)[:, None]
    want = np.zeros_like(F)
    for i in range(x.shape[0]):
        nb = ijk[i] + O
        ok = np.all((nb >= 0) & (nb < np.array(dims)), axis=1)
        want[i] = c * DX ** 3 * (s[ok, None] * ydir[ok]).sum(0)
    scale = c * eps * DX ** 3 * len(O)
    assert np.abs(F - want).max() <= 1e-8 * scale


def test_plane_traction_lattice_sum(oracle_lib):
    """Resultant on the upper half of a dilated block = exact sum over bonds crossing the plane."""
    dims = (12, 12, 8)
    x, ijk = pi.lattice(dims, DX)
    eps, c, V = 1e-4, 1e20, DX ** 3
    sim = _sim(oracle_lib, x, 3.015, c=c)
    F = sim.force(eps * x, 0)
    upper = ijk[:, 2] >= 4
    got = (V * F[upper, 2]).sum()
    O = family_offsets(3.015)
    want = 0.0
    for o in O:
        if o[2] > 0:
            N = (dims[0] - abs(o[0])) * (dims[1] - abs(o[1])) * o[2]
            want -= N * c * eps * V * V * o[2] / np.linalg.norm(o)
    assert got == pytest.approx(want, rel=1e-10)
    # the infinite-plane sum against continuum hydrostatic stress 3 K eps: ratio of the
    # lattice sum to the continuum integral, a discretisation constant near 1.0987
    m = 3.015
    ratio = 6.0 / (math.pi * m ** 4) * sum(o[2] ** 2 / np.linalg.norm(o) for o in O if o[2] > 0)
    assert ratio == pytest.approx(1.0987, abs=2e-4)


def test_break_rule_threshold_and_same_pass_zero(oracle_lib):
    """s >= s0 breaks (tie included) and the bond gives no force in that pass; compression never breaks."""
    x = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0]])
    rp, col = oracle_lib.family(x, 1.5)
    for s0, u1, broke in [(0.5, 0.5, True), (0.5 + 1e-12, 0.5, False), (0.5, -0.75, False)]:
        sim = oracle_lib.OracleSim(x, rp, col, c=2.0, s0=s0, rho=1.0, dt=1.0, vol=1.0,
                                   record_breaks=True)
        u = np.array([[0.0, 0.0, 0.0], [u1, 0.0, 0.0]])
        F = sim.force(u, 7)
        assert sim.broken_mask.all() == broke and sim.broken_mask.any() == broke
        if broke:
            assert np.all(F == 0.0)
            assert np.all(sim.break_step[:2] == 7)
        else:
            s = u1  # exact: r = 1 + u1, L = 1
            assert F[1, 0] == pytest.approx(-2.0 * s, rel=1e-15)
            assert F[0, 0] == -F[1, 0]
        # irreversible: compressing the bond afterwards does not restore it
        F2 = sim.force(np.array([[0.0, 0.0, 0.0], [-0.25, 0.0, 0.0]]), 8)
        assert np.all(F2 == 0.0) == broke


def test_body_force_added(oracle_lib):
    x, _ = pi.lattice((3, 3, 3), DX)
    n = x.shape[0]
    bhat = np.random.default_rng(0).normal(size=(n, 3))
    sim = _sim(oracle_lib, x, 1.5, bhat=bhat, bmag=3.5e8)
    F = sim.force(np.zeros((n, 3)), 0)
    assert np.array_equal(F, 3.5e8 * bhat)
