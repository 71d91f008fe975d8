"""Pins of the oracle's stiffness corrections (Secs. 2.2, 2.3 and 2.5): the conical micromodulus,
partial volumes and the volume-method surface correction.

Fixed by mathematics rather than by the oracle's own formulas: the continuum integral
that sets the conical peak value for the same bulk stiffness; plane-traction lattice
sums enumerated over integer offsets (not over the oracle's families); the family volume
with partial volumes against the sphere volume it approximates and against an offset
enumeration; the surface correction's identity in the bulk, its symmetry (third law) and
its values from integer neighbour counts on an exact lattice.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import pd_inputs as pi
from lattice_math import family_offsets

DX = 1e-3
M = 3.015


def _sim(oracle_lib, x, m_family, corrections, **kw):
    rp, col = oracle_lib.family(x, m_family * DX)
    args = dict(c=1.0e20, s0=10.0, rho=2400.0, dt=1e-7, vol=DX ** 3, corrections=corrections)
    args.update(kw)
    return oracle_lib.OracleSim(x, rp, col, **args), rp, col


def test_conical_peak_for_equal_bulk_stiffness():
    """c(r) = c0 (1 - r/delta) stores the same dilation energy as the constant c when
    c0 = 5 c: the integrals of c(r) r^3 over the horizon agree."""
    delta = M * DX
    const, _ = integrate.quad(lambda r: r ** 3, 0.0, delta, epsabs=0, epsrel=1e-13)
    con, _ = integrate.quad(lambda r: 5.0 * (1.0 - r / delta) * r ** 3, 0.0, delta, epsabs=0, epsrel=1e-13)
    assert con == pytest.approx(const, rel=1e-12)


def _traction(oracle_lib, corrections, m_family, weight):
    dims = (12, 12, 8)
    x, ijk = pi.lattice(dims, DX)
    eps, c, V = 1e-4, 1e20, DX ** 3
    sim, _, _ = _sim(oracle_lib, x, m_family, corrections, c=c)
    F = sim.force(eps * x, 0)
    got = (V * F[ijk[:, 2] >= 4, 2]).sum()
    want = 0.0
    for o in family_offsets(m_family):
        if o[2] > 0:
            N = (dims[0] - abs(o[0])) * (dims[1] - abs(o[1])) * o[2]
            want -= N * c * weight(np.linalg.norm(o)) * eps * V * V * o[2] / np.linalg.norm(o)
    return got, want


def test_conical_plane_traction_lattice_sum(oracle_lib):
    got, want = _traction(oracle_lib, dict(micro="conical", delta=M * DX), M, lambda r: 1.0 - r / M)
    assert got == pytest.approx(want, rel=1e-10)
    # with c0 = 5c the lattice traction approaches the constant micromodulus's continuum
    # value 3 K eps as the horizon grows (ratio of lattice sum to continuum integral)
    for m, lo, hi in ((3.015, 0.85, 1.15), (6.015, 0.93, 1.07)):
        O = family_offsets(m)
        ratio = 30.0 / (math.pi * m ** 4) * sum((1 - np.linalg.norm(o) / m) * o[2] ** 2 / np.linalg.norm(o)
                                                 for o in O if o[2] > 0)
        assert lo < ratio < hi


def _beta(r, m):
    return np.clip(m + 0.5 - r, 0.0, 1.0)


def test_partial_volume_family_volume_and_traction(oracle_lib):
    """Family radius delta + dx/2 with partial volumes: a bulk node's family volume is the
    offset enumeration of beta, and approximates the sphere volume 4/3 pi delta^3 within
    2.5% where the whole-cell count (122 cells against 114.8) misses by 6%."""
    dims = (12, 12, 12)
    x, ijk = pi.lattice(dims, DX)
    sim, rp, col = _sim(oracle_lib, x, M + 0.5, dict(partial_volumes=True, delta=M * DX, dx=DX))
    centre = np.flatnonzero((ijk == 6).all(1))[0]
    O = family_offsets(M + 0.5)
    want = sum(_beta(np.linalg.norm(o), M) for o in O) * DX ** 3
    assert sim.famvol[centre] == pytest.approx(want, rel=1e-13)
    sphere = 4.0 / 3.0 * math.pi * (M * DX) ** 3
    assert abs(sim.famvol[centre] - sphere) / sphere < 0.025
    assert abs(122 * DX ** 3 - sphere) / sphere > 0.06
    got, want_t = _traction(oracle_lib, dict(partial_volumes=True, delta=M * DX, dx=DX), M + 0.5,
                            lambda r: _beta(r, M))
    assert got == pytest.approx(want_t, rel=1e-10)


def test_surface_correction_bulk_identity_symmetry_and_counts(oracle_lib):
    """On an exact lattice the family volumes are neighbour counts times V: lambda is 1
    between nodes with complete families (their forces are unchanged), symmetric (the
    third law holds), and equals 2 max|H| / (|H_i| + |H_j|) everywhere."""
    dims = (16, 15, 14)
    x, ijk = pi.lattice(dims, DX)
    n = x.shape[0]
    u = np.random.default_rng(5).normal(size=x.shape) * 1e-7
    plain, rp, col = _sim(oracle_lib, x, M, None)
    corr, _, _ = _sim(oracle_lib, x, M, dict(surface=True))
    F0, F1 = plain.force(u, 0), corr.force(u, 0)
    counts = np.diff(rp)
    full = counts == counts.max()
    rows = np.repeat(np.arange(n), counts)
    interior = np.array([full[col[rp[i]:rp[i + 1]]].all() for i in range(n)]) & full
    assert interior.sum() > 10
    assert np.array_equal(F1[interior], F0[interior])
    # third law: sum of V F vanishes with the symmetric correction
    scale = np.abs(F1).sum()
    assert np.abs(F1.sum(0)).max() <= 1e-12 * scale
    # lambda from integer neighbour counts, as a per-slot stiffness on the uncorrected model
    lam = 2.0 * counts.max() / (counts[rows] + counts[col])
    ref, _, _ = _sim(oracle_lib, x, M, None, kslot=1.0e20 * lam)
    assert np.allclose(ref.force(u, 0), F1, rtol=0, atol=1e-14 * np.abs(F1).max())
    assert lam.max() > 1.5 and lam.min() == 1.0
