"""Pins of the oracle's local damage (Sec. 2.2) and break bookkeeping."""
import numpy as np
import pytest

import pd_inputs as pi
from lattice_math import family_offsets, golden

G = golden("lattice_sums.txt")


@pytest.mark.parametrize("m,dims,key", [(3.015, (9, 9, 14), "cut_plane_m3.015"),
                                        (5.015, (11, 11, 22), "cut_plane_m5.015")])
def test_cut_plane_damage_layers(oracle_lib, m, dims, key):
    """A plane cutting every bond: bulk damage at layer d + 1/2 is #{o_z >= d+1} / |H|."""
    x, ijk = pi.lattice(dims, 1e-3)
    rp, col = oracle_lib.family(x, m * 1e-3)
    n = x.shape[0]
    rows = np.repeat(np.arange(n), np.diff(rp))
    h = dims[2] // 2                        # plane between layers h-1 and h
    cut = (ijk[rows, 2] < h) != (ijk[col, 2] < h)
    sim = oracle_lib.OracleSim(x, rp, col, c=1.0, s0=1.0, rho=1.0, dt=1.0, vol=1e-9,
                               broken=cut.astype(np.uint8))
    phi = sim.damage()
    O = family_offsets(m)
    counts = [int(np.sum(O[:, 2] >= d + 1)) for d in range(len(G[key]))]
    assert counts == G[key]
    cx, cy = dims[0] // 2, dims[1] // 2
    for d, cnt in enumerate(counts):
        for z in (h + d, h - 1 - d):
            i = np.nonzero((ijk[:, 0] == cx) & (ijk[:, 1] == cy) & (ijk[:, 2] == z))[0][0]
            assert rp[i + 1] - rp[i] == len(O)
            assert phi[i] == pytest.approx(cnt / len(O), abs=len(O) * 2.3e-16)  # summation rounding


def test_damage_volume_weighted(oracle_lib):
    x = np.array([[0.0, 0, 0], [1.0, 0, 0], [-1.0, 0, 0]])
    rp, col = oracle_lib.family(x, 1.5)
    broken = np.zeros(rp[-1], dtype=np.uint8)
    broken[rp[0] + list(col[rp[0]:rp[1]]).index(1)] = 1     # slot (0 -> 1)
    sim = oracle_lib.OracleSim(x, rp, col, c=1.0, s0=1.0, rho=1.0, dt=1.0,
                               vol=np.array([1.0, 3.0, 1.0]), broken=broken)
    phi = sim.damage()
    assert phi[0] == pytest.approx(3.0 / 4.0, abs=1e-15)
    assert phi[2] == 0.0


def test_block_run_damage_monotone_symmetric(oracle_lib):
    from oracle.oracle import from_workload
    w = pi.workload("block10", steps=1000)
    sim = from_workload(w, record_breaks=True)
    prev = np.zeros(w.n)
    rows = np.repeat(np.arange(w.n), np.diff(sim.row_ptr))
    for _ in range(5):
        sim.run(200)
        phi = sim.damage()
        assert np.all(phi >= prev) and np.all((phi >= 0) & (phi <= 1))
        prev = phi
    mask = sim.broken_mask
    cut = set(zip(rows[mask].tolist(), sim.col[mask].tolist()))
    assert all((j, i) in cut for (i, j) in cut)
    assert mask.sum() > 1000                      # the block fractures
    # a slot's recorded break pass is the same for both directions of the bond
    bs = {(i, j): s for i, j, s in zip(rows[mask], sim.col[mask], sim.break_step[:sim.nnz][mask])}
    assert all(bs[(j, i)] == s for (i, j), s in bs.items())
