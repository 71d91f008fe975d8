"""Pins of the oracle's family search (Eq. family, self excluded) to lattice counts."""
import numpy as np
import pytest

import pd_inputs as pi
from lattice_math import family_offsets, golden, slot_count

G = golden("lattice_sums.txt")


def test_bulk_family_sizes_are_lattice_counts():
    assert len(family_offsets(3.015)) == G["bulk_family_m3.015"]
    assert len(family_offsets(5.015)) == G["bulk_family_m5.015"]


@pytest.mark.parametrize("m,dims", [(3.015, (9, 9, 9)), (5.015, (13, 13, 13))])
def test_oracle_bulk_family(oracle_lib, m, dims):
    x, ijk = pi.lattice(dims, 1e-3, 1e-3, seed=5)
    rp, col = oracle_lib.family(x, m * 1e-3)
    centre = np.nonzero((ijk == np.array(dims) // 2).all(axis=1))[0][0]
    assert rp[centre + 1] - rp[centre] == len(family_offsets(m))
    # the centre's neighbours are exactly the lattice offsets
    offs = ijk[col[rp[centre]:rp[centre + 1]]] - ijk[centre]
    want = {tuple(o) for o in family_offsets(m)}
    assert {tuple(o) for o in offs} == want


@pytest.mark.parametrize("dims,key", [((10, 10, 10), "slots_10x10x10_m3.015"),
                                      ((100, 25, 20), "slots_100x25x20_m3.015")])
def test_oracle_slot_counts(oracle_lib, dims, key):
    assert slot_count(dims, 3.015) == G[key]
    x, _ = pi.lattice(dims, 1e-3, 1e-3, seed=1234)
    rp, col = oracle_lib.family(x, 3.015e-3)
    assert rp[-1] == G[key]


@pytest.mark.parametrize("jitter,m", [(0.0, 2.5), (1e-3, 3.015), (0.2, 2.0)])
def test_brute_force_equals_cell_list(oracle_lib, jitter, m):
    x, _ = pi.lattice((6, 5, 7), 1e-3, jitter, seed=11)
    a = oracle_lib.family(x, m * 1e-3, "brute")
    b = oracle_lib.family(x, m * 1e-3, "cells")
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_family_random_cloud_matches_distance_matrix(oracle_lib):
    rng = np.random.default_rng(3)
    x = rng.uniform(0.0, 1.0, size=(300, 3))
    delta = 0.17
    rp, col = oracle_lib.family(x, delta)
    d = np.sqrt(((x[:, None, :] - x[None, :, :]) ** 2).sum(-1))
    for i in range(x.shape[0]):
        want = np.nonzero((d[i] <= delta) & (np.arange(x.shape[0]) != i))[0]
        assert np.array_equal(col[rp[i]:rp[i + 1]], want)


def test_family_symmetric_sorted_no_self(oracle_lib):
    x, _ = pi.lattice((7, 6, 5), 1e-3, 1e-3, seed=9)
    rp, col = oracle_lib.family(x, 3.015e-3)
    n = x.shape[0]
    pairs = set()
    for i in range(n):
        row = col[rp[i]:rp[i + 1]]
        assert np.all(np.diff(row) > 0)
        assert i not in set(row.tolist())
        pairs.update((i, int(j)) for j in row)
    assert all((j, i) in pairs for (i, j) in pairs)


def test_notch_count():
    """The notch removes exactly the integer-test count of undirected bonds."""
    dims = (200, 25, 25)
    ijk = pi.lattice_index(dims)
    O = family_offsets(3.015)
    # enumerate pairs by offset instead of building a family: independent of the oracle
    plane2, h2 = 199, 9
    count = 0
    for o in O:
        if o[0] <= 0:
            continue  # count each undirected bond once (o_x > 0 crosses from left to right)
        xs = np.arange(dims[0])
        xi = xs[(2 * xs - plane2 < 0) & (2 * (xs + o[0]) - plane2 > 0)]
        for x0 in xi:
            zi = np.arange(max(0, -o[2]), min(dims[2], dims[2] - o[2]))
            d = 2 * o[0]
            lhs = 2 * zi * d + 2 * o[2] * (plane2 - 2 * x0) - h2 * d
            ny = dims[1] - abs(o[1])
            count += int(np.sum(lhs < 0)) * ny
    assert count == G["notch_undirected_200x25x25"]


def test_notch_mask_generator_matches_count(oracle_lib):
    w = pi.workload("beam3pb")
    rp, col = oracle_lib.family(w.coords, w.horizon)
    assert rp[-1] == G["slots_200x25x25_m3.015"]
    mask = pi.notch_mask(w.ijk, rp, col, *w.notch)
    assert int(mask.sum()) == 2 * G["notch_undirected_200x25x25"]
    # symmetric: slot (i, j) cut iff (j, i) cut
    rows = np.repeat(np.arange(w.n), np.diff(rp))
    cut = set(zip(rows[mask == 1].tolist(), col[mask == 1].tolist()))
    assert all((j, i) in cut for (i, j) in cut)
