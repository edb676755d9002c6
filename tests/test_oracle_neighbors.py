"""Pins of the oracle neighbour list: an independent pure-Python enumeration
over a wide image window, exact pair symmetry, multi-image rows of small
cells, non-periodic axes and the expected mean neighbour count."""
import itertools
import math

import numpy as np
import pytest

from oracle import brute_force_neighbors
from workloads import make_batch, make_workload


def _naive(pos32, cell, pbc, rc32, window=3):
    """Every j and every image S in a fixed wide window, scalar Python floats
    (IEEE double, one rounding per operation)."""
    rc = float(np.float32(rc32))
    rc2 = rc * rc
    x = [[float(v) for v in p] for p in pos32]
    h = [[float(v) for v in row] for row in cell]
    rngs = [range(-window, window + 1) if pbc[k] else range(0, 1) for k in range(3)]
    out = []
    for i in range(len(x)):
        for j in range(len(x)):
            for S in itertools.product(*rngs):
                if i == j and S == (0, 0, 0):
                    continue
                d = [(x[j][c] - x[i][c]) + ((S[0] * h[0][c] + S[1] * h[1][c]) + S[2] * h[2][c]) for c in range(3)]
                d2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
                if 0.0 < d2 < rc2:
                    out.append((i, j) + tuple(S))
    return sorted(out)


def _triples(nl):
    return [tuple(int(v) for v in (a, b, *s)) for a, b, s in zip(nl.i, nl.j, nl.S)]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_matches_naive_enumeration_small_triclinic(seed):
    rng = np.random.default_rng(seed)
    n = 7
    cell = np.array([[4.1, 0.0, 0.0], [1.3, 3.7, 0.0], [-0.6, 0.9, 4.4]])
    frac = rng.random((n, 3)) * 1.6 - 0.3          # some atoms outside the cell
    pos = (frac @ cell).astype(np.float32)
    b = make_batch([(pos, np.zeros(n, np.int32), cell, (1, 1, 1))])
    nl = brute_force_neighbors(b, 3.5)
    ref = _naive(pos, cell, (1, 1, 1), 3.5, window=3)
    assert _triples(nl) == ref                      # same set, canonical order


def test_mixed_periodicity_matches_naive():
    rng = np.random.default_rng(5)
    cell = np.diag([5.0, 6.0, 30.0])
    pos = (rng.random((9, 3)) * [5.0, 6.0, 8.0]).astype(np.float32)
    b = make_batch([(pos, np.zeros(9, np.int32), cell, (1, 1, 0))])
    nl = brute_force_neighbors(b, 4.0)
    assert _triples(nl) == _naive(pos, cell, (1, 1, 0), 4.0, window=3)
    assert np.all(nl.S[:, 2] == 0)


def test_pair_symmetry_and_multi_image_rows():
    b, _, spec = make_workload("tiny")
    nl = brute_force_neighbors(b, spec.model.r_cut)
    s = set(_triples(nl))
    assert all((j, i, -a, -bb, -c) in s for (i, j, a, bb, c) in s)
    # the 8 A box is narrower than 2 r_c: some rows hold two images of one atom
    ij = list(zip(nl.i.tolist(), nl.j.tolist()))
    assert len(ij) > len(set(ij))
    # self images appear (|S| = 1 images of the atom itself are 8 A away: no);
    # rows are canonical
    for i in range(b.n_atoms):
        m = nl.i == i
        keys = list(zip(nl.j[m], nl.S[m, 0], nl.S[m, 1], nl.S[m, 2]))
        assert keys == sorted(keys)


def test_self_images_in_tiny_cell():
    cell = np.eye(3) * 2.5
    b = make_batch([(np.zeros((1, 3), np.float32), np.zeros(1, np.int32), cell, (1, 1, 1))])
    nl = brute_force_neighbors(b, 3.0)
    # images at 2.5 (6 of them); sqrt(2)*2.5 = 3.54 is outside
    assert nl.n_pairs == 6
    assert np.all(nl.j == 0)
    assert sorted(map(tuple, nl.S.tolist())) == sorted(
        [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)])


def test_coincident_atoms_reported():
    pos = np.array([[1.0, 1.0, 1.0], [1.0, 1.0, 1.0], [2.0, 1.0, 1.0]], np.float32)
    b = make_batch([(pos, np.zeros(3, np.int32), np.eye(3) * 20.0, (0, 0, 0))])
    nl = brute_force_neighbors(b, 3.0)
    assert nl.coincident == 2
    assert not np.any((nl.i == 0) & (nl.j == 1))


def test_mean_neighbour_count_matches_density():
    b, _, spec = make_workload("liquid", n=400, sweeps=2)
    rows = np.arange(0, 400, 4)
    nl = brute_force_neighbors(b, 5.0, rows=rows)
    L = b.cell[0, 0, 0]
    expected = 400 / L ** 3 * 4.0 / 3.0 * math.pi * 125.0
    assert abs(nl.n_pairs / len(rows) - expected) < 0.1 * expected


def test_rows_subset_equals_full_list_restricted():
    b, _, _ = make_workload("tiny")
    full = brute_force_neighbors(b, 5.0)
    rows = np.array([3, 17, 40])
    sub = brute_force_neighbors(b, 5.0, rows=rows)
    m = np.isin(full.i, rows)
    assert np.array_equal(full.i[m], sub.i) and np.array_equal(full.j[m], sub.j)
    assert np.array_equal(full.S[m], sub.S)
