"""Pins of the RCB-leaf oracle (Sec. 2.4 RCB split, Sec. 3.1 tree per bin):
hand-worked splits (mass-weighted centre, longest side), the partition and
size properties, and the plane property checked independently."""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import rcb


def _sets(lv):
    return sorted(tuple(sorted(int(i) for i in l)) for l in lv)


def test_hand_worked_mass_weighted_split():
    """Four particles in one cell of a 9-box (cells of 3): x = .1, .2, 1, 2.9.
    Unit masses: centre 1.05 splits {.1,.2,1}|{2.9}, then {.1,.2}|{1} (leaf
    size 2).  A light fourth particle (m = .01) moves the centre to 0.4415:
    {.1,.2}|{1,2.9}."""
    x = np.array([0.1, 0.2, 1.0, 2.9], np.float32)
    y = np.array([1.0, 1.01, 1.02, 1.03], np.float32)
    z = np.full(4, 1.5, np.float32)
    lv = rcb.leaves(x, y, z, np.ones(4), 9.0, 3.0, 2)
    assert _sets(lv) == [(0, 1), (2,), (3,)]
    lv = rcb.leaves(x, y, z, np.array([1, 1, 1, 0.01]), 9.0, 3.0, 2)
    assert _sets(lv) == [(0, 1), (2, 3)]


def test_longest_side_is_cut():
    """Spread along y only: the first cut is perpendicular to y."""
    y = np.array([0.1, 0.5, 2.5, 2.9], np.float32)
    x = np.array([1.0, 1.1, 1.0, 1.1], np.float32)
    z = np.full(4, 1.0, np.float32)
    lv = rcb.leaves(x, y, z, np.ones(4), 9.0, 3.0, 2)
    assert _sets(lv) == [(0, 1), (2, 3)]


def test_point_node_is_a_leaf():
    x = np.full(10, 1.25, np.float32)
    lv = rcb.leaves(x, x, x, np.ones(10), 9.0, 3.0, 3)
    assert _sets(lv) == [tuple(range(10))]


@pytest.mark.parametrize("leaf_max", [1, 7, 64])
def test_partition_sizes_cells_and_planes(leaf_max):
    rng = np.random.default_rng(leaf_max)
    n, L = 3000, 12.0
    x, y, z = (rng.random(n) * L).astype(np.float32), (rng.random(n) * L).astype(np.float32), \
        (rng.random(n) ** 3 * L).astype(np.float32)
    m = rng.uniform(0.5, 2.0, n)
    lv = rcb.leaves(x, y, z, m, L, 3.0, leaf_max)
    allidx = np.concatenate(lv)
    assert np.array_equal(np.sort(allidx), np.arange(n))
    assert max(len(l) for l in lv) <= leaf_max
    _, _, cid = O.bin(x, y, z, L, 3.0)
    for l in lv:
        assert len(set(cid[l].tolist())) == 1
    # every leaf's bounding box meets no other leaf of its cell in its interior
    # along at least one axis (leaves of one cell are separated by planes)
    pos = np.stack([x, y, z], 1).astype(np.float64)
    by_cell = {}
    for l in lv:
        by_cell.setdefault(int(cid[l[0]]), []).append(l)
    for leaves in by_cell.values():
        boxes = [(pos[l].min(0), pos[l].max(0)) for l in leaves]
        for i in range(len(boxes)):
            for j in range(i + 1, len(boxes)):
                lo_i, hi_i = boxes[i]
                lo_j, hi_j = boxes[j]
                assert np.any((hi_i < lo_j) | (hi_j < lo_i) | (hi_i == lo_j) | (hi_j == lo_i))
