"""Pins for the oracle's non-recursive views of Construct (Alg. 1), which the
full-size GPU tests use where the recursive build would take too long:

- build_splits: T and the representatives of Construct's recursion alone,
  equal to the full build's on every test cloud and axis sequence;
- leaf_cells: every leaf's closed cell from T alone, equal to the cells the
  recursion carries down, and to the hand-worked 5-point tree;
- afford_direct: the affordance set by its direct definition (Lemma 1,
  case 1), sandwiched in exact rational arithmetic between the points within
  r_max of the cell and those within r_max (1 + 2^-20), and equal to the
  unpruned recursive build's sets.
"""
from fractions import Fraction

import numpy as np
import pytest

from conftest import fnum, golden
from test_oracle_tree import CLOUDS, _exact_cell_dist2

AXES = {"cyclic": None, "x-only": [0] * 30, "z-y": [2, 1] * 15, "random": list(np.random.default_rng(3).integers(0, 3, 30))}


@pytest.mark.parametrize("axes", sorted(AXES))
@pytest.mark.parametrize("name", sorted(CLOUDS))
def test_build_splits_equal_construct(orc, name, axes):
    pts = CLOUDS[name]
    ax = AXES[axes]
    t = orc.build_tree(pts, 0.01, 0.05, axes=ax)
    T, rep = orc.build_splits(pts, axes=ax)
    assert T.tobytes() == t.T.tobytes()
    assert np.array_equal(rep, t.rep)


@pytest.mark.parametrize("axes", sorted(AXES))
@pytest.mark.parametrize("name", sorted(CLOUDS))
def test_leaf_cells_equal_construct(orc, name, axes):
    pts = CLOUDS[name]
    ax = AXES[axes]
    t = orc.build_tree(pts, 0.01, 0.05, axes=ax)
    cells = orc.leaf_cells(t.N, t.D, t.T, axes=ax)
    assert cells.tobytes() == t.cell.tobytes()


def test_leaf_cells_hand_worked_tree(orc):
    g = golden("tiny_tree.json")
    T = np.array([fnum(v) for v in g["T"]], dtype=np.float32)
    cells = orc.leaf_cells(g["N"], g["D"], T)
    assert cells.tolist() == [[fnum(v) for v in c] for c in g["cells"]]


def test_leaf_cells_single_leaf(orc):
    cells = orc.leaf_cells(1, 0, np.zeros(0, np.float32))
    assert cells.tolist() == [[-np.inf] * 3 + [np.inf] * 3]


@pytest.mark.parametrize("name", ["uniform-37", "lattice-64", "dups-50", "collinear-33", "coplanar-48", "five",
                                  "pow2p1", "three", "pair", "single"])
@pytest.mark.parametrize("r_max", [0.02, 0.05, 0.3])
def test_afford_direct_sandwich_and_recursion(orc, name, r_max):
    pts = CLOUDS[name]
    t = orc.build_tree(pts, 0.0, r_max, prune=False)
    off, idx = orc.afford_direct(pts, t.cell, r_max)
    # the direct definition reaches the recursion's sets exactly
    assert np.array_equal(off, t.off) and np.array_equal(idx, t.idx)
    rmax = Fraction(float(np.float32(r_max)))
    R = rmax * (1 + Fraction(1, 2 ** 20))
    for l in range(t.N):
        s = set(idx[off[l]:off[l + 1]].tolist())
        for j in range(len(pts)):
            d2 = _exact_cell_dist2(pts[j], t.cell[l])
            if d2 is not None and d2 <= rmax ** 2:
                assert j in s, (l, j)
            if j in s:
                assert d2 is not None and d2 <= R ** 2, (l, j)


def test_afford_direct_boundary_slack(orc):
    """A point just beyond r_max but within r_max (1 + 2^-20) of the cell is
    afforded; one beyond the slack is not."""
    r_max = 0.5
    cell = np.array([[0.0, 0.0, 0.0, 1.0, 1.0, 1.0]], np.float32)
    inside_slack = np.float32(1.0 + 0.5 * (1 + 2.0 ** -22))
    beyond = np.float32(1.0 + 0.5 * (1 + 2.0 ** -18))
    pts = np.array([[1.5, 0.5, 0.5], [inside_slack, 0.5, 0.5], [beyond, 0.5, 0.5], [0.5, 0.5, 0.5]], np.float32)
    off, idx = orc.afford_direct(pts, cell, r_max)
    assert idx.tolist() == [0, 1, 3]
