"""Pins of oracle/design.py: the design difference of Eq. (10) against values
fixed by hand and by its definition, the adaptation trigger of Sec. 4 and the
p-continuation rule against their stated cases."""
import numpy as np
import pytest

from oracle import amr, design
from oracle.mesh import uniform_leaves


def _uniform(dims):
    lv, an, L = uniform_leaves(dims)
    return (lv, an, L, dims)


def test_difference_zero_for_same_design():
    m = _uniform((4, 3, 2))
    rho = np.random.default_rng(0).uniform(0.1, 1, 24)
    assert design.design_difference(m, rho, m, rho) == 0.0


def test_difference_two_elements_by_hand():
    # 2x1x1 lattice: rho1 = (1, 0.5), rho2 = (0.25, 0.5): |0.75| / 1.5 = 0.5
    m = _uniform((2, 1, 1))
    assert design.design_difference(m, [1.0, 0.5], m, [0.25, 0.5]) == pytest.approx(0.5, abs=0)
    # not symmetric: the denominator is the first design's volume
    assert design.design_difference(m, [0.25, 0.5], m, [1.0, 0.5]) == pytest.approx(1.0, abs=0)


def test_difference_coarse_leaf_counts_its_volume():
    """One level-0 leaf of edge 2 (8 finest cells) at rho = 1 against the 8
    refined children: children at 1 except one at 0 -> D = 1/8; a refined
    design that averages to the parent's value but differs cell by cell still
    counts every cell (L1, not a difference of means)."""
    coarse = (np.array([0]), np.array([[0, 0, 0]]), 1, (2, 2, 2))
    lv, an, _ = amr.refine(coarse[0], coarse[1], 1, [True])
    fine = (lv, an, 1, (2, 2, 2))
    kids = np.ones(8)
    kids[3] = 0.0
    assert design.design_difference(coarse, [1.0], fine, kids) == pytest.approx(1 / 8, abs=1e-15)
    alt = np.array([0.5, 1.5] * 4)  # mean 1
    assert design.design_difference(coarse, [1.0], fine, alt) == pytest.approx(0.5, abs=1e-15)


def test_difference_same_field_on_octree_and_uniform():
    """A piecewise-constant field that is constant on every family of the
    refined tree gives D = 0 between the tree and its uniform refinement."""
    base = (np.zeros(8, np.int64), np.array([[i, j, k] for k in (0, 1) for j in (0, 1) for i in (0, 1)]) * 4, 2)
    lv, an, _ = amr.refine(base[0], base[1], 2, np.arange(8) % 3 == 0)
    vals = np.random.default_rng(1).uniform(0, 1, len(lv))
    tree = (lv, an, 2, (8, 8, 8))
    cells = design.finest_cells(lv, an, 2, (8, 8, 8), vals)
    uni = _uniform((8, 8, 8))
    assert design.design_difference(tree, vals, uni, cells.ravel()) == 0.0


def test_difference_rejects_gaps():
    m = (np.array([0]), np.array([[0, 0, 0]]), 0, (2, 1, 1))
    with pytest.raises(ValueError):
        design.finest_cells(*m, [1.0])


@pytest.mark.parametrize("steps,change,due", [
    (4, 0.001, False),   # settled, but fewer than five steps on this mesh
    (5, 0.001, True),    # CASE (i)
    (5, 0.01, False),    # change must be strictly below the tolerance
    (9, 0.5, False),
    (10, 0.5, True),     # CASE (ii)
    (12, 0.5, True),
])
def test_adapt_trigger_cases(steps, change, due):
    assert design.adapt_due(steps, change) is due


def test_p_continuation():
    assert design.p_next(1.0, 3, 0.2) == 1.0
    assert design.p_next(1.0, 3, 0.005) == 1.5
    assert design.p_next(1.0, 20, 0.2) == 1.5
    assert design.p_next(2.75, 1, 0.0) == 3.0
    assert design.p_next(3.0, 50, 0.0) == 3.0
