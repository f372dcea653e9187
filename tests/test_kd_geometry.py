"""Host checks of the random-point geometry of Section 7 (uniform points in the unit
square, median-split tessellation, boxes that share a boundary are neighbours) and of
the planner on it (no GPU needed).

* Every box holds n / 2^levels points up to one, and every point lies in its box's cell.
* Cells tile the square: their areas sum to 1 and no two overlap in their interiors.
* Neighbour lists are symmetric, contain the box itself, and follow the shared-boundary
  rule, checked by brute force over pairs of cells.
* The planner's lists, probe colours and tag vectors on these lists equal the oracle's.
"""
import itertools

import numpy as np
import pytest

import oracle as O
import workloads as W

lib_mod = pytest.importorskip("paper_2501_05528_amd._lib")


@pytest.mark.parametrize("n,dim,levels", [(8192, 2, 6), (20000, 2, 7), (5000, 3, 6)])
def test_kd_tessellation(n, dim, levels):
    g, near, cells = W.kd_geometry(n, dim, levels, 20250106)
    sizes = g.box_sizes()
    assert g.n == n and g.nboxes == 2 ** levels
    assert sizes.max() - sizes.min() <= 1
    for i in range(g.nboxes):
        p = g.pts[g.box_ptr[i]:g.box_ptr[i + 1]]
        assert np.all(p >= cells[i, :, 0]) and np.all(p <= cells[i, :, 1])
    assert abs(np.prod(cells[:, :, 1] - cells[:, :, 0], axis=1).sum() - 1.0) < 1e-12
    for i, j in itertools.combinations(range(g.nboxes), 2):
        overlap = np.minimum(cells[i, :, 1], cells[j, :, 1]) - np.maximum(cells[i, :, 0], cells[j, :, 0])
        assert np.any(overlap <= 0)                       # interiors are disjoint
        touch = bool(np.all(overlap >= 0))                # closed cells meet
        assert (j in near[i]) == touch and (i in near[j]) == touch
    for i in range(g.nboxes):
        assert i in near[i] and near[i] == sorted(near[i])


def test_plan_on_kd_lists_matches_oracle():
    from paper_2501_05528_amd.api import Plan, tag_columns
    g, near, _ = W.kd_geometry(8192, 2, 6, 20250106)
    far = O.far_lists(near, g.nboxes)
    ell = O.num_tag_columns(near, 3)
    assert tag_columns(g.box_ptr, None, 3, near=near) == ell
    T = W.tag_matrix(20250106, g.nboxes, ell)
    pl = Plan(g.box_ptr, None, 16, T, p=10, extra_tag_cols=3, near=near)
    _, near_idx, colour, _ = pl.lists()
    assert near_idx.tolist() == [j for nb in near for j in nb]
    assert colour.tolist() == O.greedy_colours(near).tolist()
    for i in range(g.nboxes):
        assert len({int(colour[j]) for j in near[i]}) == len(near[i])
    z, rho = pl.tags()
    zo, rhoo = O.tag_plan(T, near, far)
    assert np.allclose(rho, rhoo, rtol=1e-9, atol=0)
    assert np.allclose(z, zo, rtol=0, atol=1e-9)


def test_any_box_count():
    """With nboxes given, the tessellation has exactly that many boxes of n / nboxes points
    up to one, cells that tile the square, and every point inside its box's cell."""
    for n, b in ((2000, 77), (1500, 10), (777, 1)):
        g, near, cells = W.kd_geometry(n, 2, 0, 5, nboxes=b)
        sizes = g.box_sizes()
        assert g.nboxes == b and sizes.sum() == n
        assert sizes.max() - sizes.min() <= 1
        assert np.isclose(np.prod(cells[:, :, 1] - cells[:, :, 0], axis=1).sum(), 1.0)
        for i in range(b):
            p = g.pts[g.box_ptr[i]:g.box_ptr[i + 1]]
            assert np.all((p >= cells[i, :, 0]) & (p <= cells[i, :, 1]))
            assert i in near[i]
