"""Pins of the tolerance-driven rank choice: on a planted exact-rank uBLR matrix the
post-processed samples have exactly k nonzero singular values per box, so every
tolerance between the roundoff level and the smallest of them returns k; the rule
counts per box and takes the largest count over boxes and sides (hand-made tables)."""
import numpy as np

import oracle as O
import workloads as W


def test_planted_rank_is_recovered():
    wl = W.WORKLOADS["planted_2d_n4096"]
    g = wl.geometry()
    A, _, _ = W.planted_exact_rank(g, wl.k, wl.seed)
    near = O.near_lists(g.lattice)
    T = W.tag_matrix(wl.seed, g.nboxes, O.num_tag_columns(near, 3))
    G, H = W.gaussian_test_blocks(wl.seed, g.n, wl.r)
    res = O.reconstruct_tag(O.DenseOperator(A), g.box_ptr, g.lattice, wl.k, wl.p, 3, T, G, H, steps=("I",))
    sy = O.box_singular_values(res["Yhat"], g.box_ptr)
    sz = O.box_singular_values(res["Zhat"], g.box_ptr)
    assert sy.shape == (g.nboxes, wl.r)
    for tol in (1e-6, 1e-9, 1e-11):
        assert O.rank_for_tolerance(sy, sz, tol) == wl.k
    assert O.rank_for_tolerance(sy, sz, 1e-30) == wl.r     # below roundoff: the whole sample


def test_rule_on_hand_made_tables():
    sy = np.array([[10.0, 1.0, 0.1, 0.0], [5.0, 0.5, 0.05, 0.0]])
    sz = np.array([[8.0, 4.0, 0.001, 0.0], [1.0, 0.0, 0.0, 0.0]])
    assert O.rank_for_tolerance(sy, sz, 0.5) == 1      # Y: 10 > 5; Z: 8, 4 > 4? no -> 1
    assert O.rank_for_tolerance(sy, sz, 0.3) == 2      # Z: 8 and 4 > 2.4
    assert O.rank_for_tolerance(sy, sz, 0.009) == 3    # Y: 0.1 > 0.09
    assert O.rank_for_tolerance(sy, sz, 1e-4) == 3     # Z: 0.001 > 0.0008
    assert O.rank_for_tolerance(np.zeros((2, 3)), np.zeros((2, 3)), 0.1) == 0
