"""Pins of the tolerance-driven truncation to per-box ranks (oracle/truncate.py).

* Planted per-box ranks: a matrix whose far block rows and columns have planted ranks
  k_i <= k, compressed at k and truncated at a tolerance far above roundoff and far below
  the planted singular values, returns exactly the planted ranks and stays exact.
* Exact accounting: the change of the represented matrix, evaluated densely, equals the
  dropped squares the rule adds up (the Pythagoras identity of the two-sided truncation),
  and stays within the budget.
* The error against A is within the compression error plus the tolerance (triangle
  inequality), the representation norm equals the dense Frobenius norm, and tol = 0
  changes nothing.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W


@pytest.fixture(scope="module")
def ragged():
    g = W.grid_geometry(2, 6, 6)                   # 36 boxes of 36 points
    k, p = 10, 8
    rng = np.random.default_rng(5)
    ku = rng.integers(2, k + 1, g.nboxes)
    kv = rng.integers(2, k + 1, g.nboxes)
    A, us, vs = W.planted_ragged_rank(g, ku, kv, 31)
    near = O.near_lists(g.lattice)
    ell = O.num_tag_columns(near, 3)
    T = W.tag_matrix(31, g.nboxes, ell)
    G, H = W.gaussian_test_blocks(31, g.n, k + p)
    res = O.reconstruct_tag(O.DenseOperator(A), g.box_ptr, g.lattice, k, p, 3, T, G, H)
    return dict(g=g, k=k, A=A, ku=ku, kv=kv, res=res, near=near, far=O.far_lists(near, g.nboxes))


def _dense(g, k, d):
    return O.dense_reconstruction(d["U"], d["V"], d["Atil"], d["B"], g.box_ptr, k)


def test_planted_ragged_ranks_recovered(ragged):
    g, k, res = ragged["g"], ragged["k"], ragged["res"]
    tr = O.truncate_ublr(res["U"], res["V"], res["Atil"], res["B"], g.box_ptr, ragged["near"], ragged["far"],
                         k, 1e-9)
    assert np.array_equal(tr["ranks_u"], ragged["ku"])
    assert np.array_equal(tr["ranks_v"], ragged["kv"])
    A = ragged["A"]
    err = np.linalg.norm(A - _dense(g, k, tr)) / np.linalg.norm(A)
    assert err <= 1e-12
    bp = g.box_ptr
    for i in range(g.nboxes):                      # orthonormal kept columns, zero padding
        Ui = tr["U"][bp[i]:bp[i + 1]]
        assert np.allclose(Ui[:, :tr["ranks_u"][i]].T @ Ui[:, :tr["ranks_u"][i]], np.eye(tr["ranks_u"][i]),
                           atol=1e-13)
        assert not np.any(Ui[:, tr["ranks_u"][i]:])


@pytest.mark.parametrize("tol", [1e-3, 1e-5, 1e-7])
def test_dropped_squares_equal_dense_change(tol):
    g = W.grid_geometry(2, 6, 5, jitter=0.2, seed=3)
    k, p = 12, 8
    A = O.KernelOperator("log", g.pts).block()
    near = O.near_lists(g.lattice)
    far = O.far_lists(near, g.nboxes)
    T = W.tag_matrix(8, g.nboxes, O.num_tag_columns(near, 3))
    G, H = W.gaussian_test_blocks(8, g.n, k + p)
    res = O.reconstruct_tag(O.DenseOperator(A), g.box_ptr, g.lattice, k, p, 3, T, G, H)
    tr = O.truncate_ublr(res["U"], res["V"], res["Atil"], res["B"], g.box_ptr, near, far, k, tol)
    A0 = _dense(g, k, res)
    A1 = _dense(g, k, tr)
    change = np.linalg.norm(A0 - A1) ** 2
    assert np.isclose(tr["norm"], np.linalg.norm(A0), rtol=1e-12)
    assert np.isclose(change, tr["dropped"], rtol=1e-8, atol=1e-24 * np.linalg.norm(A0) ** 2)
    assert tr["dropped"] <= (tol * tr["norm"]) ** 2 * (1 + 1e-12)
    assert np.sum(tr["ranks_u"]) < g.nboxes * k        # something was dropped
    e0 = np.linalg.norm(A - A0) / np.linalg.norm(A)
    e1 = np.linalg.norm(A - A1) / np.linalg.norm(A)
    assert e1 <= e0 + tol * tr["norm"] / np.linalg.norm(A) * (1 + 1e-10)
    for (i, j), Bij in tr["B"].items():                # near blocks represented as before
        bp = g.box_ptr
        ri, cj = slice(bp[i], bp[i + 1]), slice(bp[j], bp[j + 1])
        assert np.allclose(A1[ri, cj], A0[ri, cj], atol=1e-13 * np.abs(A0).max())


def test_zero_tolerance_changes_nothing(ragged):
    g, k, res = ragged["g"], ragged["k"], ragged["res"]
    tr = O.truncate_ublr(res["U"], res["V"], res["Atil"], res["B"], g.box_ptr, ragged["near"], ragged["far"],
                         k, 0.0)
    assert np.all(tr["ranks_u"] == k) and np.all(tr["ranks_v"] == k)
    A0 = _dense(g, k, res)
    assert np.max(np.abs(_dense(g, k, tr) - A0)) <= 1e-12 * np.max(np.abs(A0))


def test_drop_rule_on_hand_made_table():
    sig = np.array([[3.0, 2.0, 0.5], [4.0, 0.3, 0.1]])
    ranks, dropped = O.truncate._drop_count(sig, 0.1 ** 2 + 0.3 ** 2 + 1e-12)
    assert list(ranks) == [3, 1] and np.isclose(dropped, 0.1)
    ranks, dropped = O.truncate._drop_count(sig, 0.1 ** 2 + 0.3 ** 2 + 0.5 ** 2)
    assert list(ranks) == [2, 1]
    ranks, _ = O.truncate._drop_count(sig, 0.0)
    assert list(ranks) == [3, 3]
