"""Pins of the Alg. 1 oracle (block nullification for step (I)).

Checked against what the mathematics fixes: P^(i) is orthonormal and annihilates
Omega^(i); the projected samples equal the far-field block sums taken by dense slicing
(the near field cancels exactly); a planted exact-rank uBLR matrix is recovered exactly;
the product count is s per side plus the b k and (colours) m of Table 1.
"""
import numpy as np
import pytest
import scipy.linalg

import oracle as O
import workloads as W


@pytest.fixture(scope="module")
def planted_bn():
    wl = W.WORKLOADS["planted_2d_n4096"]
    g = wl.geometry()
    A, us, vs = W.planted_exact_rank(g, wl.k, wl.seed)
    near = O.near_lists(g.lattice)
    s = O.bn_columns(g.box_ptr, near, wl.r)
    Om, Ps = W.gaussian_test_blocks(wl.seed, g.n, s)
    op = O.CountingOperator(O.DenseOperator(A))
    res = O.reconstruct_bn(op, g.box_ptr, g.lattice, wl.k, wl.p, Om, Ps)
    return dict(wl=wl, g=g, A=A, us=us, vs=vs, res=res, op=op, Om=Om, Ps=Ps, near=near, s=s)


def test_bn_columns_uniform_boxes(planted_bn):
    """On a uniform tessellation s = r + 3^d m (Alg. 1)."""
    g, wl = planted_bn["g"], planted_bn["wl"]
    assert planted_bn["s"] == wl.r + 3 ** g.dim * int(g.box_sizes()[0])


def test_null_vectors_annihilate_neighbour_rows(planted_bn):
    g, Om, near, r = planted_bn["g"], planted_bn["Om"], planted_bn["near"], planted_bn["wl"].r
    for i in (0, 9, 27, 63):
        M = Om[O.neighbour_rows(g.box_ptr, near[i])]
        P = O.null_r(M, r)
        assert P.shape == (Om.shape[1], r)
        assert np.max(np.abs(P.T @ P - np.eye(r))) <= 1e-13
        assert np.max(np.abs(M @ P)) <= 1e-12 * np.max(np.abs(M))


def test_projected_samples_vs_dense_far_sums(planted_bn):
    """Y(I_i,:) P^(i) = sum_{l in F_i} A(I_i, I_l) Omega(I_l,:) P^(i), and the adjoint side."""
    g, A, res = planted_bn["g"], planted_bn["A"], planted_bn["res"]
    Om, Ps, near, r, bp = planted_bn["Om"], planted_bn["Ps"], planted_bn["near"], planted_bn["wl"].r, g.box_ptr
    for i in range(0, g.nboxes, 9):
        nr = O.neighbour_rows(bp, near[i])
        P, Q = O.null_r(Om[nr], r), O.null_r(Ps[nr], r)
        ri = slice(bp[i], bp[i + 1])
        sy = np.zeros((bp[i + 1] - bp[i], r))
        sz = np.zeros_like(sy)
        for l in res["far"][i]:
            cl = slice(bp[l], bp[l + 1])
            sy += A[ri, cl] @ (Om[cl] @ P)
            sz += A[cl, ri].T @ (Ps[cl] @ Q)
        assert np.max(np.abs(res["SY"][ri] - sy)) <= 1e-11 * np.abs(sy).max()
        assert np.max(np.abs(res["SZ"][ri] - sz)) <= 1e-11 * np.abs(sz).max()


def test_bn_planted_exact_recovery(planted_bn):
    g, A, res, k = planted_bn["g"], planted_bn["A"], planted_bn["res"], planted_bn["wl"].k
    bp = g.box_ptr
    Ubd = scipy.linalg.block_diag(*[res["U"][bp[i]:bp[i + 1]] for i in range(g.nboxes)])
    Vbd = scipy.linalg.block_diag(*[res["V"][bp[i]:bp[i + 1]] for i in range(g.nboxes)])
    Ah = Ubd @ res["Atil"] @ Vbd.T
    for (i, j), Bij in res["B"].items():
        Ah[bp[i]:bp[i + 1], bp[j]:bp[j + 1]] += Bij
    assert np.linalg.norm(A - Ah) / np.linalg.norm(A) <= 1e-12
    for i in range(g.nboxes):
        Ui = res["U"][bp[i]:bp[i + 1]]
        assert np.linalg.norm(Ui @ Ui.T - planted_bn["us"][i] @ planted_bn["us"][i].T, 2) <= 1e-12


def test_bn_matvec_counts(planted_bn):
    g, wl, op, s = planted_bn["g"], planted_bn["wl"], planted_bn["op"], planted_bn["s"]
    m = int(np.max(g.box_sizes()))
    assert op.cols_At == s
    assert op.cols_A == s + g.nboxes * wl.k + 3 ** g.dim * m


def test_null_r_householder_on_a_coordinate_case():
    """M = [I_n 0]: null(M) is spanned by e_{n+1}..e_s, and the Householder QR of M* has
    identity reflectors, so null_r returns those unit vectors up to sign."""
    n, s, r = 3, 8, 4
    M = np.hstack([np.eye(n), np.zeros((n, s - n))])
    P = O.null_r(M, r)
    assert np.allclose(np.abs(P), np.eye(s)[:, n:n + r], atol=1e-15)
