"""Pins of the Alg. 3 oracle (basic randomized SVD for step (I)).

Checked against what the mathematics fixes: exact recovery of a planted
exact-rank uBLR matrix, the randomized range finder bound against a brute-force
SVD of each far-field block row, the product count of Alg. 3, and the far-field
samples against dense block slicing.
"""
import numpy as np
import pytest
import scipy.linalg

import oracle as O
import workloads as W


@pytest.fixture(scope="module")
def planted_basic():
    wl = W.WORKLOADS["planted_2d_n4096"]
    g = wl.geometry()
    A, us, vs = W.planted_exact_rank(g, wl.k, wl.seed)
    G, H = W.gaussian_test_blocks(wl.seed, g.n, wl.r)
    op = O.CountingOperator(O.DenseOperator(A))
    res = O.reconstruct_basic(op, g.box_ptr, g.lattice, wl.k, wl.p, G, H)
    return dict(wl=wl, g=g, A=A, us=us, vs=vs, res=res, op=op, G=G, H=H)


def test_basic_planted_exact_recovery(planted_basic):
    g, A, res, k = planted_basic["g"], planted_basic["A"], planted_basic["res"], planted_basic["wl"].k
    bp = g.box_ptr
    Ubd = scipy.linalg.block_diag(*[res["U"][bp[i]:bp[i + 1]] for i in range(g.nboxes)])
    Vbd = scipy.linalg.block_diag(*[res["V"][bp[i]:bp[i + 1]] for i in range(g.nboxes)])
    Ah = Ubd @ res["Atil"] @ Vbd.T
    for (i, j), Bij in res["B"].items():
        Ah[bp[i]:bp[i + 1], bp[j]:bp[j + 1]] += Bij
    assert np.linalg.norm(A - Ah) / np.linalg.norm(A) <= 1e-12
    for i in range(g.nboxes):
        Ui = res["U"][bp[i]:bp[i + 1]]
        Vi = res["V"][bp[i]:bp[i + 1]]
        assert np.linalg.norm(Ui @ Ui.T - planted_basic["us"][i] @ planted_basic["us"][i].T, 2) <= 1e-12
        assert np.linalg.norm(Vi @ Vi.T - planted_basic["vs"][i] @ planted_basic["vs"][i].T, 2) <= 1e-12


def test_basic_matvec_counts(planted_basic):
    """Alg. 3 applies A and A* to b test matrices of r columns each; the cores add bk
    products and the near field 3^d m (Table 1)."""
    g, wl, op = planted_basic["g"], planted_basic["wl"], planted_basic["op"]
    m = int(np.max(g.box_sizes()))
    assert op.cols_At == g.nboxes * wl.r
    assert op.cols_A == g.nboxes * wl.r + g.nboxes * wl.k + 3 ** g.dim * m


def test_basic_samples_vs_dense_block_sums(planted_basic):
    """Y^(i)(I_i,:) = sum_{l in F_i} A(I_i, I_l) G(I_l,:) and the adjoint side with A(I_l, I_i)*,
    by dense slicing of A."""
    g, A, res = planted_basic["g"], planted_basic["A"], planted_basic["res"]
    G, H, bp = planted_basic["G"], planted_basic["H"], g.box_ptr
    for i in range(0, g.nboxes, 7):
        ri = slice(bp[i], bp[i + 1])
        sy = np.zeros((bp[i + 1] - bp[i], G.shape[1]))
        sz = np.zeros_like(sy)
        for l in res["far"][i]:
            cl = slice(bp[l], bp[l + 1])
            sy += A[ri, cl] @ G[cl]
            sz += A[cl, ri].T @ H[cl]
        assert np.allclose(res["SY"][ri], sy, rtol=0, atol=1e-12 * np.abs(sy).max())
        assert np.allclose(res["SZ"][ri], sz, rtol=0, atol=1e-12 * np.abs(sz).max())


def test_basic_masked_test_matrix_rows():
    g = W.grid_geometry(2, 5, 3)
    near = O.near_lists(g.lattice)
    G, _ = W.gaussian_test_blocks(3, g.n, 4)
    i = 12                                  # interior box of the 5 x 5 lattice
    Om = O.masked_test_matrix(G, g.box_ptr, near[i])
    for l in range(g.nboxes):
        rows = slice(g.box_ptr[l], g.box_ptr[l + 1])
        if l in near[i]:
            assert not Om[rows].any()
        else:
            assert np.array_equal(Om[rows], G[rows])


def test_basic_bases_vs_bruteforce_svd():
    """Randomized range finder (Section 2.4) on each far-field block row of a small
    Laplace matrix: ||(I - U U*) A(I_i, F_i)||_2 lies between sigma_{k+1} (no rank-k
    basis beats the SVD) and a modest multiple of the tail."""
    g = W.grid_geometry(2, 6, 4)          # 36 boxes of 16 points
    k, p = 4, 6
    A = O.KernelOperator("log", g.pts).block()
    G, H = W.gaussian_test_blocks(21, g.n, k + p)
    res = O.reconstruct_basic(O.DenseOperator(A), g.box_ptr, g.lattice, k, p, G, H, steps=("I",))
    bp = g.box_ptr
    for i in range(g.nboxes):
        ri = slice(bp[i], bp[i + 1])
        cols = np.concatenate([np.arange(bp[l], bp[l + 1]) for l in res["far"][i]])
        Ai = A[ri][:, cols]
        s = np.linalg.svd(Ai, compute_uv=False)
        U = res["U"][ri]
        err = np.linalg.norm(Ai - U @ (U.T @ Ai), 2)
        assert s[k] * (1 - 1e-10) <= err <= 10 * np.sqrt(np.sum(s[k:] ** 2)) + 1e-13 * np.abs(A).max()
        Ac = A[cols][:, ri]
        sc = np.linalg.svd(Ac, compute_uv=False)
        Vi = res["V"][ri]
        errv = np.linalg.norm(Ac - (Ac @ Vi) @ Vi.T, 2)
        assert sc[k] * (1 - 1e-10) <= errv <= 10 * np.sqrt(np.sum(sc[k:] ** 2)) + 1e-13 * np.abs(A).max()
