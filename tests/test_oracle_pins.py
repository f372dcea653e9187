"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: values the
paper prints (tests/golden/paper_examples.json), closed forms (cofactors and
minors, (3B-2)^d pair counts), identities (projected-tag cancellation,
Atil = U* A V), exact recovery of planted exact-rank matrices, brute-force
SVDs and brute-force scans of the aspect-ratio problem.
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg
from scipy.spatial.distance import cdist

import oracle as O
import workloads as W

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")))


def lattice_1d(b):
    return np.arange(b, dtype=np.int32).reshape(b, 1)


# ---------------------------------------------------------------- P1 lists/colours
def test_p1_neighbour_example_1d():
    ex = GOLDEN["neighbour_example_1d"]
    near = O.near_lists(lattice_1d(ex["nboxes"]))
    # paper numbers boxes from 1
    assert [j + 1 for j in near[ex["box"] - 1]] == ex["neighbours"]
    assert O.num_tag_columns(near, extra=0) == ex["tag_columns"]


@pytest.mark.parametrize("dim,B", [(1, 9), (2, 8), (2, 5), (3, 4)])
def test_p1_pair_counts_and_interior(dim, B):
    g = W.grid_geometry(dim, B, 2)
    near = O.near_lists(g.lattice)
    assert sum(len(n) for n in near) == (3 * B - 2) ** dim
    for i, n in enumerate(near):
        interior = all(0 < g.lattice[i, t] < B - 1 for t in range(dim))
        if interior:
            assert len(n) == 3 ** dim
        assert i in n and n == sorted(n)
    far = O.far_lists(near, g.nboxes)
    for i in range(g.nboxes):
        assert sorted(near[i] + far[i]) == list(range(g.nboxes))


@pytest.mark.parametrize("dim,B", [(1, 8), (2, 7), (3, 5)])
def test_p1_colours_unique_per_neighbourhood(dim, B):
    g = W.grid_geometry(dim, B, 1)
    near = O.near_lists(g.lattice)
    col = O.colours(g.lattice)
    assert set(col.tolist()) == set(range(3 ** dim))
    for n in near:
        cs = [col[j] for j in n]
        assert len(cs) == len(set(cs))


def test_p1_probe_colour_example_1d():
    ex = GOLDEN["probe_colour_example_1d"]
    col = O.colours(lattice_1d(ex["nboxes"]))
    members = [j + 1 for j in range(ex["nboxes"]) if col[j] == col[ex["boxes_in_one_colour"][0] - 1]]
    assert members == ex["boxes_in_one_colour"]


# ---------------------------------------------------------------- P2 null vectors
def test_p2_cofactor_closed_form_and_minors():
    """With ell = 3^d + 1 an interior box has a 1-D null space; z is proportional to
    the signed cofactors of T(N_i,:) and T z lists the (ell x ell) determinants
    [t_l; T(N_i,:)] (Section 5.2, eqs. cramers_rule and 4by4, with the
    alternating signs that the cofactor expansion carries)."""
    b = 8
    near = O.near_lists(lattice_1d(b))
    T = W.tag_matrix(7, b, 4)
    i = 2
    Ti = T[near[i]]
    z = O.null_space(Ti)[:, 0]
    cof = np.array([(-1) ** j * np.linalg.det(np.delete(Ti, j, axis=1)) for j in range(4)])
    scale = cof @ z
    assert np.allclose(z * scale, cof, rtol=0, atol=1e-13 * np.linalg.norm(cof))
    minors = np.array([np.linalg.det(np.vstack([T[l], Ti])) for l in range(b)])
    assert np.allclose(T @ cof, minors, rtol=0, atol=1e-12 * np.linalg.norm(minors))
    assert np.linalg.norm(Ti @ z) <= 1e-14 * np.linalg.norm(T)
    assert abs(np.linalg.norm(z) - 1) < 1e-14


@pytest.mark.parametrize("dim,B,extra", [(2, 6, 3), (3, 4, 3), (2, 5, 0)])
def test_p2_tag_vectors_in_null_space(dim, B, extra):
    g = W.grid_geometry(dim, B, 1)
    near = O.near_lists(g.lattice)
    far = O.far_lists(near, g.nboxes)
    ell = O.num_tag_columns(near, extra)
    T = W.tag_matrix(11, g.nboxes, ell)
    z, rho = O.tag_plan(T, near, far)
    for i in range(g.nboxes):
        assert np.linalg.norm(T[near[i]] @ z[i]) <= 1e-13 * np.linalg.norm(T)
        assert abs(np.linalg.norm(z[i]) - 1) < 1e-13
        assert rho[i] >= 1.0
        assert np.isclose(rho[i], O.aspect_ratio(T, far[i], z[i]), rtol=1e-12)


# ---------------------------------------------------------------- P10 worked example
def test_p10_worked_example_zero_pattern():
    """8 boxes in 1D, T is 8 x 4: the weighted sum of the Omega_j vanishes exactly on the
    block rows of N_3 = {2,3,4} and nowhere else (eq. projected_tags)."""
    b, m, r = 8, 5, 3
    near = O.near_lists(lattice_1d(b))
    far = O.far_lists(near, b)
    T = W.tag_matrix(3, b, 4)
    z, _ = O.optimise_tag_vector(T, near[2], far[2])
    box_ptr = np.arange(b + 1) * m
    G = W.gaussian_colmajor(3, 1, b * m, r)
    Om = O.extended_test_matrix(T, G, box_ptr)
    comb = sum(z[j] * Om[:, j * r:(j + 1) * r] for j in range(4))
    for l in range(b):
        blk = comb[l * m:(l + 1) * m]
        if l + 1 in (2, 3, 4):
            assert np.max(np.abs(blk)) < 1e-14
        else:
            assert np.max(np.abs(blk)) > 1e-6


# ---------------------------------------------------------------- P3 cancellation
def _small_dense_case(dim=2, B=5, q=3, k=4, p=3, seed=5):
    g = W.grid_geometry(dim, B, q)
    rs = np.random.default_rng(seed)
    A = rs.standard_normal((g.n, g.n))
    near = O.near_lists(g.lattice)
    ell = O.num_tag_columns(near, 3)
    T = W.tag_matrix(seed, g.nboxes, ell)
    G, H = W.gaussian_test_blocks(seed, g.n, k + p)
    return g, A, near, ell, T, G, H


def test_p3_tag_cancellation_identity():
    """Yhat_i = sum_{l in F_i} (T z^(i))_l A_il G_l and the A* analogue (eq. projected_tags):
    near-field blocks drop out for any A, by brute force on a dense random matrix."""
    k, p = 4, 3
    g, A, near, ell, T, G, H = _small_dense_case(k=k, p=p)
    r = k + p
    far = O.far_lists(near, g.nboxes)
    z, _ = O.tag_plan(T, near, far)
    Y, Z = O.tagging.sketch(O.DenseOperator(A), T, G, H, g.box_ptr)
    Yh = O.tag_postprocess(Y, z, g.box_ptr, r)
    Zh = O.tag_postprocess(Z, z, g.box_ptr, r)
    bp = g.box_ptr
    for i in range(g.nboxes):
        ri = slice(bp[i], bp[i + 1])
        c = T @ z[i]
        ref_y = sum(c[l] * A[ri, bp[l]:bp[l + 1]] @ G[bp[l]:bp[l + 1]] for l in far[i])
        ref_z = sum(c[l] * A[bp[l]:bp[l + 1], ri].T @ H[bp[l]:bp[l + 1]] for l in far[i])
        assert np.allclose(Yh[ri], ref_y, rtol=0, atol=1e-12 * np.abs(ref_y).max())
        assert np.allclose(Zh[ri], ref_z, rtol=0, atol=1e-12 * np.abs(ref_z).max())


# ---------------------------------------------------------------- P4 exact recovery
@pytest.fixture(scope="module")
def planted():
    wl = W.WORKLOADS["planted_2d_n4096"]
    g = wl.geometry()
    A, us, vs = W.planted_exact_rank(g, wl.k, wl.seed)
    near = O.near_lists(g.lattice)
    ell = O.num_tag_columns(near, 3)
    T = W.tag_matrix(wl.seed, g.nboxes, ell)
    G, H = W.gaussian_test_blocks(wl.seed, g.n, wl.r)
    op = O.CountingOperator(O.DenseOperator(A))
    res = O.reconstruct_tag(op, g.box_ptr, g.lattice, wl.k, wl.p, 3, T, G, H)
    return dict(wl=wl, g=g, A=A, us=us, vs=vs, res=res, op=op, ell=ell)


def test_p4_planted_exact_recovery(planted):
    g, A, res, k = planted["g"], planted["A"], planted["res"], planted["wl"].k
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
        assert np.linalg.norm(Ui @ Ui.T - planted["us"][i] @ planted["us"][i].T, 2) <= 1e-12
        assert np.linalg.norm(Vi @ Vi.T - planted["vs"][i] @ planted["vs"][i].T, 2) <= 1e-12
        assert np.allclose(Ui.T @ Ui, np.eye(k), atol=1e-13)


def test_p6_cores_and_nearfield_vs_dense(planted):
    """Atil_ij = U_i* A_ij V_j for all pairs and, for an exact-rank matrix (no far-field
    leakage into the probes), B_ij = A_ij - U_i Atil_ij V_j* on neighbour pairs
    (eq. uniformBLRbases ff., eq. discrepancymatrix), by dense slicing."""
    g, A, res, k = planted["g"], planted["A"], planted["res"], planted["wl"].k
    bp = g.box_ptr
    U, V, At = res["U"], res["V"], res["Atil"]
    for i in range(0, g.nboxes, 5):
        for j in range(g.nboxes):
            blk = U[bp[i]:bp[i + 1]].T @ A[bp[i]:bp[i + 1], bp[j]:bp[j + 1]] @ V[bp[j]:bp[j + 1]]
            assert np.allclose(At[i * k:(i + 1) * k, j * k:(j + 1) * k], blk, atol=1e-12)
    assert set(res["B"].keys()) == {(i, j) for i in range(g.nboxes) for j in res["near"][i]}
    for (i, j), Bij in res["B"].items():
        ref = A[bp[i]:bp[i + 1], bp[j]:bp[j + 1]] - \
            U[bp[i]:bp[i + 1]] @ At[i * k:(i + 1) * k, j * k:(j + 1) * k] @ V[bp[j]:bp[j + 1]].T
        assert np.allclose(Bij, ref, atol=1e-12)


def test_p6_nearfield_leakage_closed_form():
    """For a matrix that is not of exact rank, the probe of colour c picks up the far-field
    truncation residuals of every box of colour c (Table 1, near field by probing):
    B_ij = sum over boxes l of colour(j) of (A_il - U_i Atil_il V_l*)[:, :m_j], by dense
    slicing on a ragged jittered grid (boxes of unequal size)."""
    g = W.grid_geometry(2, (7, 6), (6, 5), jitter=0.3, seed=11)
    k, p = 8, 6
    op = O.KernelOperator("log", g.pts)
    A = op.block()
    near = O.near_lists(g.lattice)
    ell = O.num_tag_columns(near, 3)
    T = W.tag_matrix(5, g.nboxes, ell)
    G, H = W.gaussian_test_blocks(5, g.n, k + p)
    res = O.reconstruct_tag(O.DenseOperator(A), g.box_ptr, g.lattice, k, p, 3, T, G, H)
    bp, U, V, At, col = g.box_ptr, res["U"], res["V"], res["Atil"], res["colour"]
    leak = 0.0
    for (i, j), Bij in res["B"].items():
        ri = slice(bp[i], bp[i + 1])
        ref = np.zeros_like(Bij)
        for l in range(g.nboxes):
            if col[l] != col[j]:
                continue
            cl = slice(bp[l], bp[l + 1])
            R = A[ri, cl] - U[ri] @ At[i * k:(i + 1) * k, l * k:(l + 1) * k] @ V[cl].T
            w = min(R.shape[1], Bij.shape[1])
            ref[:, :w] += R[:, :w]
            if l != j:
                leak = max(leak, np.max(np.abs(R)))
        assert np.max(np.abs(Bij - ref)) <= 1e-12 * np.max(np.abs(A)), (i, j)
    assert leak > 1e-8          # the far residuals are really there in this case


def test_p6_apply_equals_matrix_for_exact_rank(planted):
    g, A, res, k = planted["g"], planted["A"], planted["res"], planted["wl"].k
    x = np.random.default_rng(0).standard_normal((g.n, 3))
    y = O.ublr_apply(res["U"], res["V"], res["Atil"], res["B"], g.box_ptr, k, x)
    yt = O.ublr_apply(res["U"], res["V"], res["Atil"], res["B"], g.box_ptr, k, x, trans=True)
    assert np.allclose(y, A @ x, atol=1e-11 * np.abs(A @ x).max())
    assert np.allclose(yt, A.T @ x, atol=1e-11 * np.abs(A.T @ x).max())


def _random_factors(g, k, seed):
    """Unstructured U, V, Atil and near blocks B on the lattice neighbour pairs."""
    rng = np.random.default_rng(seed)
    near = O.near_lists(g.lattice)
    bp = g.box_ptr
    U = rng.standard_normal((g.n, k))
    V = rng.standard_normal((g.n, k))
    At = rng.standard_normal((g.nboxes * k, g.nboxes * k))
    B = {(i, j): rng.standard_normal((bp[i + 1] - bp[i], bp[j + 1] - bp[j]))
         for i in range(g.nboxes) for j in near[i]}
    return U, V, At, B


def test_dense_reconstruction_entries_bruteforce():
    """Entry (p, q) of U Atil V* + B (eq. uniformBLRfull) is
    sum_a sum_c U[p, a] Atil[i k + a, j k + c] V[q, c], plus B_ij[p - start_i, q - start_j]
    when j is a neighbour of i; evaluated with scalar loops on a ragged grid."""
    g = W.grid_geometry(2, (4, 3), (3, 2), jitter=0.2, seed=5)
    k = 2
    U, V, At, B = _random_factors(g, k, 17)
    Ah = O.dense_reconstruction(U, V, At, B, g.box_ptr, k)
    bp = g.box_ptr
    box_of = np.repeat(np.arange(g.nboxes), np.diff(bp))
    rng = np.random.default_rng(1)
    for _ in range(300):
        p, q = (int(v) for v in rng.integers(0, g.n, 2))
        i, j = int(box_of[p]), int(box_of[q])
        ref = 0.0
        for a in range(k):
            for c in range(k):
                ref += U[p, a] * At[i * k + a, j * k + c] * V[q, c]
        if (i, j) in B:
            ref += B[(i, j)][p - bp[i], q - bp[j]]
        assert abs(Ah[p, q] - ref) <= 1e-13 * (1 + abs(ref)), (p, q)


def test_dense_reconstruction_planted_factors(planted):
    """With the planted matrix's own bases (U*_i, V*_j), Atil = U* A V and
    B_ij = A_ij - U*_i Atil_ij V*_j^T on neighbour pairs, the reconstruction is A itself."""
    g, A, k = planted["g"], planted["A"], planted["wl"].k
    bp = g.box_ptr
    U = np.vstack(planted["us"])
    V = np.vstack(planted["vs"])
    Ubd = scipy.linalg.block_diag(*planted["us"])
    Vbd = scipy.linalg.block_diag(*planted["vs"])
    At = Ubd.T @ A @ Vbd
    near = O.near_lists(g.lattice)
    B = {}
    for i in range(g.nboxes):
        for j in near[i]:
            ri, cj = slice(bp[i], bp[i + 1]), slice(bp[j], bp[j + 1])
            B[(i, j)] = A[ri, cj] - planted["us"][i] @ At[i * k:(i + 1) * k, j * k:(j + 1) * k] @ planted["vs"][j].T
    Ah = O.dense_reconstruction(U, V, At, B, bp, k)
    assert np.max(np.abs(Ah - A)) <= 1e-12 * np.max(np.abs(A))


def test_dense_reconstruction_agrees_with_apply_and_fro():
    """The dense form, the apply (both orientations) and the block-wise Frobenius error
    are three separate evaluations of one representation: they must agree."""
    g = W.grid_geometry(2, 4, 3, jitter=0.1, seed=2)
    k = 3
    U, V, At, B = _random_factors(g, k, 23)
    Ah = O.dense_reconstruction(U, V, At, B, g.box_ptr, k)
    x = np.random.default_rng(4).standard_normal((g.n, 2))
    for trans, M in ((False, Ah), (True, Ah.T)):
        y = O.ublr_apply(U, V, At, B, g.box_ptr, k, x, trans=trans)
        assert np.max(np.abs(y - M @ x)) <= 1e-12 * np.max(np.abs(M @ x))
    A = O.KernelOperator("log", g.pts).block()
    fro = O.rel_fro_error(O.DenseOperator(A), U, V, At, B, g.box_ptr, k)
    assert np.isclose(fro, np.linalg.norm(A - Ah) / np.linalg.norm(A), rtol=1e-12)


# ---------------------------------------------------------------- P7 matvec counts
def test_p7_matvec_counts(planted):
    """Sketch 2 ell r products (Section 4.2), cores bk and near field 3^d m (Table 1)."""
    g, wl, op = planted["g"], planted["wl"], planted["op"]
    ell, r, k = planted["ell"], wl.r, wl.k
    m = int(np.max(g.box_sizes()))
    assert op.cols_At == ell * r
    assert op.cols_A == ell * r + g.nboxes * k + 3 ** g.dim * m


# ---------------------------------------------------------------- P8 sizing rule
def test_p8_block_count_rule():
    ex = GOLDEN["block_count_rule"]
    for c in ex["cases"]:
        assert W.blocks_for_rank(c["N"], ex["k"], ex["dim"]) == c["b"]


# ---------------------------------------------------------------- P5 bases
def test_p5_bases_vs_bruteforce_svd():
    """On a small Laplace problem the basis captures the far-field block row nearly as
    well as its optimal rank-k subspace: ||(I - U U*) A(I_i, F_i)||_2 is within a
    modest factor (times the aspect ratio) of sigma_{k+1} plus the tail
    (randomized range finder guarantee, Section 2.4)."""
    g = W.grid_geometry(2, 6, 4)          # 36 boxes of 16 points
    k, p = 4, 6
    op = O.KernelOperator("log", g.pts)
    A = op.block()
    near = O.near_lists(g.lattice)
    ell = O.num_tag_columns(near, 3)
    T = W.tag_matrix(21, g.nboxes, ell)
    G, H = W.gaussian_test_blocks(21, g.n, k + p)
    res = O.reconstruct_tag(O.DenseOperator(A), g.box_ptr, g.lattice, k, p, 3, T, G, H,
                            steps=("I",))
    bp = g.box_ptr
    for i in range(g.nboxes):
        ri = slice(bp[i], bp[i + 1])
        cols = np.concatenate([np.arange(bp[l], bp[l + 1]) for l in res["far"][i]])
        Ai = A[ri][:, cols]
        s = np.linalg.svd(Ai, compute_uv=False)
        U = res["U"][ri]
        err = np.linalg.norm(Ai - U @ (U.T @ Ai), 2)
        tail = np.sqrt(np.sum(s[k:] ** 2))
        assert err <= 10 * res["rho"][i] * tail + 1e-13 * np.abs(A).max()
        assert err >= s[k] * (1 - 1e-10)            # no rank-k basis beats the SVD
        # V from the adjoint side, against the far-field block column
        Vi = res["V"][ri]
        Ac = A[cols][:, ri]
        sc = np.linalg.svd(Ac, compute_uv=False)
        errv = np.linalg.norm(Ac - (Ac @ Vi) @ Vi.T, 2)
        assert errv <= 10 * res["rho"][i] * np.sqrt(np.sum(sc[k:] ** 2)) + 1e-13 * np.abs(A).max()


def test_col_topk_matches_known_subspace():
    rs = np.random.default_rng(1)
    Q, _ = np.linalg.qr(rs.standard_normal((30, 5)))
    M = Q @ np.diag([5, 4, 3, 2, 1.0]) @ rs.standard_normal((5, 9))
    U = O.col_topk(M, 5)
    assert np.linalg.norm(U @ U.T - Q @ Q.T, 2) < 1e-13
    for c in range(5):
        assert U[np.argmax(np.abs(U[:, c])), c] > 0


# ---------------------------------------------------------------- aspect-ratio LP
def test_lp_improves_on_every_start():
    g = W.grid_geometry(2, 6, 1)
    near = O.near_lists(g.lattice)
    far = O.far_lists(near, g.nboxes)
    ell = O.num_tag_columns(near, 3)
    T = W.tag_matrix(5, g.nboxes, ell)
    for i in range(g.nboxes):
        z, rho = O.optimise_tag_vector(T, near[i], far[i], optimise=True)
        z0, rho0 = O.optimise_tag_vector(T, near[i], far[i], optimise=False)
        assert rho <= rho0 * (1 + 1e-12)
        X = O.null_space(T[near[i]])
        P = X @ X.T
        for j in range(ell):
            w = P[:, j]
            if np.linalg.norm(w) > 1e-12:
                assert rho <= O.aspect_ratio(T, far[i], w) * (1 + 1e-9)


def test_lp_cell_optimum_matches_bruteforce_scan_2d_nullspace():
    """With a 2-D null space the unit vectors are a circle; scanning it finely and
    refining locally gives the minimum aspect ratio in each sign cell, which must
    equal the LP optimum for the cell that the LP picked."""
    b = 12
    near = O.near_lists(lattice_1d(b))
    far = O.far_lists(near, b)
    T = W.tag_matrix(9, b, 5)              # ell = 3 + 2: interior null space is 2-D
    i = 5
    X = O.null_space(T[near[i]])
    assert X.shape[1] == 2
    z, rho = O.optimise_tag_vector(T, near[i], far[i])
    Tf = T[far[i]]
    sig = np.sign(Tf @ z)
    th = np.linspace(0, 2 * np.pi, 200001)
    pts = np.cos(th)[:, None] * X[:, 0] + np.sin(th)[:, None] * X[:, 1]
    c = pts @ Tf.T
    same = np.all(np.sign(c) == sig, axis=1)
    ratios = np.where(same, np.max(np.abs(c), axis=1) / np.min(np.abs(c), axis=1), np.inf)
    j = int(np.argmin(ratios))
    lo, hi = th[max(j - 1, 0)], th[min(j + 1, th.size - 1)]
    from scipy.optimize import minimize_scalar
    f = lambda t: (lambda v: np.max(np.abs(v)) / np.min(np.abs(v)))(Tf @ (np.cos(t) * X[:, 0] + np.sin(t) * X[:, 1]))
    best = minimize_scalar(f, bounds=(lo, hi), method="bounded", options={"xatol": 1e-13}).fun
    assert abs(best - rho) <= 1e-7 * rho


# ---------------------------------------------------------------- kernels, errors
@pytest.mark.parametrize("kind", ["log", "inv_r", "exp", "cos"])
def test_kernel_blocks_vs_cdist(kind):
    g = W.grid_geometry(2, 3, 4, jitter=0.25, seed=3)
    op = O.KernelOperator(kind, g.pts)
    A = op.block()
    d = cdist(g.pts, g.pts)
    np.fill_diagonal(d, 1.0)
    ref = {"log": np.log(d), "inv_r": 1 / d, "exp": np.exp(-d / 0.1),
           "cos": np.cos(20 * d) / (d + 1e-3)}[kind]
    np.fill_diagonal(ref, {"log": 0.0, "inv_r": 0.0, "exp": 1.0, "cos": 1000.0}[kind])
    assert np.allclose(A, ref, rtol=1e-14, atol=1e-14)
    assert np.allclose(A, A.T, rtol=0, atol=0)
    x = np.random.default_rng(2).standard_normal((g.n, 2))
    assert np.allclose(op.matmat(x), ref @ x, atol=1e-12 * np.abs(ref @ x).max())


def test_p9_errors_fro_and_power():
    """Exact Frobenius error matches a dense computation; the 20-step power estimate of
    ||A - A_uBLR||_2 is a lower bound within 10% of the dense 2-norm."""
    g = W.grid_geometry(2, 6, 4)
    k, p = 3, 5
    op = O.KernelOperator("log", g.pts)
    A = op.block()
    near = O.near_lists(g.lattice)
    ell = O.num_tag_columns(near, 3)
    T = W.tag_matrix(4, g.nboxes, ell)
    G, H = W.gaussian_test_blocks(4, g.n, k + p)
    res = O.reconstruct_tag(O.DenseOperator(A), g.box_ptr, g.lattice, k, p, 3, T, G, H)
    bp = g.box_ptr
    Ubd = scipy.linalg.block_diag(*[res["U"][bp[i]:bp[i + 1]] for i in range(g.nboxes)])
    Vbd = scipy.linalg.block_diag(*[res["V"][bp[i]:bp[i + 1]] for i in range(g.nboxes)])
    Ah = Ubd @ res["Atil"] @ Vbd.T
    for (i, j), Bij in res["B"].items():
        Ah[bp[i]:bp[i + 1], bp[j]:bp[j + 1]] += Bij
    E = A - Ah
    fro = O.rel_fro_error(op, res["U"], res["V"], res["Atil"], res["B"], bp, k)
    assert np.isclose(fro, np.linalg.norm(E) / np.linalg.norm(A), rtol=1e-10)
    x0 = W.gaussian_colmajor(4, W.STREAM_POWER, g.n, 1)[:, 0]
    est = O.power_norm_estimate(lambda v: E @ v, lambda v: E.T @ v, g.n, x0, 20)
    true = np.linalg.norm(E, 2)
    assert est <= true * (1 + 1e-12) and est >= 0.9 * true


# ---------------------------------------------------------------- P11 mixed-precision refinement
def test_p11_far_sample_vs_masked_dense():
    """far_sample = (A with every near block zeroed) X, by an elementwise block mask on the
    dense matrix (both orientations), on a ragged jittered grid."""
    g = W.grid_geometry(2, (5, 4), (4, 3), jitter=0.3, seed=4)
    A = O.KernelOperator("exp", g.pts).block()
    A = A + 0.1 * np.random.default_rng(1).standard_normal(A.shape)   # make it nonsymmetric
    op = O.DenseOperator(A)
    near = O.near_lists(g.lattice)
    far = O.far_lists(near, g.nboxes)
    rb = np.repeat(np.arange(g.nboxes), np.diff(g.box_ptr))
    mask = np.ones_like(A)
    for i in range(g.nboxes):
        for j in near[i]:
            mask[np.ix_(rb == i, rb == j)] = 0.0
    X = np.random.default_rng(2).standard_normal((g.n, 5))
    assert np.allclose(O.far_sample(op, X, g.box_ptr, far), (A * mask) @ X, atol=1e-13)
    assert np.allclose(O.far_sample(op, X, g.box_ptr, far, adjoint=True), (A * mask).T @ X, atol=1e-13)


def test_p11_sample_basis_spans_and_signs():
    S = np.random.default_rng(3).standard_normal((30, 7)) @ np.diag(10.0 ** -np.arange(7))
    Q = O.sample_basis(S)
    assert np.allclose(Q.T @ Q, np.eye(7), atol=1e-14)
    assert np.allclose(Q @ (Q.T @ S), S, atol=1e-14)
    for c in range(7):
        assert Q[np.argmax(np.abs(Q[:, c])), c] > 0


def test_p11_refinement_recovers_exact_rank_from_perturbed_bases(planted):
    """For an exact-rank far field, any r_lo-column starting bases whose span holds the
    true column spaces up to a perturbation give exact bases after the refinement: the
    far-field samples are exact FP64 products, so their range is the true U_i."""
    g, A, wl = planted["g"], planted["A"], planted["wl"]
    k, bp = wl.k, g.box_ptr
    near = O.near_lists(g.lattice)
    far = O.far_lists(near, g.nboxes)
    r_lo, r = k + 6, k + 4
    rng = np.random.default_rng(5)
    U0 = np.zeros((g.n, r_lo))
    V0 = np.zeros((g.n, r_lo))
    for i in range(g.nboxes):
        rows = slice(bp[i], bp[i + 1])
        m = bp[i + 1] - bp[i]
        for Q0, tru in ((U0, planted["us"][i]), (V0, planted["vs"][i])):
            X = np.hstack([tru + 1e-3 * rng.standard_normal(tru.shape), rng.standard_normal((m, r_lo - k))])
            Q0[rows] = O.sample_basis(X)
    gu, gv = W.refinement_gammas(9, g.nboxes, r_lo, r)
    U, V, _, _ = O.refine_bases(O.DenseOperator(A), U0, V0, gu, gv, bp, far, k)
    for i in range(g.nboxes):
        rows = slice(bp[i], bp[i + 1])
        us, vs = planted["us"][i], planted["vs"][i]
        assert np.linalg.norm(U[rows] @ U[rows].T - us @ us.T, 2) <= 1e-11
        assert np.linalg.norm(V[rows] @ V[rows].T - vs @ vs.T, 2) <= 1e-11


def test_p11_refined_pipeline_exact_rank(planted):
    g, A, wl = planted["g"], planted["A"], planted["wl"]
    k, bp = wl.k, g.box_ptr
    near = O.near_lists(g.lattice)
    ell = O.num_tag_columns(near, 3)
    T = W.tag_matrix(wl.seed, g.nboxes, ell)
    r_lo = k + 10
    G, H = W.gaussian_test_blocks(wl.seed, g.n, r_lo)
    gu, gv = W.refinement_gammas(wl.seed, g.nboxes, r_lo, k + wl.p)
    op = O.DenseOperator(A)
    res = O.reconstruct_tag_refined(op, bp, g.lattice, k, wl.p, 3, T, G, H, gu, gv)
    assert O.rel_fro_error(op, res["U"], res["V"], res["Atil"], res["B"], bp, k) <= 1e-12


def test_p11_refinement_no_worse_than_plain_tagging():
    """A half-step of subspace iteration: on the log kernel the refined bases are at least
    as accurate as plain tagging with the same sketch width (same seeds)."""
    g = W.grid_geometry(2, 5, 8)
    k, p = 12, 8
    op = O.DenseOperator(O.KernelOperator("log", g.pts).block())
    near = O.near_lists(g.lattice)
    ell = O.num_tag_columns(near, 3)
    T = W.tag_matrix(21, g.nboxes, ell)
    G, H = W.gaussian_test_blocks(21, g.n, k + p)
    plain = O.reconstruct_tag(op, g.box_ptr, g.lattice, k, p, 3, T, G, H)
    gu, gv = W.refinement_gammas(21, g.nboxes, k + p, k + p)
    ref = O.reconstruct_tag_refined(op, g.box_ptr, g.lattice, k, p, 3, T, G, H, gu, gv)
    e0 = O.rel_fro_error(op, plain["U"], plain["V"], plain["Atil"], plain["B"], g.box_ptr, k)
    e1 = O.rel_fro_error(op, ref["U"], ref["V"], ref["Atil"], ref["B"], g.box_ptr, k)
    assert e1 <= 1.05 * e0, (e0, e1)


def test_p11_each_side_uses_the_other_sides_basis():
    """U_i comes from the far block row applied to blocks of V0 (and V_j from the block
    column applied to blocks of U0): with good V0 and U0 orthogonal to V0 (useless as a
    test space for the far block row) the U side still meets
    the brute-force bound ||F_i - U_i U_i* F_i||_2 <= 10 sigma_{k+1}(F_i), on a
    nonsymmetric matrix."""
    g = W.grid_geometry(2, 5, 8)
    k, p = 10, 8
    r_lo = k + p
    K = O.KernelOperator("log", g.pts).block()
    x = g.pts[:, 0]
    A = K + np.outer(np.cos(3 * x), np.sin(2 * x))          # nonsymmetric, far blocks stay low rank
    op = O.DenseOperator(A)
    bp = g.box_ptr
    near = O.near_lists(g.lattice)
    far = O.far_lists(near, g.nboxes)
    ell = O.num_tag_columns(near, 3)
    T = W.tag_matrix(31, g.nboxes, ell)
    G, H = W.gaussian_test_blocks(31, g.n, r_lo)
    z, _ = O.tag_plan(T, near, far)
    _, Z = O.tagging.sketch(op, T, G, H, bp)
    V0 = O.sample_bases(O.tag_postprocess(Z, z, bp, r_lo), bp)
    # U0 deliberately useless for the U side: orthogonal to V0 in every box
    U0 = np.zeros_like(V0)
    rng = np.random.default_rng(6)
    for i in range(g.nboxes):
        rows = slice(bp[i], bp[i + 1])
        X = rng.standard_normal((bp[i + 1] - bp[i], r_lo))
        U0[rows] = O.sample_basis(X - V0[rows] @ (V0[rows].T @ X))
    gu, gv = W.refinement_gammas(31, g.nboxes, r_lo, k + p)
    U, _, _, _ = O.refine_bases(op, U0, V0, gu, gv, bp, far, k)
    for i in range(g.nboxes):
        ri = slice(bp[i], bp[i + 1])
        cols = np.concatenate([np.arange(bp[l], bp[l + 1]) for l in far[i]])
        F = A[ri][:, cols]
        s = np.linalg.svd(F, compute_uv=False)
        Ui = U[ri]
        assert np.linalg.norm(F - Ui @ (Ui.T @ F), 2) <= 10 * s[k], i


def test_greedy_colours_chain_and_validity():
    """Greedy probe colours for given lists: on a 1D chain they are i mod 3 (the lattice
    colouring, which puts boxes 1, 4, 7 in one class as in the paper's probe figure), and
    for any symmetric relation no box has two neighbours of one colour."""
    b = 10
    chain = [[j for j in (i - 1, i, i + 1) if 0 <= j < b] for i in range(b)]
    assert O.greedy_colours(chain).tolist() == [i % 3 for i in range(b)]
    assert O.greedy_colours(chain).tolist() == O.colours(np.arange(b)[:, None]).tolist()
    rng = np.random.default_rng(5)
    for _ in range(20):
        n = 15
        M = rng.random((n, n)) < 0.2
        M = M | M.T | np.eye(n, dtype=bool)
        near = [list(np.flatnonzero(M[i])) for i in range(n)]
        col = O.greedy_colours(near)
        for i in range(n):
            assert len({int(col[j]) for j in near[i]}) == len(near[i])
        # greedy bound: at most one more colour than the largest two-step neighbourhood
        two = max(len({l for j in near[i] for l in near[j]}) for i in range(n))
        assert int(col.max()) + 1 <= two


def test_planted_exact_recovery_with_wider_admissibility():
    """A planted uniform-BLR matrix whose blocks are low rank beyond lattice distance 1 is
    still exactly recovered when distance <= 2 is declared near: the far field only shrinks
    (Section 2.5 with a caller-given neighbour relation)."""
    g = W.grid_geometry(2, 6, 4)
    k, p = 3, 5
    A, _, _ = W.planted_exact_rank(g, k, 11)
    lat = np.asarray(g.lattice)
    near = [[j for j in range(g.nboxes) if int(np.max(np.abs(lat[i] - lat[j]))) <= 2]
            for i in range(g.nboxes)]
    ell = O.num_tag_columns(near, 3)
    T = W.tag_matrix(11, g.nboxes, ell)
    G, H = W.gaussian_test_blocks(11, g.n, k + p)
    op = O.DenseOperator(A)
    res = O.reconstruct_tag(op, g.box_ptr, None, k, p, 3, T, G, H, near=near)
    assert res["ell"] == 29 and int(res["colour"].max()) + 1 >= 25
    err = O.rel_fro_error(op, res["U"], res["V"], res["Atil"], res["B"], g.box_ptr, k)
    assert err <= 1e-12, err
