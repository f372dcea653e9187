"""Alg. 2 (tagging for basis construction) in plain FP64 (test infrastructure only).

Notation follows Section 4: b boxes with index sets I_i, r = k + p, the
tagging matrix T (b x ell), Gaussian blocks G_i, H_i (m_i x r), the extended
test matrices Omega, Psi (eq. extend_test_mat), sketches Y = A Omega and
Z = A* Psi partitioned into ell blocks of r columns, the tag vector
z^(i) = null(T(N_i,:)) and the weighted sums of Alg. 2 that feed col(., k).
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import linprog


# ---------------------------------------------------------------------------
# Test matrices and sketch (Alg. 2 up to the sketch; eq. extend_test_mat)
# ---------------------------------------------------------------------------

def extended_test_matrix(T: np.ndarray, G: np.ndarray, box_ptr: np.ndarray) -> np.ndarray:
    """Omega = [Omega_1 ... Omega_ell] with block row i of Omega_j equal to t_ij G_i
    (eq. extend_test_mat; Alg. 2 appends [t_i1 G_i ... t_i,ell G_i] for each box)."""
    n, r = G.shape
    b, ell = T.shape
    om = np.zeros((n, ell * r))
    for i in range(b):
        rows = slice(int(box_ptr[i]), int(box_ptr[i + 1]))
        for j in range(ell):
            om[rows, j * r:(j + 1) * r] = T[i, j] * G[rows, :]
    return om


def sketch(op, T, G, H, box_ptr):
    """Y = A Omega and Z = A* Psi with the same T for both (Alg. 2, sketch step)."""
    om = extended_test_matrix(T, G, box_ptr)
    ps = extended_test_matrix(T, H, box_ptr)
    return op.matmat(om), op.rmatmat(ps)


# ---------------------------------------------------------------------------
# Null vectors and aspect ratios (Section 2.3, eq. tagsubmat, Section 5)
# ---------------------------------------------------------------------------

def null_space(M: np.ndarray) -> np.ndarray:
    """Orthonormal basis of null(M) (Section 2.3), from the SVD of M."""
    M = np.atleast_2d(M)
    _, s, vt = np.linalg.svd(M, full_matrices=True)
    tol = max(M.shape) * np.finfo(float).eps * (s[0] if s.size else 0.0)
    rank = int(np.sum(s > tol))
    return vt[rank:].T.copy()


def projected_tags(T: np.ndarray, z: np.ndarray) -> np.ndarray:
    """The weights T z of the Gaussian blocks after tag post-processing (eq. projected_tags)."""
    return T @ z


def aspect_ratio(T: np.ndarray, far_i, z: np.ndarray) -> float:
    """rho^(i) = max_{j in F_i} |(T z)_j| / min_{j in F_i} |(T z)_j| (eq. aspect_ratio)."""
    c = np.abs(T[np.asarray(far_i, dtype=np.int64)] @ z)
    return float(np.max(c) / np.min(c))


def canonical_sign(z: np.ndarray) -> np.ndarray:
    """Reading: z and -z are the same tag vector; fix the sign so that the entry of
    largest magnitude (lowest index on ties) is positive."""
    q = int(np.argmax(np.abs(z)))
    return -z if z[q] < 0 else z


def _lp_in_cell(T: np.ndarray, near_i, far_i, sigma: np.ndarray):
    """Minimise the aspect ratio inside one sign cell of the null space (Section 5.3).

    Reading: on the cell {x in null(T(N_i,:)) : sign(t_l^T x) = sigma_l for l in F_i}
    the ratio max|t_l^T x| / min|t_l^T x| is scale invariant, so normalising the
    smallest projected tag to 1 turns the problem into the linear program

        minimise tau  over (x, tau)
        subject to T(N_i,:) x = 0,  1 <= sigma_l t_l^T x <= tau  for l in F_i,

    whose optimal value is the cell's minimal aspect ratio.  Solved with scipy's
    HiGHS dual simplex, then polished to the exact vertex by solving the active
    constraints as a linear system.
    """
    ell = T.shape[1]
    Tn = T[np.asarray(near_i, dtype=np.int64)]
    Tf = T[np.asarray(far_i, dtype=np.int64)] * sigma[:, None]      # rows sigma_l t_l^T
    nf = Tf.shape[0]
    # variables y = (x_1..x_ell, tau); objective tau
    c = np.zeros(ell + 1)
    c[-1] = 1.0
    A_ub = np.vstack([np.hstack([-Tf, np.zeros((nf, 1))]),          # -sigma t^T x <= -1
                      np.hstack([Tf, -np.ones((nf, 1))])])            # sigma t^T x - tau <= 0
    b_ub = np.concatenate([-np.ones(nf), np.zeros(nf)])
    A_eq = np.hstack([Tn, np.zeros((Tn.shape[0], 1))])
    b_eq = np.zeros(Tn.shape[0])
    res = linprog(c, A_ub=A_ub, b_ub=b_ub, A_eq=A_eq, b_eq=b_eq,
                  bounds=[(None, None)] * (ell + 1), method="highs-ds")
    if res.status != 0:
        return None
    y = res.x
    # Vertex polish: the optimum is the solution of its active constraints.
    slack = b_ub - A_ub @ y
    act = slack <= 1e-7 * max(1.0, abs(y[-1]))
    M = np.vstack([A_eq, A_ub[act]])
    rhs = np.concatenate([b_eq, b_ub[act]])
    if np.linalg.matrix_rank(M) == ell + 1:
        y2 = np.linalg.lstsq(M, rhs, rcond=None)[0]
        if np.max(A_ub @ y2 - b_ub) <= 1e-9 * max(1.0, abs(y2[-1])) and \
                np.max(np.abs(A_eq @ y2)) <= 1e-9 * max(1.0, np.max(np.abs(y2))):
            y = y2
    return y[:ell], float(y[-1])


def optimise_tag_vector(T: np.ndarray, near_i, far_i, optimise: bool = True):
    """Unit tag vector z^(i) in null(T(N_i,:)) with small aspect ratio (Alg. 2; Section 5.3).

    Reading (the paper leaves the optimiser unspecified; it calls the problem a
    small constrained optimisation over a convex region):
      * starts are the orthogonal projections of e_1..e_ell onto the null space
        (a choice independent of how the null space basis is computed);
      * each start fixes a sign cell; the cell's optimum is an LP (_lp_in_cell);
      * the best cell wins; values within a relative 1e-9 are ties, resolved by
        the lowest start index;
      * z is normalised to unit length with canonical_sign.
    With ``optimise=False`` the first nonzero start is used as is.
    Returns (z, rho).
    """
    ell = T.shape[1]
    X = null_space(T[np.asarray(near_i, dtype=np.int64)])
    if X.shape[1] == 0:
        raise ValueError("tag submatrix has a trivial null space")
    P = X @ X.T
    starts = []
    for j in range(ell):
        w = P[:, j]
        if np.linalg.norm(w) > 1e-12:
            starts.append(w / np.linalg.norm(w))
    if not optimise:
        z = canonical_sign(starts[0])
        return z, aspect_ratio(T, far_i, z)
    best = None
    seen = {}
    Tf = T[np.asarray(far_i, dtype=np.int64)]
    for idx, w in enumerate(starts):
        sig = np.sign(Tf @ w)
        if np.any(sig == 0):
            continue
        if sig[0] < 0:          # sigma and -sigma are the same cell up to sign
            sig = -sig
        key = sig.tobytes()
        if key in seen:
            continue
        sol = _lp_in_cell(T, near_i, far_i, sig)
        seen[key] = sol
        if sol is None:
            continue
        x, tau = sol
        if best is None or tau < best[1] * (1.0 - 1e-9):
            best = (x, tau)
    if best is None:
        z = canonical_sign(starts[0])
        return z, aspect_ratio(T, far_i, z)
    z = best[0] / np.linalg.norm(best[0])
    z = canonical_sign(z)
    return z, aspect_ratio(T, far_i, z)


def tag_plan(T: np.ndarray, near, far, optimise: bool = True):
    """Tag vectors z (b x ell) and aspect ratios rho (b) for every box."""
    b, ell = T.shape
    z = np.zeros((b, ell))
    rho = np.zeros(b)
    for i in range(b):
        z[i], rho[i] = optimise_tag_vector(T, near[i], far[i], optimise)
    return z, rho


# ---------------------------------------------------------------------------
# Post-processing and bases (Alg. 2 loop over boxes; Section 2.3 col)
# ---------------------------------------------------------------------------

def tag_postprocess(Y: np.ndarray, z: np.ndarray, box_ptr: np.ndarray, r: int) -> np.ndarray:
    """Yhat(I_i,:) = sum_j z^(i)_j Y_j(I_i,:) for every box i (Alg. 2; eq. projected_tags)."""
    b, ell = z.shape
    out = np.zeros((Y.shape[0], r))
    for i in range(b):
        rows = slice(int(box_ptr[i]), int(box_ptr[i + 1]))
        for j in range(ell):
            out[rows] += z[i, j] * Y[rows, j * r:(j + 1) * r]
    return out


def col_topk(M: np.ndarray, k: int) -> np.ndarray:
    """col(M, k): k orthonormal columns spanning the dominant range of M (Section 2.3).

    Reading: the k dominant left singular vectors of the r-column sample (the
    randomized range finder of Section 2.4 truncated to rank k), with the sign
    of each column fixed so that its entry of largest magnitude (lowest row on
    ties) is positive.
    """
    u, _, _ = np.linalg.svd(M, full_matrices=False)
    u = u[:, :k].copy()
    for c in range(u.shape[1]):
        q = int(np.argmax(np.abs(u[:, c])))
        if u[q, c] < 0:
            u[:, c] = -u[:, c]
    return u


def tag_bases(Yhat: np.ndarray, Zhat: np.ndarray, box_ptr: np.ndarray, k: int):
    """U_i = col(Yhat(I_i,:), k), V_i = col(Zhat(I_i,:), k), stacked as N x k (Alg. 2)."""
    n = Yhat.shape[0]
    U = np.zeros((n, k))
    V = np.zeros((n, k))
    for i in range(len(box_ptr) - 1):
        rows = slice(int(box_ptr[i]), int(box_ptr[i + 1]))
        U[rows] = col_topk(Yhat[rows], k)
        V[rows] = col_topk(Zhat[rows], k)
    return U, V
