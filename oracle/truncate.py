"""Per-box ranks from a tolerance by truncating a computed uBLR (oracle; test
infrastructure only).

The paper fixes the rank k for its experiments and remarks that a rank can be chosen
larger than needed and the representation truncated afterwards (Section 6), and that
the randomized range finder can work to a tolerance instead of a rank (Section 2.4).
Reading (stated once here, identical in the library):

* Start from A_uBLR = U Atil V* + B (eq. uniformBLRfull) compressed at the plan's rank k,
  with U_i, V_j orthonormal.  Budget: (tol ||A_uBLR||_F)^2.
* Rows.  For every box i, X_i = Atil(i, F_i) (the k x |F_i| k far block row of the
  cores).  Its SVD X_i = W_i S_i Z_i* gives singular values s_i1 >= s_i2 >= ...  Over all
  boxes, drop the smallest singular values while their squares sum to at most half the
  budget; box i keeps k_i = its number of remaining values.  U'_i = U_i W_i(:, 1:k_i) and
  the block row becomes W_i(:, 1:k_i)* Atil(i, :).
* Columns.  On the row-truncated cores Atil1, for every box j, Y_j = Atil1(F_j, j) (the
  far block column).  Its right singular vectors J_j and values give, with the budget that
  the rows left, ranks kv_j the same way; V'_j = V_j J_j(:, 1:kv_j) and the block column
  becomes Atil1(:, j) J_j(:, 1:kv_j).
* Near pairs keep their represented block exactly:
  B'_ij = B_ij + U_i Atil_ij V_j* - U'_i Atil'_ij V'_j*.
* For far pairs the removed part is X - P X Q with P, Q orthogonal projectors, and
  ||X - P X Q||^2 = ||(I - P) X||^2 + ||P X (I - Q)||^2 (the cross term vanishes), so the
  change of the representation is exactly the dropped squares: at most the budget.

Storage keeps the uniform layout: U', V' are N x k with the columns beyond k_i zero and
Atil' is bk x bk with the matching rows and columns zero.
"""
from __future__ import annotations

import numpy as np


def _drop_count(sig: np.ndarray, budget: float):
    """Ranks per box (rows of ``sig``, each descending) after dropping the globally
    smallest values while the sum of their squares stays <= budget."""
    b, k = sig.shape
    flat = sorted((float(sig[i, j]) ** 2, i, j) for i in range(b) for j in range(k))
    ranks = np.full(b, k, dtype=np.int64)
    dropped = 0.0
    for s2, i, j in flat:
        if dropped + s2 > budget:
            break
        dropped += s2
        ranks[i] -= 1
    return ranks, dropped


def representation_norm(U, V, Atil, B, box_ptr, near, k: int) -> float:
    """||U Atil V* + B||_F, block by block (far blocks: ||Atil_ij||_F, U and V orthonormal)."""
    b = len(box_ptr) - 1
    tot = 0.0
    for i in range(b):
        ri = slice(int(box_ptr[i]), int(box_ptr[i + 1]))
        for j in range(b):
            blk = Atil[i * k:(i + 1) * k, j * k:(j + 1) * k]
            if j in near[i]:
                cj = slice(int(box_ptr[j]), int(box_ptr[j + 1]))
                tot += float(np.sum((U[ri] @ blk @ V[cj].T + B[(i, j)]) ** 2))
            else:
                tot += float(np.sum(blk * blk))
    return float(np.sqrt(tot))


def truncate_ublr(U, V, Atil, B, box_ptr, near, far, k: int, tol: float):
    """The truncation of the reading above.  Returns a dict with U, V, Atil, B (new
    arrays), ranks_u, ranks_v, sig_row, sig_col (b x k, descending), norm (||A_uBLR||_F
    before truncation) and dropped (the sum of the dropped squares)."""
    box_ptr = np.asarray(box_ptr, dtype=np.int64)
    b = len(box_ptr) - 1
    norm = representation_norm(U, V, Atil, B, box_ptr, near, k)
    budget = (tol * norm) ** 2
    # rows: left singular vectors of the far block rows
    W = np.zeros((b, k, k))
    sig_row = np.zeros((b, k))
    for i in range(b):
        X = np.hstack([Atil[i * k:(i + 1) * k, j * k:(j + 1) * k] for j in far[i]])
        Wi, s, _ = np.linalg.svd(X, full_matrices=True)
        W[i] = Wi
        sig_row[i, :len(s)] = s
    ku, drop_u = _drop_count(sig_row, 0.5 * budget)
    A1 = np.zeros_like(Atil)
    U2 = np.zeros_like(U)
    for i in range(b):
        Wk = W[i][:, :ku[i]]
        A1[i * k:i * k + ku[i], :] = Wk.T @ Atil[i * k:(i + 1) * k, :]
        ri = slice(int(box_ptr[i]), int(box_ptr[i + 1]))
        U2[ri, :ku[i]] = U[ri] @ Wk
    # columns: right singular vectors of the far block columns of the row-truncated cores
    J = np.zeros((b, k, k))
    sig_col = np.zeros((b, k))
    for j in range(b):
        Y = np.vstack([A1[i * k:(i + 1) * k, j * k:(j + 1) * k] for i in far[j]])
        _, s, Jt = np.linalg.svd(Y, full_matrices=True)
        J[j] = Jt.T
        sig_col[j, :len(s)] = s
    kv, drop_v = _drop_count(sig_col, budget - drop_u)
    A2 = np.zeros_like(Atil)
    V2 = np.zeros_like(V)
    for j in range(b):
        Jk = J[j][:, :kv[j]]
        A2[:, j * k:j * k + kv[j]] = A1[:, j * k:(j + 1) * k] @ Jk
        cj = slice(int(box_ptr[j]), int(box_ptr[j + 1]))
        V2[cj, :kv[j]] = V[cj] @ Jk
    B2 = {}
    for (i, j), Bij in B.items():
        ri = slice(int(box_ptr[i]), int(box_ptr[i + 1]))
        cj = slice(int(box_ptr[j]), int(box_ptr[j + 1]))
        old = U[ri] @ Atil[i * k:(i + 1) * k, j * k:(j + 1) * k] @ V[cj].T
        new = U2[ri] @ A2[i * k:(i + 1) * k, j * k:(j + 1) * k] @ V2[cj].T
        B2[(i, j)] = Bij + old - new
    return dict(U=U2, V=V2, Atil=A2, B=B2, ranks_u=ku, ranks_v=kv, sig_row=sig_row, sig_col=sig_col,
                norm=norm, dropped=drop_u + drop_v)
