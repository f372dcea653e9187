"""Alg. 1 (block nullification for basis construction) in plain FP64 (oracle; test
infrastructure only).

One sketch Y = A Omega, Z = A* Psi with s >= r + max_i |rows of N_i| Gaussian columns
(Section 3.1; s >= r + 3^d m on a uniform tessellation).  For every box i the
rows of Omega that belong to the neighbours of i form Omega^(i); P^(i) holds r
orthonormal vectors of null(Omega^(i)), so Y(I_i,:) P^(i) only sees the far field,
and U_i = col(Y(I_i,:) P^(i), k).  V_i likewise from Z and Psi.

Reading (stated once here): null(Omega^(i), r) is taken from the Householder QR of
Omega^(i)* whose reflectors use the sign that avoids cancellation (Section 3.2 costs
the null spaces as Householder QRs): P^(i) = the r columns of the full orthogonal
factor that follow its first |rows of N_i| columns.  Omega^(i) stacks the rows of
the neighbour boxes in ascending box order, each box's rows in row order.
"""
from __future__ import annotations

import numpy as np

from . import admissibility
from .reconstruct import cores, nearfield_probes
from .tagging import col_topk


def bn_columns(box_ptr, near, r: int) -> int:
    """The smallest s for which every null(Omega^(i)) has r dimensions:
    r + max_i sum_{j in N_i} m_j (Alg. 1 asks for s >= r + 3^d m)."""
    sizes = np.diff(np.asarray(box_ptr, dtype=np.int64))
    return int(r + max(int(sizes[list(n)].sum()) for n in near))


def neighbour_rows(box_ptr, near_i) -> np.ndarray:
    """Row indices of the boxes in N_i, ascending box order (the rows of Omega^(i))."""
    return np.concatenate([np.arange(int(box_ptr[j]), int(box_ptr[j + 1])) for j in sorted(near_i)])


def null_r(M: np.ndarray, r: int) -> np.ndarray:
    """null(M, r) for M (n x s, n + r <= s): the r columns after the first n of the
    orthogonal factor of the Householder QR of M* (LAPACK's reflector signs)."""
    n, s = M.shape
    assert n + r <= s
    Q, _ = np.linalg.qr(M.T, mode="complete")
    return Q[:, n:n + r].copy()


def bn_bases(op, Omega: np.ndarray, Psi: np.ndarray, box_ptr, near, k: int, r: int):
    """[U, V] = bn(A, A*, k) of Alg. 1.  Returns (U, V, SY, SZ) with SY, SZ the
    stacked projected samples Y(I_i,:) P^(i), Z(I_i,:) Q^(i)."""
    box_ptr = np.asarray(box_ptr, dtype=np.int64)
    n = Omega.shape[0]
    Y = op.matmat(Omega)
    Z = op.rmatmat(Psi)
    SY = np.zeros((n, r))
    SZ = np.zeros((n, r))
    U = np.zeros((n, k))
    V = np.zeros((n, k))
    for i in range(len(box_ptr) - 1):
        rows = slice(int(box_ptr[i]), int(box_ptr[i + 1]))
        nr = neighbour_rows(box_ptr, near[i])
        P = null_r(Omega[nr], r)
        Q = null_r(Psi[nr], r)
        SY[rows] = Y[rows] @ P
        SZ[rows] = Z[rows] @ Q
        U[rows] = col_topk(SY[rows], k)
        V[rows] = col_topk(SZ[rows], k)
    return U, V, SY, SZ


def reconstruct_bn(op, box_ptr, lattice, k: int, p: int, Omega, Psi, steps=("I", "II", "III"),
                   near=None):
    """Alg. 1 for step (I), then Atil = U*(A V) and B by probes (Table 1, steps (II)-(III)).

    Omega, Psi must be N x s with s >= bn_columns(box_ptr, near, k + p).  ``near``:
    optional neighbour lists replacing the lattice rule (probe colours then greedy)."""
    box_ptr = np.asarray(box_ptr, dtype=np.int64)
    b = len(box_ptr) - 1
    r = k + p
    near, col = admissibility.lists_and_colours(lattice, near)
    far = admissibility.far_lists(near, b)
    assert Omega.shape == Psi.shape and Omega.shape[0] == int(box_ptr[-1])
    assert Omega.shape[1] >= bn_columns(box_ptr, near, r)
    out = dict(near=near, far=far, colour=col, r=r, k=k, s=Omega.shape[1])
    U, V, SY, SZ = bn_bases(op, Omega, Psi, box_ptr, near, k, r)
    out.update(U=U, V=V, SY=SY, SZ=SZ)
    if "II" in steps:
        out["Atil"] = cores(op, U, V, box_ptr, k)
    if "III" in steps:
        out["B"] = nearfield_probes(op, U, V, out["Atil"], box_ptr, near, col, k)
    return out
