"""Alg. 3 (basic randomized SVD for basis construction) in plain FP64 (oracle;
test infrastructure only).

The paper's benchmark for step (I) of Table 1: for every box i, a Gaussian
test matrix with the rows of every neighbour box zeroed is applied to A (and
another to A*), and the bases are col(Y(I_i,:), k) and col(Z(I_i,:), k) of the
box's own rows.  Steps (II)-(III) of Table 1 follow unchanged.

Reading (stated once here): the test matrices of different boxes are drawn
from one N x r Gaussian G (one H for the adjoint side) and masked per box:
Omega^(i) = G with G(I_j,:) = 0 for j in N_i.  Box i's sample only involves
the far rows of its own test matrix, so every basis sees an N(0,1) test
matrix on its far field, exactly as in Alg. 3; only independence between the
samples of different boxes is dropped, and no output depends on it.
"""
from __future__ import annotations

import numpy as np

from . import admissibility
from .reconstruct import cores, nearfield_probes
from .tagging import col_topk


def masked_test_matrix(G: np.ndarray, box_ptr: np.ndarray, near_i) -> np.ndarray:
    """Omega^(i): G with the rows of every box in N_i set to zero (Alg. 3)."""
    Om = np.array(G, dtype=np.float64, copy=True)
    for j in near_i:
        Om[int(box_ptr[j]):int(box_ptr[j + 1])] = 0.0
    return Om


def basic_bases(op, G: np.ndarray, H: np.ndarray, box_ptr, near, k: int):
    """[U, V] = basic(A, A*, k) of Alg. 3: one product with A and one with A* per box,
    each on r columns (2 b r columns in all), then U_i = col(Y(I_i,:), k) and
    V_i = col(Z(I_i,:), k).  Returns (U, V, SY, SZ) with SY, SZ the stacked samples
    Y^(i)(I_i,:), Z^(i)(I_i,:)."""
    box_ptr = np.asarray(box_ptr, dtype=np.int64)
    n, r = G.shape
    SY = np.zeros((n, r))
    SZ = np.zeros((n, r))
    U = np.zeros((n, k))
    V = np.zeros((n, k))
    for i in range(len(box_ptr) - 1):
        rows = slice(int(box_ptr[i]), int(box_ptr[i + 1]))
        Y = op.matmat(masked_test_matrix(G, box_ptr, near[i]))
        Z = op.rmatmat(masked_test_matrix(H, box_ptr, near[i]))
        SY[rows] = Y[rows]
        SZ[rows] = Z[rows]
        U[rows] = col_topk(SY[rows], k)
        V[rows] = col_topk(SZ[rows], k)
    return U, V, SY, SZ


def reconstruct_basic(op, box_ptr, lattice, k: int, p: int, G, H, steps=("I", "II", "III"),
                      near=None):
    """Alg. 3 for step (I), then Atil = U*(A V) and B by probes (Table 1, steps (II)-(III)).

    G, H must be N x (k+p).  ``near``: optional neighbour lists replacing the lattice
    rule (probe colours then greedy).  Returns a dict with every intermediate.
    """
    box_ptr = np.asarray(box_ptr, dtype=np.int64)
    b = len(box_ptr) - 1
    r = k + p
    near, col = admissibility.lists_and_colours(lattice, near)
    far = admissibility.far_lists(near, b)
    assert G.shape == (int(box_ptr[-1]), r) and H.shape == G.shape
    out = dict(near=near, far=far, colour=col, r=r, k=k)
    U, V, SY, SZ = basic_bases(op, G, H, box_ptr, near, k)
    out.update(U=U, V=V, SY=SY, SZ=SZ)
    if "II" in steps:
        out["Atil"] = cores(op, U, V, box_ptr, k)
    if "III" in steps:
        out["B"] = nearfield_probes(op, U, V, out["Atil"], box_ptr, near, col, k)
    return out
