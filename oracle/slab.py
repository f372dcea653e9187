"""Schur complement of a thin slab of the 3D Helmholtz finite-difference operator, the
paper's second black box (Section 7.2, eq. bvp) (oracle; test infrastructure only).

Reading (stated once here, identical in the library):

* Grid: n x n x l points (x, y in the plane of the slab, z across it), spacing h = 1,
  unknown u(x, y, z) for 0 <= x, y < n and 0 <= z < l, zero Dirichlet values outside.
* Operator: second-order finite differences of -Laplace(u) - kappa^2 u, i.e. 6 - (kappa h)^2
  on the diagonal and -1 for each of the six grid neighbours inside the grid.  The paper keeps
  100 points per wavelength: kappa h = 2 pi / 100.
* Frontal nodes: the face z = l - 1 (N = n^2 unknowns, plane index x + n y); internal nodes:
  the planes z = 0 .. l - 2.  The operator is the Schur complement
  S = A_ff - A_fi A_ii^{-1} A_if (dense N x N, symmetric), applied to vectors with a sparse LU
  factorisation of A_ii (the "sparsity of its components").
* The rows of a compression plan are the frontal nodes in the plan's box-major order:
  ``perm[row]`` is the plane index of plan row ``row``.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

KAPPA_H = 2.0 * math.pi / 100.0


def slab_matrix(n: int, l: int, kappa_h: float = KAPPA_H) -> sp.csr_matrix:
    """The 7-point finite-difference matrix of -Laplace - kappa^2 on the n x n x l grid,
    unknowns numbered x + n y + n^2 z."""
    N3 = n * n * l
    idx = np.arange(N3)
    x = idx % n
    y = (idx // n) % n
    z = idx // (n * n)
    rows = [idx]
    cols = [idx]
    vals = [np.full(N3, 6.0 - kappa_h * kappa_h)]
    for d, coord, lim in ((1, x, n), (n, y, n), (n * n, z, l)):
        for sgn in (-1, 1):
            ok = (coord + sgn >= 0) & (coord + sgn < lim)
            rows.append(idx[ok])
            cols.append(idx[ok] + sgn * d)
            vals.append(np.full(int(ok.sum()), -1.0))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(N3, N3))


class SlabOperator:
    """S = A_ff - A_fi A_ii^{-1} A_if on the frontal face, rows in plan order via ``perm``."""

    symmetric = True

    def __init__(self, n: int, l: int, perm, kappa_h: float = KAPPA_H):
        self.nx, self.l, self.kappa_h = n, l, kappa_h
        self.n = n * n
        self.perm = np.asarray(perm, dtype=np.int64)
        assert np.array_equal(np.sort(self.perm), np.arange(self.n))
        A = slab_matrix(n, l, kappa_h).tocsc()
        front = np.arange(n * n * (l - 1), n * n * l)
        inner = np.arange(0, n * n * (l - 1))
        self.A_ff = A[front][:, front].tocsr()
        if l > 1:
            self.A_fi = A[front][:, inner].tocsr()
            self.A_if = A[inner][:, front].tocsr()
            self.lu = spla.splu(A[inner][:, inner].tocsc())
        else:
            self.lu = None

    def _apply_plane(self, Xp: np.ndarray) -> np.ndarray:
        Y = self.A_ff @ Xp
        if self.lu is not None:
            Y = Y - self.A_fi @ self.lu.solve(np.asarray(self.A_if @ Xp))
        return Y

    def matmat(self, X: np.ndarray, rows=None) -> np.ndarray:
        """(S X)(rows, :) with X and the result in plan row order."""
        X2 = X.reshape(X.shape[0], -1)
        Xp = np.zeros_like(X2)
        Xp[self.perm] = X2
        Y = self._apply_plane(Xp)[self.perm]
        Y = Y if rows is None else Y[np.asarray(rows)]
        return Y.reshape(Y.shape[0], *X.shape[1:]) if X.ndim == 1 else Y

    def rmatmat(self, X: np.ndarray, rows=None) -> np.ndarray:
        return self.matmat(X, rows)        # S is symmetric

    def block(self, rows=None, cols=None) -> np.ndarray:
        """Entries S(rows, cols) in plan order (evaluation harness): S applied to unit vectors
        of the requested columns, or, when fewer rows than columns are asked for, to those
        of the rows (S is symmetric, so S(rows, cols) = S(cols, rows)^T)."""
        r = np.arange(self.n) if rows is None else np.atleast_1d(np.asarray(rows))
        c = np.arange(self.n) if cols is None else np.atleast_1d(np.asarray(cols))
        small, other, transpose = (r, c, True) if r.size < c.size else (c, r, False)
        E = np.zeros((self.n, small.size))
        E[small, np.arange(small.size)] = 1.0
        Sx = self.matmat(E)[other]
        return Sx.T if transpose else Sx
