"""Black-box operators for the oracle (test infrastructure only).

The method only ever touches A through products X -> A X and X -> A* X
(Section 1; Section 3 opening).  The oracle's operators expose exactly those
two products; ``block`` (entry access) is a harness privilege used only to
build test matrices, to evaluate exact errors and to sample parity outputs.

Kernel matrices (Section 7.1 and the workloads built on it):
    log   : A_ij = log |x_i - x_j|,              diagonal 0   (Section 7.1)
    inv_r : A_ij = 1 / |x_i - x_j|,              diagonal 0   (reading, by analogy)
    exp   : A_ij = exp(-|x_i - x_j| / 0.1),      diagonal 1   (the limit)
    cos   : A_ij = cos(20 |x_i - x_j|) / (|x_i - x_j| + 1e-3), diagonal 1000 (the limit)
The diagonal rule applies where the row and column index coincide.
"""
from __future__ import annotations

import numpy as np

KERNELS = ("log", "inv_r", "exp", "cos")
DIAG = {"log": 0.0, "inv_r": 0.0, "exp": 1.0, "cos": 1000.0}


def kernel_values(kind: str, dist: np.ndarray) -> np.ndarray:
    """kappa(|x - y|) for the kernel ``kind``, off-diagonal formula."""
    with np.errstate(divide="ignore", invalid="ignore"):
        if kind == "log":
            return np.log(dist)
        if kind == "inv_r":
            return 1.0 / dist
        if kind == "exp":
            return np.exp(-dist / 0.1)
        if kind == "cos":
            return np.cos(20.0 * dist) / (dist + 1e-3)
    raise ValueError(f"unknown kernel {kind}")


def _as_index(ix, n):
    if ix is None:
        return np.arange(n)
    if isinstance(ix, slice):
        return np.arange(n)[ix]
    return np.asarray(ix, dtype=np.int64)


class DenseOperator:
    """A held as a dense matrix; products by plain matmul."""

    symmetric = False

    def __init__(self, A: np.ndarray):
        self.A = np.asarray(A, dtype=np.float64)
        self.n = self.A.shape[0]

    def block(self, rows=None, cols=None) -> np.ndarray:
        r = _as_index(rows, self.n)
        c = _as_index(cols, self.n)
        return self.A[np.ix_(r, c)]

    def matmat(self, X: np.ndarray, rows=None) -> np.ndarray:
        """(A X)(rows, :)."""
        if rows is None:
            return self.A @ X
        return self.A[_as_index(rows, self.n), :] @ X

    def rmatmat(self, X: np.ndarray, rows=None) -> np.ndarray:
        """(A* X)(rows, :)."""
        if rows is None:
            return self.A.T @ X
        return self.A[:, _as_index(rows, self.n)].T @ X


class KernelOperator:
    """A_ij = kappa(x_i, x_j) on a point cloud, never stored whole.

    Products are evaluated row-chunk by row-chunk: each chunk of rows of A is
    generated from the points and multiplied by X.  Every output row is the
    same dot product as in the definition (A X)(i,:) = sum_j A_ij X(j,:).
    """

    symmetric = True

    def __init__(self, kind: str, pts: np.ndarray, chunk: int = 1024):
        if kind not in KERNELS:
            raise ValueError(kind)
        self.kind = kind
        self.pts = np.asarray(pts, dtype=np.float64)
        self.n = self.pts.shape[0]
        self.chunk = chunk

    def block(self, rows=None, cols=None) -> np.ndarray:
        r = _as_index(rows, self.n)
        c = _as_index(cols, self.n)
        diff = self.pts[r][:, None, :] - self.pts[c][None, :, :]
        dist = np.sqrt(np.sum(diff * diff, axis=2))
        vals = kernel_values(self.kind, dist)
        same = r[:, None] == c[None, :]
        vals[same] = DIAG[self.kind]
        return vals

    def matmat(self, X: np.ndarray, rows=None) -> np.ndarray:
        r = _as_index(rows, self.n)
        out = np.empty((r.size, X.shape[1]))
        for s in range(0, r.size, self.chunk):
            rr = r[s:s + self.chunk]
            out[s:s + rr.size] = self.block(rr, None) @ X
        return out

    def rmatmat(self, X: np.ndarray, rows=None) -> np.ndarray:
        # kappa depends on |x - y| only, so A* = A.
        return self.matmat(X, rows)


class CountingOperator:
    """Wraps an operator and counts the columns applied to A and to A*."""

    def __init__(self, op):
        self.op = op
        self.n = op.n
        self.symmetric = getattr(op, "symmetric", False)
        self.cols_A = 0
        self.cols_At = 0

    def block(self, rows=None, cols=None):
        return self.op.block(rows, cols)

    def matmat(self, X, rows=None):
        self.cols_A += X.shape[1]
        return self.op.matmat(X, rows)

    def rmatmat(self, X, rows=None):
        self.cols_At += X.shape[1]
        return self.op.rmatmat(X, rows)
