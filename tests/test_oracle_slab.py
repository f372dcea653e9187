"""Pins of the thin-slab Schur-complement operator (oracle/slab.py, Section 7.2).

* The Schur complement of a tiny slab equals A_ff - A_fi inv(A_ii) A_if formed densely from a
  matrix assembled by plain loops over grid points and their six neighbours.
* A one-plane slab (l = 1) has nothing to eliminate: S is the plane's own 5-point block with
  6 - (kappa h)^2 on the diagonal.
* Separation of variables: the eigenvalues of S are, for every pair of in-plane sine modes
  (p, q), the last pivot of the tridiagonal z-line matrix with diagonal
  2 + 4 sin^2(pi p / (2 (n+1))) + 4 sin^2(pi q / (2 (n+1))) - (kappa h)^2 and off-diagonal -1.
* S is symmetric positive definite (the slab is thin: electrically small across), and the
  plan-order permutation acts as P S P^T.
"""
import math

import numpy as np
import pytest

from oracle import slab

KH = slab.KAPPA_H


def dense_slab(n, l, kh):
    """Dense 7-point matrix by loops (unknown x + n y + n^2 z)."""
    N3 = n * n * l
    A = np.zeros((N3, N3))
    for z in range(l):
        for y in range(n):
            for x in range(n):
                i = x + n * y + n * n * z
                A[i, i] = 6.0 - kh * kh
                for dx, dy, dz in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                    xx, yy, zz = x + dx, y + dy, z + dz
                    if 0 <= xx < n and 0 <= yy < n and 0 <= zz < l:
                        A[i, xx + n * yy + n * n * zz] = -1.0
    return A


@pytest.mark.parametrize("n,l", [(4, 3), (5, 4), (3, 6)])
def test_schur_complement_vs_dense(n, l):
    A = dense_slab(n, l, KH)
    f = np.arange(n * n * (l - 1), n * n * l)
    i = np.arange(0, n * n * (l - 1))
    S = A[np.ix_(f, f)] - A[np.ix_(f, i)] @ np.linalg.solve(A[np.ix_(i, i)], A[np.ix_(i, f)])
    op = slab.SlabOperator(n, l, np.arange(n * n), KH)
    assert np.max(np.abs(op.block() - S)) <= 1e-12 * np.max(np.abs(S))


def test_single_plane_is_the_frontal_block():
    n = 5
    op = slab.SlabOperator(n, 1, np.arange(n * n), KH)
    A2 = dense_slab(n, 1, KH)                     # one plane: the 5-point block itself
    assert np.array_equal(op.block(), A2)
    assert np.all(np.diag(A2) == 6.0 - KH * KH)


def test_eigenvalues_by_separation_of_variables():
    n, l = 6, 5
    S = slab.SlabOperator(n, l, np.arange(n * n), KH).block()
    ref = []
    for p in range(1, n + 1):
        for q in range(1, n + 1):
            d = 2.0 + 4 * math.sin(math.pi * p / (2 * (n + 1))) ** 2 + \
                4 * math.sin(math.pi * q / (2 * (n + 1))) ** 2 - KH * KH
            e = d
            for _ in range(l - 1):
                e = d - 1.0 / e
            ref.append(e)
    ev = np.linalg.eigvalsh(S)
    assert np.allclose(np.sort(ev), np.sort(ref), rtol=1e-12, atol=0)


def test_symmetric_positive_definite_and_permutation():
    n, l = 5, 4
    S = slab.SlabOperator(n, l, np.arange(n * n), KH).block()
    assert np.max(np.abs(S - S.T)) <= 1e-14 * np.max(np.abs(S))
    assert np.linalg.eigvalsh(S).min() > 0
    perm = np.random.default_rng(3).permutation(n * n)
    Sp = slab.SlabOperator(n, l, perm, KH).block()
    assert np.allclose(Sp, S[np.ix_(perm, perm)], atol=1e-14)
    x = np.random.default_rng(4).standard_normal((n * n, 3))
    opp = slab.SlabOperator(n, l, perm, KH)
    assert np.allclose(opp.matmat(x), Sp @ x, atol=1e-13)
