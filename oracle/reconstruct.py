"""Steps (II)-(III) of uniform-BLR compression, the uBLR apply and error metrics
(oracle; test infrastructure only).

Representation (eq. uniformBLRfull): A ~ U Atil V* + B with U = diag(U_i),
V = diag(V_j) (stored stacked as N x k), Atil = U* A V dense (bk x bk) and B
block sparse on neighbour pairs (eq. discrepancymatrix), stored as a dict
{(i, j): m_i x m_j} for j in N_i.
"""
from __future__ import annotations

import numpy as np

from . import admissibility, tagging


def _blockdiag(S: np.ndarray, box_ptr: np.ndarray, k: int) -> np.ndarray:
    """diag(S_1, ..., S_b) as a dense N x bk matrix from the stacked N x k array."""
    b = len(box_ptr) - 1
    out = np.zeros((S.shape[0], b * k))
    for i in range(b):
        rows = slice(int(box_ptr[i]), int(box_ptr[i + 1]))
        out[rows, i * k:(i + 1) * k] = S[rows]
    return out


def cores(op, U: np.ndarray, V: np.ndarray, box_ptr: np.ndarray, k: int) -> np.ndarray:
    """Atil = U* (A V) with bk products by A (Table 1, reconstruct_tag step 2)."""
    Vbd = _blockdiag(V, box_ptr, k)
    W = op.matmat(Vbd)
    Ubd = _blockdiag(U, box_ptr, k)
    return Ubd.T @ W


def nearfield_probes(op, U, V, Atil, box_ptr, near, colour, k: int):
    """B from 3^d sparse identity probes (Table 1 step 3; eq. sparse_struct_ids).

    For each colour c, X_c (N x m_max) holds an identity block I_{m_l} in the
    rows of every box l of colour c; the probe is P_c = (A - U Atil V*) X_c and
    B_il = P_c(I_i, 1:m_l) for the neighbour l of box i that has colour c.
    Far boxes of colour c also contribute to P_c(I_i, :) through their (small)
    far-field residuals, exactly as in the paper's probe construction.
    """
    b = len(box_ptr) - 1
    n = int(box_ptr[-1])
    sizes = np.diff(box_ptr)
    mmax = int(np.max(sizes))
    B = {}
    Ubd = _blockdiag(U, box_ptr, k)
    Vbd = _blockdiag(V, box_ptr, k)
    for c in sorted(set(int(x) for x in colour)):
        X = np.zeros((n, mmax))
        for l in range(b):
            if colour[l] == c:
                X[int(box_ptr[l]):int(box_ptr[l + 1]), :sizes[l]] = np.eye(sizes[l])
        P = op.matmat(X) - Ubd @ (Atil @ (Vbd.T @ X))
        for i in range(b):
            for l in near[i]:
                if colour[l] == c:
                    B[(i, l)] = P[int(box_ptr[i]):int(box_ptr[i + 1]), :sizes[l]].copy()
    return B


def ublr_apply(U, V, Atil, B, box_ptr, k: int, x: np.ndarray, trans: bool = False) -> np.ndarray:
    """y = U (Atil (V* x)) + B x, or its transpose (eq. uniformBLRfull)."""
    Ubd = _blockdiag(U, box_ptr, k)
    Vbd = _blockdiag(V, box_ptr, k)
    x2 = x.reshape(x.shape[0], -1)
    if not trans:
        y = Ubd @ (Atil @ (Vbd.T @ x2))
    else:
        y = Vbd @ (Atil.T @ (Ubd.T @ x2))
    for (i, j), Bij in B.items():
        ri = slice(int(box_ptr[i]), int(box_ptr[i + 1]))
        cj = slice(int(box_ptr[j]), int(box_ptr[j + 1]))
        if not trans:
            y[ri] += Bij @ x2[cj]
        else:
            y[cj] += Bij.T @ x2[ri]
    return y.reshape(x.shape[0], *x.shape[1:]) if x.ndim == 1 else y


def dense_reconstruction(U, V, Atil, B, box_ptr, k: int) -> np.ndarray:
    """A_uBLR = U Atil V* + B as a dense matrix (small problems only)."""
    Ubd = _blockdiag(U, box_ptr, k)
    Vbd = _blockdiag(V, box_ptr, k)
    Ah = Ubd @ Atil @ Vbd.T
    for (i, j), Bij in B.items():
        Ah[int(box_ptr[i]):int(box_ptr[i + 1]), int(box_ptr[j]):int(box_ptr[j + 1])] += Bij
    return Ah


def rel_fro_error(op, U, V, Atil, B, box_ptr, k: int) -> float:
    """||A - A_uBLR||_F / ||A||_F, block by block with entry access (harness)."""
    b = len(box_ptr) - 1
    num = 0.0
    den = 0.0
    for i in range(b):
        ri = np.arange(int(box_ptr[i]), int(box_ptr[i + 1]))
        Arow = op.block(ri, None)
        for j in range(b):
            cj = slice(int(box_ptr[j]), int(box_ptr[j + 1]))
            Aij = Arow[:, cj]
            E = Aij - U[ri] @ Atil[i * k:(i + 1) * k, j * k:(j + 1) * k] @ V[cj].T
            if (i, j) in B:
                E = E - B[(i, j)]
            num += float(np.sum(E * E))
            den += float(np.sum(Aij * Aij))
    return float(np.sqrt(num / den))


def power_norm_estimate(apply, apply_t, n: int, x0: np.ndarray, iters: int = 20) -> float:
    """||M||_2 by the power method on M* M (Section 7: 20 iterations of the
    randomized power method).  Reading: start from the given Gaussian vector,
    x <- M* M x / ||M* M x||, and report ||M x|| for the final unit x."""
    x = x0 / np.linalg.norm(x0)
    est = 0.0
    for _ in range(iters):
        y = apply(x)
        est = float(np.linalg.norm(y))
        w = apply_t(y)
        nw = np.linalg.norm(w)
        if nw == 0.0:
            return 0.0
        x = w / nw
    return float(np.linalg.norm(apply(x))) if iters > 0 else est


def reconstruct_tag(op, box_ptr, lattice, k: int, p: int, extra: int, T, G, H,
                    optimise: bool = True, steps=("I", "II", "III"), near=None):
    """reconstruct_tag of Table 1: [U, V] = tag(A, A*, k); Atil = U*(A V); B by probes.

    ``T`` must have num_tag_columns(near, extra) columns and G, H must be N x (k+p).
    ``near``: optional neighbour lists replacing the lattice rule (probe colours then
    greedy).  Returns a dict with every intermediate.
    """
    box_ptr = np.asarray(box_ptr, dtype=np.int64)
    b = len(box_ptr) - 1
    r = k + p
    near, col = admissibility.lists_and_colours(lattice, near)
    far = admissibility.far_lists(near, b)
    ell = admissibility.num_tag_columns(near, extra)
    assert T.shape == (b, ell), (T.shape, (b, ell))
    assert G.shape == (int(box_ptr[-1]), r) and H.shape == G.shape
    out = dict(near=near, far=far, colour=col, ell=ell, r=r, k=k)
    z, rho = tagging.tag_plan(T, near, far, optimise)
    out.update(z=z, rho=rho)
    Y, Z = tagging.sketch(op, T, G, H, box_ptr)
    out.update(Y=Y, Z=Z)
    Yhat = tagging.tag_postprocess(Y, z, box_ptr, r)
    Zhat = tagging.tag_postprocess(Z, z, box_ptr, r)
    U, V = tagging.tag_bases(Yhat, Zhat, box_ptr, k)
    out.update(Yhat=Yhat, Zhat=Zhat, U=U, V=V)
    if "II" in steps:
        out["Atil"] = cores(op, U, V, box_ptr, k)
    if "III" in steps:
        out["B"] = nearfield_probes(op, U, V, out["Atil"], box_ptr, near, col, k)
    return out
