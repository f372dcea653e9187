"""Mixed-precision tagging with one FP64 refinement sketch (oracle; test
infrastructure only).

Not in the paper: the paper runs every step in one precision.  The design
reading (stated once here, used by every function below):

1. The tagged sketches of Alg. 2 are taken with ``r_lo = k + p_lo`` columns per
   tag column (on the GPU in BF16 or FP32; here in FP64, the oracle's precision),
   post-processed as in Alg. 2, and turned into orthonormal bases ``U0_i``,
   ``V0_i`` of all ``r_lo`` sample columns (Householder QR, each column signed so
   that its largest-magnitude entry is positive).
2. One FP64 refinement sketch: with r_lo x r Gaussian blocks ``Gv_l``, ``Gu_l``
   per box, the test blocks are ``Vt_l = V0_l Gv_l`` and ``Ut_l = U0_l Gu_l``,
   and the far-field samples are
       SY(I_i) = sum_{l in F_i} A(I_i, I_l) Vt_l,
       SZ(I_i) = sum_{l in F_i} A(I_l, I_i)* Ut_l,
   i.e. the far-field block row of box i applied to a test matrix whose block l
   lies in the span of V0_l (one half-step of subspace iteration).
3. ``U_i = col(SY(I_i), k)`` and ``V_i = col(SZ(I_i), k)`` (the same ``col`` as
   Alg. 2), then steps (II)-(III) of Table 1 unchanged.
The far-field samples use block access to A (``2 b r`` columns of block-sparse
products for a black box), the same access the cores of Table 1 step (II) use.
"""
from __future__ import annotations

import numpy as np

from . import admissibility, tagging
from .reconstruct import cores, nearfield_probes


def sample_basis(S: np.ndarray) -> np.ndarray:
    """Orthonormal basis of the columns of an m x c sample (c <= m): the Q factor of
    a QR factorisation, each column signed so that its entry of largest magnitude
    (lowest row on ties) is positive."""
    q, _ = np.linalg.qr(S, mode="reduced")
    q = q.copy()
    for c in range(q.shape[1]):
        i = int(np.argmax(np.abs(q[:, c])))
        if q[i, c] < 0:
            q[:, c] = -q[:, c]
    return q


def sample_bases(Shat: np.ndarray, box_ptr: np.ndarray) -> np.ndarray:
    """Per-box ``sample_basis`` of a stacked N x c sample."""
    out = np.zeros_like(Shat)
    for i in range(len(box_ptr) - 1):
        rows = slice(int(box_ptr[i]), int(box_ptr[i + 1]))
        out[rows] = sample_basis(Shat[rows])
    return out


def mixed_test_blocks(Q0: np.ndarray, gamma: np.ndarray, box_ptr: np.ndarray) -> np.ndarray:
    """Stacked N x r test blocks X(I_l) = Q0(I_l) gamma[l] (gamma: b x r_lo x r)."""
    b = len(box_ptr) - 1
    out = np.zeros((Q0.shape[0], gamma.shape[2]))
    for l in range(b):
        rows = slice(int(box_ptr[l]), int(box_ptr[l + 1]))
        out[rows] = Q0[rows] @ gamma[l]
    return out


def far_sample(op, X: np.ndarray, box_ptr: np.ndarray, far, adjoint: bool = False) -> np.ndarray:
    """S(I_i) = sum_{l in F_i} A(I_i, I_l) X(I_l), or with A(I_l, I_i)* when ``adjoint``."""
    b = len(box_ptr) - 1
    S = np.zeros_like(X)
    for i in range(b):
        ri = np.arange(int(box_ptr[i]), int(box_ptr[i + 1]))
        for l in far[i]:
            rl = np.arange(int(box_ptr[l]), int(box_ptr[l + 1]))
            blk = op.block(rl, ri).T if adjoint else op.block(ri, rl)
            S[ri] += blk @ X[rl]
    return S


def refine_bases(op, U0, V0, gamma_u, gamma_v, box_ptr, far, k: int):
    """Steps 2-3 of the reading above: far-field samples on the mixed test blocks and
    their rank-k column spaces.  Returns (U, V, SY, SZ)."""
    Vt = mixed_test_blocks(V0, gamma_v, box_ptr)
    Ut = mixed_test_blocks(U0, gamma_u, box_ptr)
    SY = far_sample(op, Vt, box_ptr, far)
    SZ = far_sample(op, Ut, box_ptr, far, adjoint=True)
    U, V = tagging.tag_bases(SY, SZ, box_ptr, k)
    return U, V, SY, SZ


def reconstruct_tag_refined(op, box_ptr, lattice, k: int, p: int, extra: int, T, G, H,
                            gamma_u, gamma_v, optimise: bool = True, near=None):
    """The mixed-precision pipeline with every step in FP64: Alg. 2 sketches with
    r_lo = G.shape[1] columns per tag column, post-processing, sample bases, one
    refinement sketch, then Table 1 steps (II)-(III).  ``p`` is the oversampling of
    the refinement (gamma blocks are r_lo x (k + p))."""
    box_ptr = np.asarray(box_ptr, dtype=np.int64)
    b = len(box_ptr) - 1
    r_lo = G.shape[1]
    near, col = admissibility.lists_and_colours(lattice, near)
    far = admissibility.far_lists(near, b)
    ell = admissibility.num_tag_columns(near, extra)
    assert T.shape == (b, ell) and H.shape == G.shape
    assert gamma_u.shape == (b, r_lo, k + p) and gamma_v.shape == gamma_u.shape
    z, rho = tagging.tag_plan(T, near, far, optimise)
    Y, Z = tagging.sketch(op, T, G, H, box_ptr)
    Yhat = tagging.tag_postprocess(Y, z, box_ptr, r_lo)
    Zhat = tagging.tag_postprocess(Z, z, box_ptr, r_lo)
    U0 = sample_bases(Yhat, box_ptr)
    V0 = sample_bases(Zhat, box_ptr)
    U, V, SY, SZ = refine_bases(op, U0, V0, gamma_u, gamma_v, box_ptr, far, k)
    Atil = cores(op, U, V, box_ptr, k)
    B = nearfield_probes(op, U, V, Atil, box_ptr, near, col, k)
    return dict(near=near, far=far, colour=col, ell=ell, z=z, rho=rho, Y=Y, Z=Z, Yhat=Yhat,
                Zhat=Zhat, U0=U0, V0=V0, SY=SY, SZ=SZ, U=U, V=V, Atil=Atil, B=B)
