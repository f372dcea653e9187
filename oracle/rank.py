"""Tolerance-driven choice of the uniform rank k (oracle; test infrastructure only).

The paper fixes k for its comparisons and notes that larger ranks can be chosen and
truncated as needed, or chosen adaptively with a tolerance (Section 2.3, Section 6).
Reading (stated once here): sketch once at r columns, take the singular values of every
box's post-processed samples Yhat_i and Zhat_i, and pick the smallest uniform k that keeps
every singular value above tol times the largest one of the same side over all boxes:
k = max over boxes and sides of #{j : sigma_j(Yhat_i) > tol * max_l sigma_1(Yhat_l)}.
k = r means the tolerance was not reached within the sample.
"""
from __future__ import annotations

import numpy as np


def box_singular_values(S: np.ndarray, box_ptr) -> np.ndarray:
    """b x r: the singular values (descending) of every m_i x r block of S."""
    box_ptr = np.asarray(box_ptr, dtype=np.int64)
    return np.stack([np.linalg.svd(S[box_ptr[i]:box_ptr[i + 1]], compute_uv=False)
                     for i in range(len(box_ptr) - 1)])


def rank_for_tolerance(sig_y: np.ndarray, sig_z: np.ndarray, tol: float) -> int:
    """The uniform rank of the reading above from the two b x r singular-value tables."""
    k = 0
    for sig in (sig_y, sig_z):
        top = float(np.max(sig[:, 0]))
        if top > 0.0:
            k = max(k, int(np.max(np.sum(sig > tol * top, axis=1))))
    return k
