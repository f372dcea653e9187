"""blr_apply_noalloc (the allocation-free apply) against blr_apply through the C ABI.

Both run the same kernels with the same column split, so their results agree bit for
bit; each is also checked against the oracle's apply of the library's own factors
(1e-12 of the largest output entry).  Two calls in a row share the library's scratch
array, the second on a smaller problem with fewer vectors, so stale contents of the
array from the first call must not leak into the second.
"""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def _announce(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _handle(P, g, k, seed, kind):
    near = O.near_lists(g.lattice)
    ell = O.num_tag_columns(near, 3)
    T = W.tag_matrix(seed, g.nboxes, ell)
    G, H = W.gaussian_test_blocks(seed, g.n, k + 10)
    plan = P.Plan(g.box_ptr, g.lattice, k, T, p=10, extra_tag_cols=3)
    op = P.Operator.kernel(kind, g.pts)
    h, _ = P.compress(plan, op, P.colmajor(G), P.colmajor(H))
    return plan, op, h


def _factors(h, plan, g):
    U, V, At = (h.part(n).cpu().numpy() for n in ("U", "V", "Atil"))
    Bf = h.part("B").cpu().numpy()[:, 0]
    near_ptr, near_idx, _, boff = plan.lists()
    bp = g.box_ptr
    B = {}
    for i in range(g.nboxes):
        for q in range(near_ptr[i], near_ptr[i + 1]):
            j = int(near_idx[q])
            mi, mj = bp[i + 1] - bp[i], bp[j + 1] - bp[j]
            B[(i, j)] = Bf[boff[q]:boff[q] + mi * mj].reshape((mi, mj), order="F")
    return U, V, At, B


def test_noalloc_apply_matches_apply_twice():
    import torch
    import paper_2501_05528_amd as P
    cases = [("laplace_n9216", W.grid_geometry(2, 6, 16), 32, 20250102, "log", 5),
             ("exp_n1600", W.grid_geometry(2, 5, 8, jitter=0.25, seed=3), 10, 11, "exp", 2)]
    for name, g, k, seed, kind, ncols in cases:
        _announce(f"noalloc apply {name} N={g.n} b={g.nboxes} k={k} ncols={ncols}")
        plan, op, h = _handle(P, g, k, seed, kind)
        U, V, At, B = _factors(h, plan, g)
        x = np.random.default_rng(seed).standard_normal((g.n, ncols))
        xd = P.colmajor(x)
        for trans in (False, True):
            y_ref = h.apply(xd, trans=trans).cpu().numpy()
            out = P.colmajor(np.full((g.n, ncols), np.nan))
            y = h.apply(xd, trans=trans, out=out, noalloc=True)
            torch.cuda.synchronize()
            y = y.cpu().numpy()
            assert np.array_equal(y, y_ref), (name, trans, np.max(np.abs(y - y_ref)))
            yo = O.ublr_apply(U, V, At, B, g.box_ptr, k, x, trans=trans)
            assert np.max(np.abs(y - yo)) <= 1e-12 * np.max(np.abs(yo)), (name, trans)
        del h


def test_noalloc_apply_rejects_oversized_workspace():
    import paper_2501_05528_amd as P
    g = W.grid_geometry(2, 5, 8, jitter=0.25, seed=3)
    plan, op, h = _handle(P, g, 10, 11, "log")
    x = P.colmajor(np.zeros((g.n, 6000)))     # (2 + 1) * 250 * 6000 doubles > 32 MiB
    with pytest.raises(P.BlrError) as ei:
        h.apply(x, noalloc=True)
    assert ei.value.name == "BLR_ERR_INVALID_ARG" and "32 MiB" in str(ei.value)
