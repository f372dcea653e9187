"""GPU parity of the FP64 tagged sketch (Alg. 2; eq. extend_test_mat) across the column
counts r that select the two forms of the last 16-column tile: the 4 x 16 x 4 form, and the
narrow form used when the last tile holds at most 12 columns (2 or 3 tiles for every entry
source; 4 tiles for 1/r only).  Both sides of the sketch against the oracle's
Y = A Omega, Z = A* Psi on the same seeded inputs, max |gpu - oracle| <= 1e-12 max|oracle|.
"""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

# (kind, dim, boxes per axis, points per box axis, r): r on both sides of every tile boundary
CASES = [
    ("log", 2, 4, 8, 12),      # one tile (standard form)
    ("log", 2, 4, 8, 16),
    ("log", 2, 4, 8, 17),      # two tiles, 1 column in the last: narrow
    ("log", 2, 4, 8, 28),      # 12 in the last tile: narrow
    ("log", 2, 4, 8, 29),      # 13: standard
    ("exp", 2, 4, 8, 44),      # three tiles, 12 in the last: narrow
    ("cos", 2, 4, 8, 45),      # 13: standard
    ("log", 2, 4, 8, 60),      # four tiles: standard for log
    ("inv_r", 3, 4, 4, 60),    # four tiles, 12 in the last: narrow for 1/r
    ("inv_r", 3, 4, 4, 61),    # 13: standard
    ("dense", 2, 4, 8, 28),    # a dense matrix, not symmetric
]


def _announce(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("kind,dim,B,q,r", CASES)
def test_sketch_tail_forms(kind, dim, B, q, r):
    import torch
    import paper_2501_05528_amd as P
    seed = 20250300 + r
    g = W.grid_geometry(dim, B, q, jitter=0.2, seed=seed)
    k, p = r - 10, 10
    near = O.near_lists(g.lattice)
    ell = O.num_tag_columns(near, 3)
    T = W.tag_matrix(seed, g.nboxes, ell)
    G, H = W.gaussian_test_blocks(seed, g.n, r)
    if kind == "dense":
        A = np.random.default_rng(seed).standard_normal((g.n, g.n))
        op = P.Operator.dense(P.colmajor(A))
    else:
        A = O.KernelOperator(kind, g.pts).block()
        op = P.Operator.kernel(kind, g.pts)
    _announce(f"sketch tail form: kind={kind} dim={dim} N={g.n} b={g.nboxes} ell={ell} r={r} seed={seed}")
    Yo, Zo = O.tagging.sketch(O.DenseOperator(A), T, G, H, g.box_ptr)
    plan = P.Plan(g.box_ptr, g.lattice, k, T, p=p, extra_tag_cols=3)
    Y, Z = P.sketch(plan, op, P.colmajor(G), P.colmajor(H))
    torch.cuda.synchronize()
    for got, ref in ((Y, Yo), (Z, Zo)):
        got = got.cpu().numpy()
        assert got.shape == ref.shape
        err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        assert err <= 1e-12, f"normwise max error {err:.3e}"
