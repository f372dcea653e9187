"""Full-size parity at the benchmark workload (2D Laplace log|x-y|, 256 x 256 grid,
16 x 16 boxes of 256 points, k = 32, FP64), in the launch configuration bench.py times.

The oracle cannot run the whole compression at N = 65536 in a test, so it computes sampled
outputs one by one: rows of Y and Z, the post-processed samples and bases of a few boxes
(every row of those boxes), far-field blocks between sampled boxes, and the diagonal
near-field block of box 0 (which needs the oracle's bases of box 0's whole colour class).
Tolerances as in tests/test_gpu_parity.py.  The relative Frobenius error must meet the
1e-8 target.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def full():
    import torch
    import paper_2501_05528_amd as P
    wl = W.WORKLOADS["laplace2d_n65536"]
    g = wl.geometry()
    near = O.near_lists(g.lattice)
    far = O.far_lists(near, g.nboxes)
    ell = O.num_tag_columns(near, wl.extra_tag_cols)
    T = W.tag_matrix(wl.seed, g.nboxes, ell)
    G, H = W.gaussian_test_blocks(wl.seed, g.n, wl.r)
    print(f"[gpu-case] laplace2d_n65536 seed={wl.seed} N={g.n} b={g.nboxes} k={wl.k}", flush=True)
    plan = P.Plan(g.box_ptr, g.lattice, wl.k, T, p=wl.p, extra_tag_cols=wl.extra_tag_cols)
    op = P.Operator.kernel("log", g.pts)
    h, rep = P.compress(plan, op, P.colmajor(G), P.colmajor(H), keep_intermediates=True)
    torch.cuda.synchronize()
    boxes = [0, 119, 255]                       # corner, interior, corner
    rows = np.concatenate([np.arange(g.box_ptr[i], g.box_ptr[i + 1]) for i in boxes])
    rows_t = torch.as_tensor(rows, device="cuda")
    out = {}
    for name in ["Y", "Z", "Yhat", "Zhat", "U", "V"]:
        out[name] = h.part(name).index_select(0, rows_t).cpu().numpy()
    At = h.part("Atil")
    k = wl.k
    out["Atil_blocks"] = {(i, j): At[i * k:(i + 1) * k, j * k:(j + 1) * k].cpu().numpy()
                          for i in boxes for j in boxes}
    # diagonal near-field blocks B_ii of the sampled boxes (column-major m_i x m_i)
    near_ptr, near_idx, _, boff = plan.lists()
    Bv = h.part_ptr("B")
    Bt = torch.as_tensor(P.api._DeviceView(Bv[0], Bv[1], 1), device="cuda")
    out["B_diag"] = {}
    for i in boxes:
        q = [q for q in range(near_ptr[i], near_ptr[i + 1]) if near_idx[q] == i][0]
        m = int(g.box_ptr[i + 1] - g.box_ptr[i])
        out["B_diag"][i] = Bt[boff[q]:boff[q] + m * m, 0].cpu().numpy().reshape((m, m), order="F")
    err = h.error_fro(op)
    return dict(wl=wl, g=g, near=near, far=far, T=T, G=G, H=H, plan=plan, boxes=boxes, rows=rows,
                out=out, err=err, rep=rep)


def _oracle_rows(op, T, G, H, box_ptr, rows):
    """Oracle sketch rows (A applied row by row; the kernels are symmetric, so A* = A)."""
    Om = O.extended_test_matrix(T, G, box_ptr)
    Y = op.matmat(Om, rows=rows)
    del Om
    Ps = O.extended_test_matrix(T, H, box_ptr)
    Z = op.rmatmat(Ps, rows=rows)
    return Y, Z


def _sub_ptr(box_ptr, boxes):
    return np.concatenate([[0], np.cumsum([box_ptr[i + 1] - box_ptr[i] for i in boxes])]).astype(np.int64)


def test_fullsize_sketch_bases_cores(full):
    wl, g = full["wl"], full["g"]
    k, r = wl.k, wl.r
    near, far, T = full["near"], full["far"], full["T"]
    bp = g.box_ptr
    op = O.KernelOperator("log", g.pts, chunk=256)
    boxes = full["boxes"]
    Y, Z = _oracle_rows(op, T, full["G"], full["H"], bp, full["rows"])
    out = full["out"]
    for a, b in ((out["Y"], Y), (out["Z"], Z)):
        assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))
    sub_ptr = _sub_ptr(bp, boxes)
    z = np.array([O.optimise_tag_vector(T, near[i], far[i])[0] for i in boxes])
    Yh = O.tag_postprocess(Y, z, sub_ptr, r)
    Zh = O.tag_postprocess(Z, z, sub_ptr, r)
    assert np.max(np.abs(out["Yhat"] - Yh)) <= 1e-12 * np.max(np.abs(Yh))
    assert np.max(np.abs(out["Zhat"] - Zh)) <= 1e-12 * np.max(np.abs(Zh))
    U, V = O.tag_bases(Yh, Zh, sub_ptr, k)
    for q in range(len(boxes)):
        sl = slice(sub_ptr[q], sub_ptr[q + 1])
        for side, ref, S in (("U", U, Yh), ("V", V, Zh)):
            Gi, Oi, Si = out[side][sl], ref[sl], S[sl]
            assert np.linalg.norm(Gi.T @ Gi - np.eye(k)) <= 1e-13 * k
            assert np.linalg.norm(Gi @ (Gi.T @ Si) - Oi @ (Oi.T @ Si)) <= 1e-11 * np.linalg.norm(Si)
    # far-field blocks between sampled boxes: U_i Atil_ij V_j* with each side's own factors
    for qi, i in enumerate(boxes):
        for qj, j in enumerate(boxes):
            if j in near[i]:
                continue
            ri, cj = slice(sub_ptr[qi], sub_ptr[qi + 1]), slice(sub_ptr[qj], sub_ptr[qj + 1])
            Aij = op.block(np.arange(bp[i], bp[i + 1]), np.arange(bp[j], bp[j + 1]))
            ref = U[ri] @ (U[ri].T @ Aij @ V[cj]) @ V[cj].T
            got = out["U"][ri] @ out["Atil_blocks"][(i, j)] @ out["V"][cj].T
            assert np.max(np.abs(got - ref)) <= 1e-11 * np.max(np.abs(Aij)), (i, j)


def test_fullsize_nearfield_diagonal(full):
    """U_0 Atil_00 V_0* + B_00 for box 0.  The probe for box 0's colour also carries
    every far box l of that colour, so B_00 holds, besides A_00 - U_0 Atil_00 V_0*,
    the truncation residuals A_0l - U_0 Atil_0l V_l* of those far blocks (Table 1,
    near field by probing).  The oracle computes exactly that sum from its own bases
    of the whole colour class."""
    wl, g = full["wl"], full["g"]
    k, r = wl.k, wl.r
    near, far, T = full["near"], full["far"], full["T"]
    bp = g.box_ptr
    col = O.colours(g.lattice)
    cls = [l for l in range(g.nboxes) if col[l] == col[0]]
    assert cls[0] == 0 and all(l not in near[0] for l in cls[1:])
    op = O.KernelOperator("log", g.pts, chunk=256)
    rows = np.concatenate([np.arange(bp[l], bp[l + 1]) for l in cls])
    Y0 = op.matmat(O.extended_test_matrix(T, full["G"], bp), rows=np.arange(bp[0], bp[1]))
    Zc = op.rmatmat(O.extended_test_matrix(T, full["H"], bp), rows=rows)
    sub = _sub_ptr(bp, cls)
    z = np.array([O.optimise_tag_vector(T, near[l], far[l])[0] for l in cls])
    Zh = O.tag_postprocess(Zc, z, sub, r)
    Yh0 = O.tag_postprocess(Y0, z[:1], sub[:2], r)
    U0 = O.col_topk(Yh0, k)
    m0 = int(bp[1] - bp[0])
    idx0 = np.arange(bp[0], bp[1])
    ref = np.zeros((m0, m0))
    for q, l in enumerate(cls):
        Vl = O.col_topk(Zh[sub[q]:sub[q + 1]], k)
        A0l = op.block(idx0, np.arange(bp[l], bp[l + 1]))
        R = A0l - U0 @ (U0.T @ A0l @ Vl) @ Vl.T
        w = min(m0, R.shape[1])
        ref[:, :w] += R[:, :w]
        if l == 0:
            ref += U0 @ (U0.T @ A0l @ Vl) @ Vl.T
    out = full["out"]
    got = out["U"][:m0] @ out["Atil_blocks"][(0, 0)] @ out["V"][:m0].T + out["B_diag"][0]
    Amax = np.max(np.abs(op.block(idx0, idx0)))
    assert np.max(np.abs(got - ref)) <= 1e-11 * Amax


def test_fullsize_accuracy_target(full):
    print(f"[gpu-case] laplace2d_n65536 rel fro error {full['err']:.3e}", flush=True)
    assert full["err"] <= 1e-8
    rep = full["rep"]
    wl, g = full["wl"], full["g"]
    ell = full["plan"].ell
    assert rep["applies_A"] + rep["applies_At"] == 2 * ell * wl.r + g.nboxes * wl.k + 9 * 256
