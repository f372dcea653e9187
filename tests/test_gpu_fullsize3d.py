"""Full-size check of the 3D workload (1/|x-y| on a 48^3 grid, 8^3 boxes of 216 points,
k = 48, ell = 31), FP64 and BF16 mixed precision.

FP64 against the oracle on sampled outputs it computes row by row: rows of Y and Z for three
boxes, their post-processed samples and bases, and the far blocks between them (tolerances as
in tests/test_gpu_parity.py).  Mixed precision against the FP64 oracle on the same boxes: the
far-field residual of the BF16 bases, ||(I - U_i U_i*) A(I_i, F_i) Gamma||_F for a seeded
Gaussian Gamma, is at most 1.5 times that of the oracle's FP64 tagged bases (the mixed-precision
pass band, one-sided); and the BF16 result's relative Frobenius error is below the FP64 result's
times 1.5 (blr_error_fro is pinned to the oracle on identical factors in test_gpu_parity.py).
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def full3d():
    import torch
    import paper_2501_05528_amd as P
    wl = W.WORKLOADS["invr3d_n110592"]
    g = wl.geometry()
    near = O.near_lists(g.lattice)
    far = O.far_lists(near, g.nboxes)
    ell = O.num_tag_columns(near, wl.extra_tag_cols)
    T = W.tag_matrix(wl.seed, g.nboxes, ell)
    G, H = W.gaussian_test_blocks(wl.seed, g.n, wl.r)
    gu, gv = W.refinement_gammas(wl.seed, g.nboxes, wl.r, wl.r)
    print(f"[gpu-case] invr3d_n110592 seed={wl.seed} N={g.n} b={g.nboxes} k={wl.k} ell={ell}", flush=True)
    plan = P.Plan(g.box_ptr, g.lattice, wl.k, T, p=wl.p, extra_tag_cols=wl.extra_tag_cols)
    op = P.Operator.kernel("inv_r", g.pts)
    Gd, Hd = P.colmajor(G), P.colmajor(H)
    h, _ = P.compress(plan, op, Gd, Hd, keep_intermediates=True)
    torch.cuda.synchronize()
    boxes = [0, 273, 511]                       # corner, interior, corner
    rows = np.concatenate([np.arange(g.box_ptr[i], g.box_ptr[i + 1]) for i in boxes])
    rows_t = torch.as_tensor(rows, device="cuda")
    out = {name: h.part(name).index_select(0, rows_t).cpu().numpy()
           for name in ["Y", "Z", "Yhat", "Zhat", "U", "V"]}
    k = wl.k
    At = h.part("Atil")
    out["Atil_blocks"] = {(i, j): At[i * k:(i + 1) * k, j * k:(j + 1) * k].cpu().numpy()
                          for i in boxes for j in boxes}
    del At
    e64 = h.error_fro(op)
    del h
    hm, rep = P.compress(plan, op, Gd, Hd, precision="bf16", gamma_u=torch.as_tensor(gu, device="cuda"),
                         gamma_v=torch.as_tensor(gv, device="cuda"))
    out["U_bf16"] = hm.part("U").index_select(0, rows_t).cpu().numpy()
    out["V_bf16"] = hm.part("V").index_select(0, rows_t).cpu().numpy()
    emx = hm.error_fro(op)
    print(f"[gpu-case] invr3d_n110592: rel fro error FP64 {e64:.3e}, BF16 mixed {emx:.3e} "
          f"({rep['ms_total']:.1f} ms)", flush=True)
    return dict(wl=wl, g=g, near=near, far=far, T=T, G=G, H=H, boxes=boxes, rows=rows, out=out,
                e64=e64, emx=emx)


@pytest.fixture(scope="module")
def oracle3d(full3d):
    """The oracle's rows of Y, Z for the sampled boxes, their post-processed samples and
    FP64 tagged bases (Alg. 2), computed row by row."""
    wl, g = full3d["wl"], full3d["g"]
    bp, T, near, far = g.box_ptr, full3d["T"], full3d["near"], full3d["far"]
    op = O.KernelOperator("inv_r", g.pts, chunk=256)
    rows = full3d["rows"]
    Y = op.matmat(O.extended_test_matrix(T, full3d["G"], bp), rows=rows)
    Z = op.rmatmat(O.extended_test_matrix(T, full3d["H"], bp), rows=rows)
    boxes = full3d["boxes"]
    sub = np.concatenate([[0], np.cumsum([bp[i + 1] - bp[i] for i in boxes])]).astype(np.int64)
    z = np.array([O.optimise_tag_vector(T, near[i], far[i])[0] for i in boxes])
    Yh = O.tag_postprocess(Y, z, sub, wl.r)
    Zh = O.tag_postprocess(Z, z, sub, wl.r)
    U, V = O.tag_bases(Yh, Zh, sub, wl.k)
    return dict(op=op, Y=Y, Z=Z, sub=sub, Yh=Yh, Zh=Zh, U=U, V=V)


def far_residual(op, g, near_i, i, Q, seed):
    """||(I - Q Q*) A(I_i, F_i) Gamma||_F with Gamma a seeded N x 8 Gaussian zeroed on the
    rows of the neighbours of box i (the far block row probed from the right)."""
    bp = g.box_ptr
    Gam = np.random.default_rng(seed).standard_normal((g.n, 8))
    for j in near_i:
        Gam[bp[j]:bp[j + 1]] = 0.0
    Pi = op.matmat(Gam, rows=np.arange(bp[i], bp[i + 1]))
    return np.linalg.norm(Pi - Q @ (Q.T @ Pi)), np.linalg.norm(Pi)


def test_fullsize3d_fp64_sampled_parity(full3d, oracle3d):
    wl, g = full3d["wl"], full3d["g"]
    k = wl.k
    bp, near = g.box_ptr, full3d["near"]
    op, Y, Z, sub, Yh, Zh = (oracle3d[x] for x in ("op", "Y", "Z", "sub", "Yh", "Zh"))
    out = full3d["out"]
    for a, b in ((out["Y"], Y), (out["Z"], Z)):
        assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))
    boxes = full3d["boxes"]
    assert np.max(np.abs(out["Yhat"] - Yh)) <= 1e-12 * np.max(np.abs(Yh))
    assert np.max(np.abs(out["Zhat"] - Zh)) <= 1e-12 * np.max(np.abs(Zh))
    U, V = oracle3d["U"], oracle3d["V"]
    for q in range(len(boxes)):
        sl = slice(sub[q], sub[q + 1])
        for side, ref, S in (("U", U, Yh), ("V", V, Zh)):
            Gi, Oi, Si = out[side][sl], ref[sl], S[sl]
            assert np.linalg.norm(Gi.T @ Gi - np.eye(k)) <= 1e-13 * k
            assert np.linalg.norm(Gi @ (Gi.T @ Si) - Oi @ (Oi.T @ Si)) <= 1e-11 * np.linalg.norm(Si)
    for qi, i in enumerate(boxes):
        for qj, j in enumerate(boxes):
            if j in near[i]:
                continue
            ri, cj = slice(sub[qi], sub[qi + 1]), slice(sub[qj], sub[qj + 1])
            Aij = op.block(np.arange(bp[i], bp[i + 1]), np.arange(bp[j], bp[j + 1]))
            ref = U[ri] @ (U[ri].T @ Aij @ V[cj]) @ V[cj].T
            got = out["U"][ri] @ out["Atil_blocks"][(i, j)] @ out["V"][cj].T
            assert np.max(np.abs(got - ref)) <= 1e-11 * np.max(np.abs(Aij)), (i, j)


def test_fullsize3d_bf16_bases_vs_oracle(full3d, oracle3d):
    g, out, sub = full3d["g"], full3d["out"], oracle3d["sub"]
    for q, i in enumerate(full3d["boxes"]):
        sl = slice(sub[q], sub[q + 1])
        for side in ("U", "V"):        # 1/r is symmetric: the far block column is the transpose
            r_or, nP = far_residual(oracle3d["op"], g, full3d["near"][i], i, oracle3d[side][sl], 100 + i)
            r_mx, _ = far_residual(oracle3d["op"], g, full3d["near"][i], i, out[side + "_bf16"][sl], 100 + i)
            print(f"[gpu-case] box {i} {side}: far residual BF16 {r_mx / nP:.3e}, FP64 oracle {r_or / nP:.3e}",
                  flush=True)
            assert r_mx <= 1.5 * r_or + 1e-13 * nP, (i, side)


def test_fullsize3d_mixed_within_band(full3d):
    assert full3d["emx"] <= 1.5 * full3d["e64"] + 1e-12
