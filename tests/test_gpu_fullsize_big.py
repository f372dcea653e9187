"""Largest 2D job size of the serving mix: 2D Laplace log|x-y| on a 512 x 512 grid, 32 x 32
boxes of 256 points, k = 48 (N = 262144, bk = 49152, so Atil has 2.4e9 entries and its
indices pass 2^31).

Checked with the library's own factors (the oracle computes the reference entries one block
at a time, so these are exact identities of the representation, basis independent):
* far-field cores: Atil_ij = U_i* A_ij V_j for sampled pairs, including the last block row and
  column (indices beyond 2^31);
* near field: B_ii equals the probe of box i's colour minus the low-rank part, i.e. the sum
  over the colour class of A_il - U_i Atil_il V_l* (first m columns) plus U_i Atil_ii V_i*;
* blr_apply rows of the last box against U_i sum_j Atil_ij V_j* x_j + sum_l B_il x_l;
* the BF16 mixed result's relative Frobenius error within 1.5 times the FP64 result's and under
  the 1e-8 target (blr_error_fro is pinned to the oracle on identical factors in
  tests/test_gpu_parity.py).
Against the oracle directly, on two sampled boxes (an interior one and the last one):
* FP64: rows of Y and Z, the post-processed samples and the tagged bases (projectors on the
  samples) as the oracle computes them row by row (Alg. 2);
* BF16 mixed: the far-field residual ||(I - U_i U_i*) A(I_i, F_i) Gamma||_F of its bases is at
  most 1.5 times that of the oracle's FP64 tagged bases (the mixed-precision pass band).
Tolerances as in tests/test_gpu_parity.py.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def big():
    import torch
    import paper_2501_05528_amd as P
    wl = W.WORKLOADS["laplace2d_n262144"]
    g = wl.geometry()
    near = O.near_lists(g.lattice)
    ell = O.num_tag_columns(near, wl.extra_tag_cols)
    T = W.tag_matrix(wl.seed, g.nboxes, ell)
    G, H = W.gaussian_test_blocks(wl.seed, g.n, wl.r)
    gu, gv = W.refinement_gammas(wl.seed, g.nboxes, wl.r, wl.r)
    print(f"[gpu-case] laplace2d_n262144 seed={wl.seed} N={g.n} b={g.nboxes} k={wl.k} ell={ell}", flush=True)
    plan = P.Plan(g.box_ptr, g.lattice, wl.k, T, p=wl.p, extra_tag_cols=wl.extra_tag_cols)
    op = P.Operator.kernel("log", g.pts)
    Gd, Hd = P.colmajor(G), P.colmajor(H)
    h, rep = P.compress(plan, op, Gd, Hd, precision="bf16", gamma_u=torch.as_tensor(gu, device="cuda"),
                        gamma_v=torch.as_tensor(gv, device="cuda"))
    torch.cuda.synchronize()
    print(f"[gpu-case] laplace2d_n262144 BF16 mixed: {rep['ms_total']:.1f} ms", flush=True)
    k = wl.k
    b = g.nboxes
    last = b - 1
    boxes = [0, 527, last]
    U = h.part("U")
    V = h.part("V")
    At = h.part("Atil")
    out = dict(U=U.cpu().numpy(), V=V.cpu().numpy())
    out["Atil_rows"] = {i: At[i * k:(i + 1) * k, :].cpu().numpy() for i in (0, last)}
    out["Atil_blocks"] = {(i, j): At[i * k:(i + 1) * k, j * k:(j + 1) * k].cpu().numpy()
                          for i in boxes for j in boxes}
    del At
    near_ptr, near_idx, colour, boff = plan.lists()
    Bv = h.part_ptr("B")
    Bt = torch.as_tensor(P.api._DeviceView(Bv[0], Bv[1], 1), device="cuda")
    out["B_row_last"] = {}
    for q in range(near_ptr[last], near_ptr[last + 1]):
        l = int(near_idx[q])
        mi, ml = int(g.box_ptr[last + 1] - g.box_ptr[last]), int(g.box_ptr[l + 1] - g.box_ptr[l])
        out["B_row_last"][l] = Bt[boff[q]:boff[q] + mi * ml, 0].cpu().numpy().reshape((mi, ml), order="F")
    x = W.gaussian_colmajor(wl.seed, W.STREAM_POWER, g.n, 1)
    y = h.apply(P.colmajor(x)).cpu().numpy()
    e_mixed = h.error_fro(op)
    del h, Bt
    torch.cuda.synchronize()
    h64, rep64 = P.compress(plan, op, Gd, Hd, keep_intermediates=True)
    e64 = h64.error_fro(op)
    sboxes = [527, last]
    srows = np.concatenate([np.arange(g.box_ptr[i], g.box_ptr[i + 1]) for i in sboxes])
    srows_t = torch.as_tensor(srows, device="cuda")
    out64 = {name: h64.part(name).index_select(0, srows_t).cpu().numpy()
             for name in ["Y", "Z", "Yhat", "Zhat", "U", "V"]}
    print(f"[gpu-case] laplace2d_n262144: FP64 {rep64['ms_total']:.1f} ms, rel fro error FP64 {e64:.3e}, "
          f"BF16 mixed {e_mixed:.3e}", flush=True)
    del h64
    return dict(wl=wl, g=g, near=near, colour=colour, boxes=boxes, out=out, x=x[:, 0], y=y[:, 0],
                e_mixed=e_mixed, e64=e64, T=T, G=G, H=H, sboxes=sboxes, srows=srows, out64=out64)


@pytest.fixture(scope="module")
def oracle_big(big):
    """The oracle's rows of Y, Z, samples and FP64 tagged bases for the sampled boxes."""
    wl, g = big["wl"], big["g"]
    bp, T, near = g.box_ptr, big["T"], big["near"]
    far = O.far_lists(near, g.nboxes)
    op = O.KernelOperator("log", g.pts, chunk=256)
    rows = big["srows"]
    Y = op.matmat(O.extended_test_matrix(T, big["G"], bp), rows=rows)
    Z = op.rmatmat(O.extended_test_matrix(T, big["H"], bp), rows=rows)
    sb = big["sboxes"]
    sub = np.concatenate([[0], np.cumsum([bp[i + 1] - bp[i] for i in sb])]).astype(np.int64)
    z = np.array([O.optimise_tag_vector(T, near[i], far[i])[0] for i in sb])
    Yh = O.tag_postprocess(Y, z, sub, wl.r)
    Zh = O.tag_postprocess(Z, z, sub, wl.r)
    U, V = O.tag_bases(Yh, Zh, sub, wl.k)
    return dict(op=op, Y=Y, Z=Z, sub=sub, Yh=Yh, Zh=Zh, U=U, V=V)


def test_big_fp64_sampled_vs_oracle(big, oracle_big):
    k = big["wl"].k
    o, out = oracle_big, big["out64"]
    for name, ref in (("Y", o["Y"]), ("Z", o["Z"]), ("Yhat", o["Yh"]), ("Zhat", o["Zh"])):
        assert np.max(np.abs(out[name] - ref)) <= 1e-12 * np.max(np.abs(ref)), name
    sub = o["sub"]
    for q in range(len(big["sboxes"])):
        sl = slice(sub[q], sub[q + 1])
        for side, S in (("U", "Yh"), ("V", "Zh")):
            Gi, Oi, Si = out[side][sl], o[side][sl], o[S][sl]
            assert np.linalg.norm(Gi.T @ Gi - np.eye(k)) <= 1e-13 * k
            assert np.linalg.norm(Gi @ (Gi.T @ Si) - Oi @ (Oi.T @ Si)) <= 1e-11 * np.linalg.norm(Si)


def test_big_bf16_bases_vs_oracle(big, oracle_big):
    g, o = big["g"], oracle_big
    bp = g.box_ptr
    sub = o["sub"]
    for q, i in enumerate(big["sboxes"]):
        sl = slice(sub[q], sub[q + 1])
        rows = np.arange(bp[i], bp[i + 1])
        Gam = np.random.default_rng(200 + i).standard_normal((g.n, 8))
        for j in big["near"][i]:
            Gam[bp[j]:bp[j + 1]] = 0.0
        Pi = o["op"].matmat(Gam, rows=rows)          # A(I_i, F_i) Gamma; log is symmetric
        nP = np.linalg.norm(Pi)
        for side in ("U", "V"):
            Qo = o[side][sl]
            Qm = big["out"][side][rows]
            r_or = np.linalg.norm(Pi - Qo @ (Qo.T @ Pi))
            r_mx = np.linalg.norm(Pi - Qm @ (Qm.T @ Pi))
            print(f"[gpu-case] box {i} {side}: far residual BF16 {r_mx / nP:.3e}, FP64 oracle {r_or / nP:.3e}",
                  flush=True)
            assert r_mx <= 1.5 * r_or + 1e-13 * nP, (i, side)


def test_big_cores_beyond_int32(big):
    g, wl, out = big["g"], big["wl"], big["out"]
    k, bp = wl.k, g.box_ptr
    op = O.KernelOperator("log", g.pts, chunk=256)
    U, V = out["U"], out["V"]
    worst = 0.0
    for (i, j), got in out["Atil_blocks"].items():
        ri, cj = slice(bp[i], bp[i + 1]), slice(bp[j], bp[j + 1])
        Aij = op.block(np.arange(bp[i], bp[i + 1]), np.arange(bp[j], bp[j + 1]))
        ref = U[ri].T @ Aij @ V[cj]
        worst = max(worst, np.max(np.abs(got - ref)) / np.max(np.abs(Aij)))
    assert worst <= 1e-11, worst


def test_big_nearfield_diagonal(big):
    g, wl, out = big["g"], big["wl"], big["out"]
    k, bp = wl.k, g.box_ptr
    i = g.nboxes - 1
    op = O.KernelOperator("log", g.pts, chunk=256)
    col = big["colour"]
    cls = [l for l in range(g.nboxes) if col[l] == col[i]]
    U, V, Arow = out["U"], out["V"], out["Atil_rows"][i]
    ri = np.arange(bp[i], bp[i + 1])
    mi = len(ri)
    ref = np.zeros((mi, mi))
    for l in cls:
        cl = np.arange(bp[l], bp[l + 1])
        Ail = op.block(ri, cl)
        low = U[ri] @ Arow[:, l * k:(l + 1) * k] @ V[cl].T
        R = Ail - low
        w = min(mi, R.shape[1])
        ref[:, :w] += R[:, :w]
        if l == i:
            ref += low
    got = U[ri] @ Arow[:, i * k:(i + 1) * k] @ V[ri].T + out["B_row_last"][i]
    Amax = np.max(np.abs(op.block(ri, ri)))
    assert np.max(np.abs(got - ref)) <= 1e-11 * Amax


def test_big_apply_last_box(big):
    g, wl, out = big["g"], big["wl"], big["out"]
    k, bp = wl.k, g.box_ptr
    i = g.nboxes - 1
    U, V, Arow, x = out["U"], out["V"], out["Atil_rows"][i], big["x"]
    t = np.concatenate([V[bp[j]:bp[j + 1]].T @ x[bp[j]:bp[j + 1]] for j in range(g.nboxes)])
    ri = slice(bp[i], bp[i + 1])
    ref = U[ri] @ (Arow @ t)
    for l, Bil in out["B_row_last"].items():
        ref = ref + Bil @ x[bp[l]:bp[l + 1]]
    got = big["y"][ri]
    assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_big_mixed_error_band(big):
    assert big["e64"] <= 1e-8
    assert big["e_mixed"] <= 1.5 * big["e64"] + 1e-12
