"""GPU parity of the mixed-precision mode (low-precision tagged sketch + one FP64
far-field refinement sketch), through the C ABI, against the CPU oracle.

Stage checks (inputs from the seeded generators, never from the GPU):
  * low-precision sketch: elementwise |Y0 - Y| <= c (|A| + 1) |Omega|, with Y the
    oracle's FP64 sketch of the kernel matrix on FP32-rounded coordinates and
    c = 2 u + N 2^-24 + 1e-5 (u = 2^-8 for BF16 operands, 2^-24 for FP32; N 2^-24
    bounds FP32 accumulation of N terms; 1e-5 covers the FP32 kernel entries),
    and ||Y0 - Y||_F <= 1e-2 ||Y||_F (BF16) or 1e-4 (FP32);
  * post-processing of FP32 samples: 1e-13 relative to the oracle on the same values;
  * sample bases: Householder Q with the sign rule against the oracle's QR, 1e-12;
  * refinement sketch: 1e-12 relative to the oracle's far-field sums.
End to end: the relative Frobenius error of the mixed result is at most 1.5 times
the FP64 oracle's (plain tagging with r = k + p); exact-rank input is recovered.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

MODES = ["bf16", "fp32"]


def _announce(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _np(t):
    return t.detach().cpu().numpy()


def _geom(name):
    if name == "laplace_n9216":
        return W.grid_geometry(2, 6, 16), 32, 10, "log", 20250102
    if name == "laplace_ragged_jitter":
        return W.grid_geometry(2, (6, 5), (15, 13), jitter=0.25, seed=20250112), 20, 10, "log", 20250112
    if name == "invr3d_n8000":
        return W.grid_geometry(3, 4, 5), 24, 10, "inv_r", 20250103
    if name == "exp_n2500":
        return W.grid_geometry(2, 5, 10, jitter=0.25, seed=7), 16, 10, "exp", 20250104
    if name == "cos_uneven":
        g = W.irregular_grid_geometry([[9, 12, 10, 14, 11, 9], [10, 13, 9, 12, 11]], jitter=0.2, seed=9)
        return g, 20, 10, "cos", 20250105
    raise KeyError(name)


KERNEL_CASES = ["laplace_n9216", "laplace_ragged_jitter", "invr3d_n8000", "exp_n2500", "cos_uneven"]


def _setup(name, r_lo_extra=0):
    import paper_2501_05528_amd as P
    g, k, p, kind, seed = _geom(name)
    near = O.near_lists(g.lattice)
    ell = O.num_tag_columns(near, 3)
    T = W.tag_matrix(seed, g.nboxes, ell)
    r = k + p
    r_lo = r + r_lo_extra
    G, H = W.gaussian_test_blocks(seed, g.n, r_lo)
    gu, gv = W.refinement_gammas(seed, g.nboxes, r_lo, r)
    plan = P.Plan(g.box_ptr, g.lattice, k, T, p=p, extra_tag_cols=3)
    op = P.Operator.kernel(kind, g.pts)
    return dict(P=P, g=g, k=k, p=p, r=r, r_lo=r_lo, kind=kind, seed=seed, T=T, G=G, H=H, gu=gu,
                gv=gv, plan=plan, op=op, near=near, far=O.far_lists(near, g.nboxes))


# ---------------------------------------------------------------- stages
@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("name", ["laplace_n9216", "invr3d_n8000", "cos_uneven"])
def test_lowp_sketch_bound(name, mode):
    S = _setup(name)
    g, P = S["g"], S["P"]
    _announce(f"lowp sketch {name} {mode} N={g.n} r_lo={S['r_lo']}")
    Y0, Z0 = P.sketch_lowp(S["plan"], S["op"], mode, P.colmajor(S["G"]), P.colmajor(S["H"]))
    Y0, Z0 = _np(Y0).astype(np.float64), _np(Z0).astype(np.float64)
    pts32 = g.pts.astype(np.float32).astype(np.float64)
    A = O.KernelOperator(S["kind"], pts32).block()
    Om = O.extended_test_matrix(S["T"], S["G"], g.box_ptr)
    Ps = O.extended_test_matrix(S["T"], S["H"], g.box_ptr)
    u = 2.0 ** -8 if mode == "bf16" else 2.0 ** -24
    c = 2 * u + g.n * 2.0 ** -24 + 1e-5
    for got, Xm, Am in ((Y0, Om, A), (Z0, Ps, A.T)):
        ref = Am @ Xm
        bound = c * ((np.abs(Am) + 1.0) @ np.abs(Xm))
        assert np.all(np.abs(got - ref) <= bound)
        rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        assert rel <= (1e-2 if mode == "bf16" else 1e-4), rel


def test_postprocess_lowp_exact():
    S = _setup("laplace_ragged_jitter")
    P, g, plan = S["P"], S["g"], S["plan"]
    torch = __import__("torch")
    r_lo = S["r_lo"]
    rng = np.random.default_rng(11)
    Y0 = rng.standard_normal((g.n, plan.ell * r_lo)).astype(np.float32)
    Z0 = rng.standard_normal((g.n, plan.ell * r_lo)).astype(np.float32)
    Yd = P.colmajor_empty(g.n, plan.ell * r_lo, "cuda", torch.float32)
    Zd = P.colmajor_empty(g.n, plan.ell * r_lo, "cuda", torch.float32)
    Yd.copy_(torch.as_tensor(Y0))
    Zd.copy_(torch.as_tensor(Z0))
    Yh, Zh = P.postprocess_lowp(plan, r_lo, Yd, Zd)
    z, _ = O.tag_plan(S["T"], S["near"], S["far"])
    for got, src in ((Yh, Y0), (Zh, Z0)):
        ref = O.tag_postprocess(src.astype(np.float64), z, g.box_ptr, r_lo)
        assert np.max(np.abs(_np(got) - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_sample_bases_vs_oracle_qr():
    S = _setup("cos_uneven")
    P, g, plan = S["P"], S["g"], S["plan"]
    X = W.gaussian_colmajor(S["seed"], W.STREAM_POWER, g.n, S["r_lo"])
    Q = _np(P.sample_bases(plan, P.colmajor(X)))
    ref = O.sample_bases(X, g.box_ptr)
    assert np.max(np.abs(Q - ref)) <= 1e-12


@pytest.mark.parametrize("name", ["laplace_n9216", "invr3d_n8000", "exp_n2500", "cos_uneven", "planted"])
def test_refine_sketch_vs_oracle(name):
    import paper_2501_05528_amd as P
    if name == "planted":
        wl = W.WORKLOADS["planted_2d_n4096"]
        g = wl.geometry()
        A, _, _ = W.planted_exact_rank(g, wl.k, wl.seed)
        k, p, seed = wl.k, wl.p, wl.seed
        near = O.near_lists(g.lattice)
        T = W.tag_matrix(seed, g.nboxes, O.num_tag_columns(near, 3))
        plan = P.Plan(g.box_ptr, g.lattice, k, T, p=p, extra_tag_cols=3)
        Ad = P.colmajor(A)
        op = P.Operator.dense(Ad)
        oop = O.DenseOperator(A)
        far = O.far_lists(near, g.nboxes)
        r = k + p
    else:
        S = _setup(name)
        g, plan, op, far, r, seed = S["g"], S["plan"], S["op"], S["far"], S["r"], S["seed"]
        oop = O.KernelOperator(S["kind"], g.pts)
    r_lo = r + 4
    _announce(f"refine sketch {name} N={g.n} r={r} r_lo={r_lo}")
    U0 = W.gaussian_colmajor(seed, W.STREAM_POWER, g.n, r_lo)
    V0 = W.gaussian_colmajor(seed + 1, W.STREAM_POWER, g.n, r_lo)
    gu, gv = W.refinement_gammas(seed, g.nboxes, r_lo, r)
    torch = __import__("torch")
    SY, SZ = P.refine_sketch(plan, op, P.colmajor(U0), P.colmajor(V0),
                             torch.as_tensor(gu, device="cuda"), torch.as_tensor(gv, device="cuda"))
    refY = O.far_sample(oop, O.mixed_test_blocks(V0, gv, g.box_ptr), g.box_ptr, far)
    refZ = O.far_sample(oop, O.mixed_test_blocks(U0, gu, g.box_ptr), g.box_ptr, far, adjoint=True)
    for got, ref in ((SY, refY), (SZ, refZ)):
        assert np.max(np.abs(_np(got) - ref)) <= 1e-12 * np.max(np.abs(ref))


# ---------------------------------------------------------------- end to end
def _oracle_plain_error(S):
    g = S["g"]
    A = O.KernelOperator(S["kind"], g.pts).block()
    op = O.DenseOperator(A)
    G, H = W.gaussian_test_blocks(S["seed"], g.n, S["r"])
    res = O.reconstruct_tag(op, g.box_ptr, g.lattice, S["k"], S["p"], 3, S["T"], G, H)
    return O.rel_fro_error(op, res["U"], res["V"], res["Atil"], res["B"], g.box_ptr, S["k"])


@pytest.fixture(scope="module")
def plain_errors():
    return {}


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("name", KERNEL_CASES)
def test_mixed_error_within_band(name, mode, plain_errors):
    import torch
    S = _setup(name)
    P, g = S["P"], S["g"]
    if name not in plain_errors:
        plain_errors[name] = _oracle_plain_error(S)
    e_or = plain_errors[name]
    _announce(f"mixed {mode} {name} N={g.n} k={S['k']} r_lo={S['r_lo']}")
    h, rep = P.compress(S["plan"], S["op"], P.colmajor(S["G"]), P.colmajor(S["H"]), precision=mode,
                        gamma_u=torch.as_tensor(S["gu"], device="cuda"),
                        gamma_v=torch.as_tensor(S["gv"], device="cuda"))
    e = h.error_fro(S["op"])
    _announce(f"mixed {mode} {name}: rel fro error {e:.3e}, FP64 oracle {e_or:.3e}")
    assert e <= 1.5 * e_or + 1e-12
    ell, r = S["plan"].ell, S["r"]
    m = int(np.max(g.box_sizes()))
    assert rep["applies_At"] == ell * S["r_lo"] + g.nboxes * r
    assert rep["applies_A"] == ell * S["r_lo"] + g.nboxes * r + g.nboxes * S["k"] + 3 ** g.dim * m
    assert rep["precision"] == {"fp32": 1, "bf16": 2}[mode] and rep["r_lo"] == S["r_lo"]


@pytest.mark.parametrize("mode", MODES)
def test_mixed_exact_rank_recovery(mode):
    import torch
    import paper_2501_05528_amd as P
    wl = W.WORKLOADS["planted_2d_n4096"]
    g = wl.geometry()
    A, _, _ = W.planted_exact_rank(g, wl.k, wl.seed)
    near = O.near_lists(g.lattice)
    T = W.tag_matrix(wl.seed, g.nboxes, O.num_tag_columns(near, 3))
    r = wl.k + wl.p
    G, H = W.gaussian_test_blocks(wl.seed, g.n, r)
    gu, gv = W.refinement_gammas(wl.seed, g.nboxes, r, r)
    _announce(f"mixed {mode} planted N={g.n} k={wl.k}")
    plan = P.Plan(g.box_ptr, g.lattice, wl.k, T, p=wl.p, extra_tag_cols=3)
    Ad = P.colmajor(A)
    op = P.Operator.dense(Ad)
    h, _ = P.compress(plan, op, P.colmajor(G), P.colmajor(H), precision=mode,
                      gamma_u=torch.as_tensor(gu, device="cuda"), gamma_v=torch.as_tensor(gv, device="cuda"))
    assert h.error_fro(op) <= 1e-12


def test_mixed_pipeline_wiring():
    """The kept intermediates of one compression are consistent with the stage entry
    points (same kernels): the sample bases are orthonormal per box and the kept
    refinement samples equal a fresh refinement sketch on the kept bases."""
    import torch
    S = _setup("laplace_ragged_jitter", r_lo_extra=6)
    P, g = S["P"], S["g"]
    gu = torch.as_tensor(S["gu"], device="cuda")
    gv = torch.as_tensor(S["gv"], device="cuda")
    h, _ = P.compress(S["plan"], S["op"], P.colmajor(S["G"]), P.colmajor(S["H"]), precision="bf16",
                      gamma_u=gu, gamma_v=gv, keep_intermediates=True)
    U0, V0 = h.part("U0"), h.part("V0")
    bp = g.box_ptr
    for Q in (_np(U0), _np(V0)):
        for i in range(g.nboxes):
            Qi = Q[bp[i]:bp[i + 1]]
            assert np.linalg.norm(Qi.T @ Qi - np.eye(Q.shape[1])) <= 1e-13 * Q.shape[1]
    SY, SZ = P.refine_sketch(S["plan"], S["op"], U0, V0, gu, gv)
    assert torch.equal(SY, h.part("SY")) and torch.equal(SZ, h.part("SZ"))
    Y0 = h.part("Y0")
    assert Y0.dtype == torch.float32 and tuple(Y0.shape) == (g.n, S["plan"].ell * S["r_lo"])
