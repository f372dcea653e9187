"""GPU parity of the mixed-precision modes through a black box (the caller's products
only), against the oracle.

Stages (inputs from the seeded generators, never from the GPU):
  * low-precision sketch with the caller's FP32-operand products (computed here from FP32 or
    BF16-rounded operands with FP32 accumulation): elementwise within c (|A| + 1) |Omega| of
    the oracle's FP64 sketch, c = 2 u + N 2^-24 (u = 2^-8 for BF16, 2^-24 for FP32), as for
    the built-in operators in test_gpu_mixed.py;
  * low-precision sketch without such products (FP64 products rounded to FP32): within
    2^-24 |Y| + 1e-12 max|Y| of the oracle's sketch;
  * refinement sketch through block-diagonal products and far-block sums: 1e-12 of the
    oracle's far-field sums (oracle/refine.py far_sample) on the same test blocks.
End to end (FP32 and BF16): a planted exact-rank matrix is recovered to 1e-12, and on the
2D log kernel the relative Frobenius error of the library's factors (evaluated by the
oracle) is at most 1.5 times the oracle's plain FP64 tagging error; product counts include
the refinement's b r columns per side.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def _announce(msg):
    print(f"[gpu-case] {msg}", flush=True)


class DenseProducts:
    """The caller's products with a dense A held as torch tensors (FP64, and FP32 operands
    rounded to the requested precision with FP32 accumulation)."""

    def __init__(self, A):
        import torch
        self.torch = torch
        self.A = torch.as_tensor(A, device="cuda")
        self.At = self.A.t().contiguous()
        self.cols = {0: 0, 1: 0}
        self.lp_cols = {0: 0, 1: 0}

    def __call__(self, X, trans):
        self.cols[int(trans)] += X.shape[1]
        return (self.At if trans else self.A) @ X

    def lp(self, X, trans, precision):
        t = self.torch
        self.lp_cols[int(trans)] += X.shape[1]
        M = (self.At if trans else self.A).float()
        Xf = X.contiguous()
        if precision == "bf16":
            M = M.to(t.bfloat16).float()
            Xf = Xf.to(t.bfloat16).float()
        return (M @ Xf).contiguous()


def _setup(name):
    import paper_2501_05528_amd as P
    if name == "planted":
        wl = W.WORKLOADS["planted_2d_n4096"]
        g = wl.geometry()
        A, _, _ = W.planted_exact_rank(g, wl.k, wl.seed)
        k, p, seed = wl.k, wl.p, wl.seed
    else:
        g = W.grid_geometry(2, (6, 5), (15, 13), jitter=0.25, seed=20250112)
        A = O.KernelOperator("log", g.pts).block()
        k, p, seed = 20, 10, 20250112
    near = O.near_lists(g.lattice)
    T = W.tag_matrix(seed, g.nboxes, O.num_tag_columns(near, 3))
    plan = P.Plan(g.box_ptr, g.lattice, k, T, p=p, extra_tag_cols=3)
    return dict(P=P, g=g, A=A, k=k, p=p, r=k + p, seed=seed, T=T, near=near, plan=plan,
                far=O.far_lists(near, g.nboxes))


@pytest.mark.parametrize("mode", ["fp32", "bf16"])
def test_lowp_sketch_through_callback(mode):
    S = _setup("log")
    P, g, A = S["P"], S["g"], S["A"]
    prod = DenseProducts(A)
    op = P.Operator.from_matmat(g.n, prod, prod.lp)
    G, H = W.gaussian_test_blocks(S["seed"], g.n, S["r"])
    _announce(f"black-box lowp sketch {mode} N={g.n}")
    Y0, Z0 = P.sketch_lowp(S["plan"], op, mode, P.colmajor(G), P.colmajor(H))
    Y0, Z0 = Y0.cpu().numpy().astype(np.float64), Z0.cpu().numpy().astype(np.float64)
    Om = O.extended_test_matrix(S["T"], G, g.box_ptr)
    Ps = O.extended_test_matrix(S["T"], H, g.box_ptr)
    u = 2.0 ** -8 if mode == "bf16" else 2.0 ** -24
    c = 2 * u + g.n * 2.0 ** -24
    for got, Xm, Am in ((Y0, Om, A), (Z0, Ps, A.T)):
        ref = Am @ Xm
        assert np.all(np.abs(got - ref) <= c * ((np.abs(Am) + 1.0) @ np.abs(Xm)))
    LR = S["plan"].ell * S["r"]
    assert prod.lp_cols == {0: LR, 1: LR} and prod.cols == {0: 0, 1: 0}


def test_lowp_sketch_without_lp_products():
    S = _setup("log")
    P, g, A = S["P"], S["g"], S["A"]
    prod = DenseProducts(A)
    op = P.Operator.from_matmat(g.n, prod)
    G, H = W.gaussian_test_blocks(S["seed"], g.n, S["r"])
    Y0, Z0 = P.sketch_lowp(S["plan"], op, "bf16", P.colmajor(G), P.colmajor(H))
    res = O.reconstruct_tag(O.DenseOperator(A), g.box_ptr, g.lattice, S["k"], S["p"], 3, S["T"], G, H,
                            steps=("I",))
    for got, ref in ((Y0, res["Y"]), (Z0, res["Z"])):
        d = np.abs(got.cpu().numpy().astype(np.float64) - ref)
        assert np.all(d <= 2.0 ** -24 * np.abs(ref) + 1e-12 * np.max(np.abs(ref)))


@pytest.mark.parametrize("name", ["log", "planted"])
def test_refine_sketch_through_callback(name):
    import torch
    S = _setup(name)
    P, g, A = S["P"], S["g"], S["A"]
    prod = DenseProducts(A)
    op = P.Operator.from_matmat(g.n, prod)
    r, seed = S["r"], S["seed"]
    r_lo = r + 4
    U0 = W.gaussian_colmajor(seed, W.STREAM_POWER, g.n, r_lo)
    V0 = W.gaussian_colmajor(seed + 1, W.STREAM_POWER, g.n, r_lo)
    gu, gv = W.refinement_gammas(seed, g.nboxes, r_lo, r)
    _announce(f"black-box refinement sketch {name} N={g.n} r={r}")
    SY, SZ = P.refine_sketch(S["plan"], op, P.colmajor(U0), P.colmajor(V0),
                             torch.as_tensor(gu, device="cuda"), torch.as_tensor(gv, device="cuda"))
    oop = O.DenseOperator(A)
    refY = O.far_sample(oop, O.mixed_test_blocks(V0, gv, g.box_ptr), g.box_ptr, S["far"])
    refZ = O.far_sample(oop, O.mixed_test_blocks(U0, gu, g.box_ptr), g.box_ptr, S["far"], adjoint=True)
    for got, ref in ((SY, refY), (SZ, refZ)):
        assert np.max(np.abs(got.cpu().numpy() - ref)) <= 1e-12 * np.max(np.abs(ref))
    assert prod.cols == {0: g.nboxes * r, 1: g.nboxes * r}


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


@pytest.mark.parametrize("mode", ["fp32", "bf16"])
@pytest.mark.parametrize("name", ["planted", "log"])
def test_mixed_compress_through_callback(name, mode):
    import torch
    S = _setup(name)
    P, g, A, k = S["P"], S["g"], S["A"], S["k"]
    prod = DenseProducts(A)
    op = P.Operator.from_matmat(g.n, prod, prod.lp)
    r = S["r"]
    G, H = W.gaussian_test_blocks(S["seed"], g.n, r)
    gu, gv = W.refinement_gammas(S["seed"], g.nboxes, r, r)
    h, rep = P.compress(S["plan"], op, P.colmajor(G), P.colmajor(H), precision=mode,
                        gamma_u=torch.as_tensor(gu, device="cuda"), gamma_v=torch.as_tensor(gv, device="cuda"))
    torch.cuda.synchronize()
    dop = O.DenseOperator(A)
    e = O.rel_fro_error(dop, *_factors(h, S["plan"], g), g.box_ptr, k)
    res = O.reconstruct_tag(dop, g.box_ptr, g.lattice, k, S["p"], 3, S["T"], G, H)
    e_or = O.rel_fro_error(dop, res["U"], res["V"], res["Atil"], res["B"], g.box_ptr, k)
    _announce(f"black-box mixed {mode} {name} N={g.n}: error {e:.3e}, FP64 oracle {e_or:.3e}")
    if name == "planted":
        assert e <= 1e-12
    else:
        assert e <= 1.5 * e_or + 1e-12
    ell, m = S["plan"].ell, int(np.max(g.box_sizes()))
    assert rep["applies_At"] == ell * r + g.nboxes * r
    assert rep["applies_A"] == ell * r + g.nboxes * r + g.nboxes * k + 3 ** g.dim * m
    assert prod.lp_cols == {0: ell * r, 1: ell * r}
    assert prod.cols == {0: g.nboxes * r + g.nboxes * k + 3 ** g.dim * m, 1: g.nboxes * r}
