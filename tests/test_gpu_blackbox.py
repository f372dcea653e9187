"""GPU parity of the black-box operator path: the library sees A only through the
caller's products (Python callback running a dense product on the library's stream).

* Product counts: columns applied to A and A* equal the paper's 2 ell r + b k +
  3^d m_max (A) and ell r (A*) (Alg. 2 sketch widths, Table 1 steps 2-3).
* Results against the oracle (same tolerances as tests/test_gpu_parity.py): the
  sketches to 1e-12, every far block U_i Atil_ij V_j* and near block plus B_ij to
  1e-11 max|A|, and the power estimate of ||A - A_uBLR||_2 in the 1.5 band.
* A failing product ends the call with BLR_ERR_OPERATOR.
* The exact Frobenius error takes the entries from N products with unit columns and equals
  the oracle's error of the same factors; batches, which need entry access, are refused
  with BLR_ERR_UNSUPPORTED (the mixed-precision modes through a black box are tested in
  test_gpu_blackbox_mixed.py).
* The host export returns the same arrays as the device parts.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def _announce(msg):
    print(f"[gpu-case] {msg}", flush=True)


class Counter:
    def __init__(self, A):
        import torch
        self.A = A
        self.At = A.t().contiguous()
        self.cols = {0: 0, 1: 0}
        self.torch = torch

    def __call__(self, X, trans):
        self.cols[int(trans)] += X.shape[1]
        return (self.At if trans else self.A) @ X


def _case(name):
    if name == "planted":
        wl = W.WORKLOADS["planted_2d_n4096"]
        g = wl.geometry()
        A, _, _ = W.planted_exact_rank(g, wl.k, wl.seed)
        return g, A, wl.k, wl.p, wl.seed
    if name == "log_ragged":
        g = W.grid_geometry(2, (6, 5), (15, 13), jitter=0.25, seed=20250112)
        return g, O.KernelOperator("log", g.pts).block(), 20, 10, 20250112
    if name == "invr3d":
        g = W.grid_geometry(3, 4, 5)
        return g, O.KernelOperator("inv_r", g.pts).block(), 24, 10, 20250103
    raise KeyError(name)


@pytest.fixture(scope="module", params=["planted", "log_ragged", "invr3d"])
def run(request):
    import torch
    import paper_2501_05528_amd as P
    g, A, k, p, seed = _case(request.param)
    near = O.near_lists(g.lattice)
    T = W.tag_matrix(seed, g.nboxes, O.num_tag_columns(near, 3))
    G, H = W.gaussian_test_blocks(seed, g.n, k + p)
    res = O.reconstruct_tag(O.DenseOperator(A), g.box_ptr, g.lattice, k, p, 3, T, G, H)
    _announce(f"black box {request.param} N={g.n} b={g.nboxes} k={k}")
    plan = P.Plan(g.box_ptr, g.lattice, k, T, p=p, extra_tag_cols=3)
    Ad = P.colmajor(A)
    cnt = Counter(Ad)
    op = P.Operator.from_matmat(g.n, cnt)
    h, rep = P.compress(plan, op, P.colmajor(G), P.colmajor(H), keep_intermediates=True)
    torch.cuda.synchronize()
    cols = dict(cnt.cols)
    return dict(P=P, g=g, A=A, Ad=Ad, k=k, p=p, seed=seed, T=T, res=res, plan=plan, op=op, h=h, rep=rep,
                cols=cols, cnt=cnt, name=request.param)


def test_product_counts(run):
    g, plan = run["g"], run["plan"]
    r = run["k"] + run["p"]
    m = int(np.max(g.box_sizes()))
    assert run["cols"][1] == plan.ell * r
    assert run["cols"][0] == plan.ell * r + g.nboxes * run["k"] + 3 ** g.dim * m
    assert run["rep"]["applies_A"] == run["cols"][0] and run["rep"]["applies_At"] == run["cols"][1]


def test_sketch_and_blocks_vs_oracle(run):
    g, k, res, h = run["g"], run["k"], run["res"], run["h"]
    bp = g.box_ptr
    for name in ("Y", "Z"):
        got = h.part(name).cpu().numpy()
        assert np.max(np.abs(got - res[name])) <= 1e-12 * np.max(np.abs(res[name]))
    U, V, At = (h.part(x).cpu().numpy() for x in ("U", "V", "Atil"))
    Bflat = h.part("B").cpu().numpy()[:, 0]
    near_ptr, near_idx, _, boff = run["plan"].lists()
    Amax = np.max(np.abs(run["A"]))
    worst = 0.0
    for i in range(g.nboxes):
        nb = {near_idx[q]: boff[q] for q in range(near_ptr[i], near_ptr[i + 1])}
        for j in range(g.nboxes):
            ri, cj = slice(bp[i], bp[i + 1]), slice(bp[j], bp[j + 1])
            rg = U[ri] @ At[i * k:(i + 1) * k, j * k:(j + 1) * k] @ V[cj].T
            ro = res["U"][ri] @ res["Atil"][i * k:(i + 1) * k, j * k:(j + 1) * k] @ res["V"][cj].T
            if j in nb:
                mi, mj = bp[i + 1] - bp[i], bp[j + 1] - bp[j]
                rg = rg + Bflat[nb[j]:nb[j] + mi * mj].reshape((mi, mj), order="F")
                ro = ro + res["B"][(i, j)]
            worst = max(worst, np.max(np.abs(rg - ro)) / Amax)
    assert worst <= 1e-11, worst


def test_power_error_vs_oracle(run):
    P, g, k, res = run["P"], run["g"], run["k"], run["res"]
    x0 = W.gaussian_colmajor(run["seed"], W.STREAM_POWER, g.n, 1)[:, 0]
    x0 = x0 / np.linalg.norm(x0)
    e_gpu, a_gpu = run["h"].error_power(run["op"], P.colmajor(x0), iters=20)
    A = run["A"]
    E = A - O.dense_reconstruction(res["U"], res["V"], res["Atil"], res["B"], g.box_ptr, k)
    e_or = O.power_norm_estimate(lambda v: E @ v, lambda v: E.T @ v, g.n, x0, 20)
    a_or = O.power_norm_estimate(lambda v: A @ v, lambda v: A.T @ v, g.n, x0, 20)
    assert abs(a_gpu - a_or) <= 1e-8 * a_or
    assert (abs(e_gpu - e_or) <= 1e-12 * a_or) or (1 / 1.5 <= e_gpu / e_or <= 1.5)


def test_error_fro_from_products(run):
    """blr_error_fro on a black box takes A's entries from N products with unit columns;
    it must equal the oracle's exact error of the library's own factors (1e-10 relative
    plus 2e-14) and cost exactly N products of A (none of A*)."""
    g, k, h = run["g"], run["k"], run["h"]
    cnt = run["cnt"]
    before = dict(cnt.cols)
    e_gpu = h.error_fro(run["op"])
    assert cnt.cols[0] - before[0] == g.n and cnt.cols[1] == before[1]
    U, V, At = (h.part(x).cpu().numpy() for x in ("U", "V", "Atil"))
    Bflat = h.part("B").cpu().numpy()[:, 0]
    near_ptr, near_idx, _, boff = run["plan"].lists()
    bp = g.box_ptr
    B = {}
    for i in range(g.nboxes):
        for q in range(near_ptr[i], near_ptr[i + 1]):
            j = near_idx[q]
            mi, mj = bp[i + 1] - bp[i], bp[j + 1] - bp[j]
            B[(i, j)] = Bflat[boff[q]:boff[q] + mi * mj].reshape((mi, mj), order="F")
    e_same = O.rel_fro_error(O.DenseOperator(run["A"]), U, V, At, B, bp, k)
    _announce(f"black box {run['name']}: rel fro error from products {e_gpu:.6e}, "
              f"oracle on the same factors {e_same:.6e}")
    assert abs(e_gpu - e_same) <= 1e-10 * e_same + 2e-14


def test_batch_refused(run):
    """Batches need entry access: a black-box job is refused with BLR_ERR_UNSUPPORTED."""
    import torch
    P, g = run["P"], run["g"]
    G, H = W.gaussian_test_blocks(run["seed"], g.n, run["k"] + run["p"])
    with pytest.raises(P.BlrError) as ei:
        P.Batch([dict(plan=run["plan"], op=run["op"], G=P.colmajor(G), H=P.colmajor(H), precision="fp64")])
    assert ei.value.name == "BLR_ERR_UNSUPPORTED"
    torch.cuda.synchronize()


def test_export_matches_parts(run):
    h = run["h"]
    for name in ("U", "Atil", "B", "Yhat"):
        dev = h.part(name).cpu().numpy()
        host = h.export(name)
        assert np.array_equal(host, dev.reshape(-1, order="F"))


def test_operator_failure_reported():
    """A caller's product that fails (nonzero return) ends the call with BLR_ERR_OPERATOR
    and no handle; the same for the low-precision products of the mixed modes."""
    import torch
    import paper_2501_05528_amd as P
    g, A, k, p, seed = _case("log_ragged")
    near = O.near_lists(g.lattice)
    T = W.tag_matrix(seed, g.nboxes, O.num_tag_columns(near, 3))
    G, H = (P.colmajor(a) for a in W.gaussian_test_blocks(seed, g.n, k + p))
    plan = P.Plan(g.box_ptr, g.lattice, k, T, p=p, extra_tag_cols=3)
    Ad = torch.as_tensor(A, device="cuda")
    calls = {"n": 0}

    def flaky(X, trans):
        calls["n"] += 1
        if calls["n"] >= 2:
            raise RuntimeError("planted operator failure")
        return (Ad.t().contiguous() if trans else Ad) @ X

    op = P.Operator.from_matmat(g.n, flaky)
    with pytest.raises(P.BlrError) as ei:
        P.compress(plan, op, G, H)
    assert ei.value.name == "BLR_ERR_OPERATOR"
    assert calls["n"] == 2                     # the failing call ends the compression

    def bad_lp(X, trans, precision):
        raise RuntimeError("planted low-precision failure")

    op2 = P.Operator.from_matmat(g.n, lambda X, trans: (Ad.t().contiguous() if trans else Ad) @ X, bad_lp)
    gam = torch.as_tensor(W.refinement_gammas(seed, g.nboxes, k + p, k + p)[0], device="cuda")
    with pytest.raises(P.BlrError) as ei:
        P.compress(plan, op2, G, H, precision="bf16", gamma_u=gam, gamma_v=gam)
    assert ei.value.name == "BLR_ERR_OPERATOR"
