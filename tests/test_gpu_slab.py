"""GPU parity of the thin-slab Schur-complement operator (blr_op_slab_create, Section 7.2)
against the oracle (oracle/slab.py: sparse LU of the internal planes, pinned in
tests/test_oracle_slab.py), and of tagging through it as a black box.

* Products: S X in plan order to 1e-12 of the largest entry (n below and above one 64-wide
  tile, slabs of 1 and 10 planes).
* Tagging (Alg. 2 and Table 1 through products only): sketches to 1e-12, samples to
  sqrt(ell) 1e-12 of the sketches (see the test), bases (projectors on the samples) within the
  samples' difference, and every represented block to 1e-11 of max|S|;
  the relative Frobenius error of the library's factors (evaluated by the oracle) in the
  band of the oracle's own; the 20-step power estimate on identical factors; the product
  count 2 ell r + b k + 3^d m_max.
"""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import slab as OS

pytestmark = pytest.mark.gpu


def _announce(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("B,q,l", [(3, 4, 4), (6, 8, 10), (5, 20, 10), (4, 4, 1)])
def test_slab_products(B, q, l):
    import paper_2501_05528_amd as P
    g, perm = W.slab_front(B, q)
    n = B * q
    _announce(f"slab products n={n} l={l} N={g.n}")
    op = P.Operator.slab(n, l, perm)
    ref = OS.SlabOperator(n, l, perm)
    for ncols in (1, 5):
        x = np.random.default_rng(ncols + n).standard_normal((g.n, ncols))
        y = op.apply(P.colmajor(x)).cpu().numpy()
        yo = ref.matmat(x)
        assert np.max(np.abs(y - yo)) <= 1e-12 * np.max(np.abs(yo)), (n, l, ncols)
        yt = op.apply(P.colmajor(x), trans=True).cpu().numpy()
        assert np.max(np.abs(yt - yo)) <= 1e-12 * np.max(np.abs(yo))


def test_slab_rejects_bad_arguments():
    import paper_2501_05528_amd as P
    with pytest.raises(P.BlrError) as ei:
        P.Operator.slab(4, 3, np.zeros(16, dtype=np.int64))
    assert ei.value.name == "BLR_ERR_INVALID_ARG"
    with pytest.raises(P.BlrError):
        P.Operator.slab(4, 0, np.arange(16))


@pytest.fixture(scope="module")
def tagged():
    import torch
    import paper_2501_05528_amd as P
    B, q, l, k, p, seed = 6, 8, 10, 16, 10, 20250108
    g, perm = W.slab_front(B, q)
    n = B * q
    ref = OS.SlabOperator(n, l, perm)
    near = O.near_lists(g.lattice)
    ell = O.num_tag_columns(near, 3)
    T = W.tag_matrix(seed, g.nboxes, ell)
    G, H = W.gaussian_test_blocks(seed, g.n, k + p)
    res = O.reconstruct_tag(ref, g.box_ptr, g.lattice, k, p, 3, T, G, H)
    Sd = O.DenseOperator(ref.block())          # entries for the error evaluation (harness)
    res["err"] = O.rel_fro_error(Sd, res["U"], res["V"], res["Atil"], res["B"], g.box_ptr, k)
    _announce(f"slab tagging n={n} l={l} N={g.n} b={g.nboxes} k={k}; oracle error {res['err']:.3e}")
    plan = P.Plan(g.box_ptr, g.lattice, k, T, p=p, extra_tag_cols=3)
    op = P.Operator.slab(n, l, perm)
    h, rep = P.compress(plan, op, P.colmajor(G), P.colmajor(H), keep_intermediates=True)
    torch.cuda.synchronize()
    out = {name: h.part(name).cpu().numpy() for name in ["U", "V", "Atil", "B", "Y", "Z", "Yhat", "Zhat"]}
    near_ptr, near_idx, _, boff = plan.lists()
    bp = g.box_ptr
    Bd = {}
    for i in range(g.nboxes):
        for qq in range(near_ptr[i], near_ptr[i + 1]):
            j = int(near_idx[qq])
            mi, mj = bp[i + 1] - bp[i], bp[j + 1] - bp[j]
            Bd[(i, j)] = out["B"][boff[qq]:boff[qq] + mi * mj, 0].reshape((mi, mj), order="F")
    return dict(g=g, k=k, ref=ref, Sd=Sd, res=res, h=h, rep=rep, out=out, Bd=Bd, plan=plan, op=op, P=P, seed=seed)


def test_slab_sketch_and_bases(tagged):
    """The Schur complement's near field is several orders of magnitude above its far field,
    so the post-processed samples (the far field left after the tags cancel the near field,
    eq. projected_tags) are far smaller than the sketches they come from: their difference is
    bounded by the sketches' rounding, sum_j |z_j| 1e-12 max|Y| <= sqrt(ell) 1e-12 max|Y|, not
    by their own size; and the bases agree as closely as the samples they are computed from."""
    out, res, g, k = tagged["out"], tagged["res"], tagged["g"], tagged["k"]
    ell = tagged["plan"].ell
    for a, src in (("Y", "Y"), ("Z", "Z")):
        assert np.max(np.abs(out[a] - res[a])) <= 1e-12 * np.max(np.abs(res[a])), a
    for a, src in (("Yhat", "Y"), ("Zhat", "Z")):
        d = np.max(np.abs(out[a] - res[a]))
        assert d <= 1e-12 * np.sqrt(ell) * np.max(np.abs(res[src])), a
    bp = g.box_ptr
    for side, S in (("U", "Yhat"), ("V", "Zhat")):
        for i in range(g.nboxes):
            rows = slice(bp[i], bp[i + 1])
            Gi, Oi, Yi = out[side][rows], res[side][rows], res[S][rows]
            dS = np.linalg.norm(out[S][rows] - Yi)
            assert np.linalg.norm(Gi.T @ Gi - np.eye(k)) <= 1e-13 * k
            assert np.linalg.norm(Gi @ (Gi.T @ Yi) - Oi @ (Oi.T @ Yi)) <= 1e-11 * np.linalg.norm(Yi) + 10 * dS, \
                (side, i)


def test_slab_blocks(tagged):
    out, res, g, k, Bd = tagged["out"], tagged["res"], tagged["g"], tagged["k"], tagged["Bd"]
    bp = g.box_ptr
    Smax = np.max(np.abs(tagged["Sd"].A))
    worst = 0.0
    for i in range(g.nboxes):
        for j in range(g.nboxes):
            ri, cj = slice(bp[i], bp[i + 1]), slice(bp[j], bp[j + 1])
            rg = out["U"][ri] @ out["Atil"][i * k:(i + 1) * k, j * k:(j + 1) * k] @ out["V"][cj].T
            ro = res["U"][ri] @ res["Atil"][i * k:(i + 1) * k, j * k:(j + 1) * k] @ res["V"][cj].T
            if (i, j) in Bd:
                rg = rg + Bd[(i, j)]
                ro = ro + res["B"][(i, j)]
            worst = max(worst, np.max(np.abs(rg - ro)) / Smax)
    assert worst <= 1e-11, worst


def test_slab_error_and_counts(tagged):
    g, k, res = tagged["g"], tagged["k"], tagged["res"]
    out, Bd = tagged["out"], tagged["Bd"]
    e_gpu = O.rel_fro_error(tagged["Sd"], out["U"], out["V"], out["Atil"], Bd, g.box_ptr, k)
    _announce(f"slab: error of the library's factors {e_gpu:.3e}, oracle {res['err']:.3e}")
    assert abs(e_gpu - res["err"]) <= 1e-12 or 1 / 1.5 <= e_gpu / res["err"] <= 1.5
    # the library's own exact error of the same factors, from N products of the black box
    e_lib = tagged["h"].error_fro(tagged["op"])
    _announce(f"slab: blr_error_fro from products {e_lib:.6e}, oracle on the same factors {e_gpu:.6e}")
    assert abs(e_lib - e_gpu) <= 1e-10 * e_gpu + 2e-14
    rep = tagged["rep"]
    ell, r = tagged["plan"].ell, k + 10
    assert rep["applies_At"] == ell * r
    assert rep["applies_A"] == ell * r + g.nboxes * k + 9 * int(np.max(g.box_sizes()))


def test_slab_power_estimate_identical_factors(tagged):
    g, k, P = tagged["g"], tagged["k"], tagged["P"]
    out, Bd = tagged["out"], tagged["Bd"]
    x0 = W.gaussian_colmajor(tagged["seed"], W.STREAM_POWER, g.n, 1)[:, 0]
    e_gpu, a_gpu = tagged["h"].error_power(tagged["op"], P.colmajor(x0), iters=20)
    S = tagged["Sd"].A
    E = S - O.dense_reconstruction(out["U"], out["V"], out["Atil"], Bd, g.box_ptr, k)
    e_or = O.power_norm_estimate(lambda v: E @ v, lambda v: E.T @ v, g.n, x0, 20)
    a_or = O.power_norm_estimate(lambda v: S @ v, lambda v: S.T @ v, g.n, x0, 20)
    _announce(f"slab: power estimate {e_gpu / a_gpu:.3e} (oracle {e_or / a_or:.3e})")
    assert abs(a_gpu - a_or) <= 1e-10 * a_or
    assert abs(e_gpu - e_or) <= 1e-10 * e_or + 1e-12 * a_or
