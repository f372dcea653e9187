"""GPU tests of BLR_ERR_NUMERICAL: a compression that is asked for a report checks the
compressed operator (U, V, Atil, B) for non-finite values and fails with BLR_ERR_NUMERICAL,
returning no handle.  Non-finite entries planted in a far block (they reach the sketch, the
bases and the cores) and in a near block (they reach only B) are both caught, in FP64 and in
the BF16 mixed mode; a clean compression afterwards still matches the one before.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def _announce(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def planted():
    import torch
    import paper_2501_05528_amd as P
    wl = W.WORKLOADS["planted_2d_n4096"]
    g = wl.geometry()
    A, _, _ = W.planted_exact_rank(g, wl.k, wl.seed)
    near = O.near_lists(g.lattice)
    far = O.far_lists(near, g.nboxes)
    T = W.tag_matrix(wl.seed, g.nboxes, O.num_tag_columns(near, 3))
    G, H = W.gaussian_test_blocks(wl.seed, g.n, wl.r)
    gu, gv = W.refinement_gammas(wl.seed, g.nboxes, wl.r, wl.r)
    plan = P.Plan(g.box_ptr, g.lattice, wl.k, T, p=wl.p, extra_tag_cols=3)
    _announce(f"numerical checks on planted_2d_n4096 N={g.n} b={g.nboxes}")
    return dict(P=P, g=g, A=A, near=near, far=far, plan=plan, G=P.colmajor(G), H=P.colmajor(H),
                gu=torch.as_tensor(gu, device="cuda"), gv=torch.as_tensor(gv, device="cuda"))


def _entry(s, i, j):
    bp = s["g"].box_ptr
    return int(bp[i]) + 1, int(bp[j]) + 2


def _compress(s, A, precision):
    P = s["P"]
    op = P.Operator.dense(P.colmajor(A))
    kw = {} if precision == "fp64" else dict(precision=precision, gamma_u=s["gu"], gamma_v=s["gv"])
    return P.compress(s["plan"], op, s["G"], s["H"], **kw)


@pytest.mark.parametrize("where,value", [("far", np.nan), ("near", np.inf)])
@pytest.mark.parametrize("precision", ["fp64", "bf16"])
def test_nonfinite_entry_is_reported(planted, where, value, precision):
    s = planted
    P = s["P"]
    i = 0
    j = s["far"][i][0] if where == "far" else s["near"][i][-1]
    a, b = _entry(s, i, j)
    A = s["A"].copy()
    A[a, b] = value
    _announce(f"non-finite A[{a},{b}] in a {where} block, {precision}")
    with pytest.raises(P.BlrError) as ei:
        _compress(s, A, precision)
    assert ei.value.name == "BLR_ERR_NUMERICAL"


def test_clean_compression_after_errors(planted):
    s = planted
    h1, _ = _compress(s, s["A"], "fp64")
    ref = {x: h1.part(x).clone() for x in ("U", "V", "Atil", "B")}
    A = s["A"].copy()
    A[_entry(s, 0, s["far"][0][0])] = np.nan
    with pytest.raises(s["P"].BlrError):
        _compress(s, A, "fp64")
    h2, rep = _compress(s, s["A"], "fp64")
    for x, t in ref.items():
        assert (h2.part(x) == t).all().item(), x
    assert rep["ms_total"] > 0
