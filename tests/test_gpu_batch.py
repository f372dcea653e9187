"""GPU tests of batched compression (blr_batch_*): uneven jobs from the batch generator
(N, box size, rank and kernel drawn per job), mixed BF16 / FP32 and FP64 jobs, a dense
operator among them.

* Every job's U, V, Atil, B from the batch equal those of blr_tag_compress on the same
  inputs, bit for bit, on the eager first run, on the run that captures the HIP graph and
  on later replays (with unrelated eager work on the stream between replays).
* The autotuner picks one of the offered tile shapes per persistent sketch class; every
  kernel-matrix job, FP64 ones included, sketches in a persistent class launch.
* A sampled job's error meets the 1.5 band of the FP64 oracle's plain tagging.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

SPW_CANDIDATES = {2: {1: (8, 4), 2: (8, 4), 3: (6, 4), 4: (4, 3), 5: (3, 2)},
                  1: {1: (8, 4), 2: (7, 4), 3: (4, 3), 4: (3, 2), 5: (2, 1)},
                  0: {1: (8, 7), 2: (6, 5), 3: (4, 3), 4: (3, 2), 5: (2, 1)}}   # FP64: as many as the jobs need
KIND_CODE = {"log": 0, "inv_r": 1, "exp": 2, "cos": 3}


def _announce(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def batch_setup():
    import torch
    import paper_2501_05528_amd as P
    jobs = W.uneven_batch_jobs(9, 20250104, n_lo=2048, n_hi=12288)
    precs = ["bf16", "fp32", "fp64"]
    specs = []
    for q, wl in enumerate(jobs):
        g = wl.geometry()
        near = O.near_lists(g.lattice)
        T = W.tag_matrix(wl.seed, g.nboxes, O.num_tag_columns(near, 3))
        prec = precs[q % 3]
        r = wl.k + wl.p
        G, H = W.gaussian_test_blocks(wl.seed, g.n, r)
        gu, gv = W.refinement_gammas(wl.seed, g.nboxes, r, r)
        plan = P.Plan(g.box_ptr, g.lattice, wl.k, T, p=wl.p, extra_tag_cols=3)
        op = P.Operator.kernel(wl.kind, g.pts)
        specs.append(dict(wl=wl, g=g, T=T, plan=plan, op=op, G=P.colmajor(G), H=P.colmajor(H),
                          gamma_u=torch.as_tensor(gu, device="cuda"), gamma_v=torch.as_tensor(gv, device="cuda"),
                          precision=prec))
    # a dense operator in mixed mode (single-job sketch inside the batch)
    wl = W.WORKLOADS["planted_2d_n4096"]
    g = wl.geometry()
    A, _, _ = W.planted_exact_rank(g, wl.k, wl.seed)
    near = O.near_lists(g.lattice)
    T = W.tag_matrix(wl.seed, g.nboxes, O.num_tag_columns(near, 3))
    G, H = W.gaussian_test_blocks(wl.seed, g.n, wl.r)
    gu, gv = W.refinement_gammas(wl.seed, g.nboxes, wl.r, wl.r)
    Ad = P.colmajor(A)
    specs.append(dict(wl=wl, g=g, T=T, plan=P.Plan(g.box_ptr, g.lattice, wl.k, T, p=wl.p, extra_tag_cols=3),
                      op=P.Operator.dense(Ad), A=Ad, G=P.colmajor(G), H=P.colmajor(H),
                      gamma_u=torch.as_tensor(gu, device="cuda"), gamma_v=torch.as_tensor(gv, device="cuda"),
                      precision="bf16"))
    for q, sp in enumerate(specs):
        _announce(f"batch job {q}: N={sp['g'].n} b={sp['g'].nboxes} k={sp['wl'].k} "
                  f"kind={sp['wl'].kind} {sp['precision']}")
    singles = []
    for sp in specs:
        kw = {} if sp["precision"] == "fp64" else dict(precision=sp["precision"], gamma_u=sp["gamma_u"],
                                                        gamma_v=sp["gamma_v"])
        h, _ = P.compress(sp["plan"], sp["op"], sp["G"], sp["H"], **kw)
        singles.append({x: h.part(x) for x in ("U", "V", "Atil", "B")})
    torch.cuda.synchronize()
    return dict(P=P, specs=specs, singles=singles)


def _check_equal(batch, singles):
    for q, ref in enumerate(singles):
        h = batch.result(q)
        for x in ("U", "V", "Atil", "B"):
            got = h.part(x)
            assert (got == ref[x]).all().item(), (q, x)


def test_batch_equals_single_jobs_eager_and_graph(batch_setup):
    import torch
    P, specs, singles = batch_setup["P"], batch_setup["specs"], batch_setup["singles"]
    jobs = [dict(plan=s["plan"], op=s["op"], G=s["G"], H=s["H"], precision=s["precision"],
                 gamma_u=s["gamma_u"], gamma_v=s["gamma_v"]) for s in specs]
    b = P.Batch(jobs, graph=True, autotune=True)
    rep1 = b.run()
    torch.cuda.synchronize()
    _announce(f"batch eager run: {rep1['ms_total']:.2f} ms, classes ntr={rep1['class_ntr']} "
              f"spw={rep1['class_spw']} jobs={rep1['class_jobs']}")
    assert rep1["graph_replayed"] == 0 and rep1["nclasses"] >= 1
    _check_equal(b, singles)
    rep2 = b.run()            # captures and launches the graph
    torch.cuda.synchronize()
    assert rep2["graph_replayed"] == 1
    _check_equal(b, singles)
    for _ in range(2):        # replays with unrelated eager work in between
        sp = specs[0]
        P.compress(sp["plan"], sp["op"], sp["G"], sp["H"], precision=sp["precision"],
                   gamma_u=sp["gamma_u"], gamma_v=sp["gamma_v"])
        rep = b.run()
        torch.cuda.synchronize()
        assert rep["graph_replayed"] == 1
        _check_equal(b, singles)
    for prec, ntr, spw in zip(rep2["class_precision"], rep2["class_ntr"], rep2["class_spw"]):
        assert spw in SPW_CANDIDATES[prec][ntr]
    # every kernel-matrix job sketches in a persistent launch: FP64 jobs in classes of one
    # kernel kind, column-tile count and last-tile form (narrow when it holds <= 12 columns)
    fp64 = [sp for sp in specs if sp["precision"] == "fp64" and "A" not in sp]
    assert sum(nj for prec, nj in zip(rep2["class_precision"], rep2["class_jobs"]) if prec == 0) == len(fp64)

    def tail_form(kind, r):
        ntr = (r + 15) // 16
        narrow = ntr in (2, 3) or (ntr == 4 and kind == "inv_r")
        return 3 if narrow and r - 16 * (ntr - 1) <= 12 else 0

    want = sorted({(KIND_CODE[sp["wl"].kind], (sp["wl"].k + sp["wl"].p + 15) // 16,
                    tail_form(sp["wl"].kind, sp["wl"].k + sp["wl"].p)) for sp in fp64})
    got = sorted((kd, ntr, tl) for prec, kd, ntr, tl in zip(rep2["class_precision"], rep2["class_kind"],
                                                            rep2["class_ntr"], rep2["class_tail"]) if prec == 0)
    assert got == want, (got, want)
    assert all(tl == 0 for prec, tl in zip(rep2["class_precision"], rep2["class_tail"]) if prec != 0)
    assert rep2["sketch_flops"] > 0 and rep2["applies"] > 0


def test_batch_job_error_band(batch_setup):
    import torch
    P, specs = batch_setup["P"], batch_setup["specs"]
    jobs = [dict(plan=s["plan"], op=s["op"], G=s["G"], H=s["H"], precision=s["precision"],
                 gamma_u=s["gamma_u"], gamma_v=s["gamma_v"]) for s in specs]
    b = P.Batch(jobs, graph=False, autotune=False)
    b.run()
    torch.cuda.synchronize()
    q = min(range(len(specs) - 1), key=lambda i: specs[i]["g"].n)   # smallest kernel job
    sp = specs[q]
    g, wl = sp["g"], sp["wl"]
    A = O.KernelOperator(wl.kind, g.pts).block()
    G, H = W.gaussian_test_blocks(wl.seed, g.n, wl.r)
    res = O.reconstruct_tag(O.DenseOperator(A), g.box_ptr, g.lattice, wl.k, wl.p, 3, sp["T"], G, H)
    e_or = O.rel_fro_error(O.DenseOperator(A), res["U"], res["V"], res["Atil"], res["B"], g.box_ptr, wl.k)
    e = b.result(q).error_fro(sp["op"])
    _announce(f"batch job {q} ({sp['precision']}): rel fro error {e:.3e}, oracle {e_or:.3e}")
    assert e <= 1.5 * e_or + 1e-12


def test_footprint(batch_setup):
    P, specs = batch_setup["P"], batch_setup["specs"]
    for sp in specs:
        plan = sp["plan"]
        out_bytes = 8 * (2 * plan.n * plan.k + (plan.b * plan.k) ** 2 + plan.info["b_values"])
        for prec in ("fp64", "bf16", "fp32"):
            assert P.footprint(plan, prec) > out_bytes


def test_fp64_class_with_different_tag_counts():
    """Two FP64 1/r jobs with 4 column tiles of r in one persistent class: a 2D one (ell = 13,
    two groups of 6 and 7 tag columns, 2 per wave would do) and a 3D one (ell = 31, three groups
    of 10 or 11, 3 per wave needed).  The class takes the larger tag-columns-per-wave, and both
    jobs' results equal their single-job compressions bit for bit."""
    import torch
    import paper_2501_05528_amd as P
    specs = []
    for dim, B, q, seed in ((2, 6, 8, 20250201), (3, 4, 4, 20250202)):
        g = W.grid_geometry(dim, B, q)
        k, p = 48, 10                                   # r = 58: four 16-column tiles
        near = O.near_lists(g.lattice)
        T = W.tag_matrix(seed, g.nboxes, O.num_tag_columns(near, 3))
        G, H = W.gaussian_test_blocks(seed, g.n, k + p)
        plan = P.Plan(g.box_ptr, g.lattice, k, T, p=p, extra_tag_cols=3)
        specs.append(dict(plan=plan, op=P.Operator.kernel("inv_r", g.pts), G=P.colmajor(G), H=P.colmajor(H),
                          n=g.n, ell=plan.ell))
        _announce(f"fp64 class job: dim={dim} N={g.n} b={g.nboxes} ell={plan.ell} r={k + p}")
    singles = []
    for sp in specs:
        h, _ = P.compress(sp["plan"], sp["op"], sp["G"], sp["H"])
        singles.append({x: h.part(x) for x in ("U", "V", "Atil", "B")})
    b = P.Batch([dict(plan=s["plan"], op=s["op"], G=s["G"], H=s["H"], precision="fp64") for s in specs],
                graph=False, autotune=False)
    rep = b.run()
    torch.cuda.synchronize()
    assert rep["nclasses"] == 1 and rep["class_precision"] == [0] and rep["class_ntr"] == [4]
    assert rep["class_kind"] == [KIND_CODE["inv_r"]] and rep["class_jobs"] == [2]
    assert rep["class_spw"] == [3] and rep["class_tail"] == [3]     # r = 58: 10 columns in the last tile
    _check_equal(b, singles)
