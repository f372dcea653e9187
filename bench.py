#!/usr/bin/env python3
"""Benchmark: tagged uniform-BLR compression (reconstruct_tag) on one MI355X.

A step is one full compression -- tagged sketches, tag post-processing,
per-box bases, cores and near field -- of a synthetic kernel matrix whose
inputs (points, T, G, H) are resident in HBM before timing starts.  The
default workload is the 2D Laplace kernel log|x - y| on a 256 x 256 grid
(N = 65536), 16 x 16 boxes of 256 points, k = 32, p = 10, ell = 13, FP64.

Prints one JSON line (metric, value, unit, steps, timing, dtype, config) plus the
roofline of the dominant kernel (the sketch, FP64 MFMA) and a CPU baseline (the FP64 oracle
timed on a bounded sample of the same workload).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

METRIC = "BLR compressions/s + operator-applies per compression at 1e-8 rel err; %MFMA/HBM"
PEAK_FP64_TFLOPS = 78.6   # MI355X dense FP64 (matrix = vector)
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}   # dense MFMA peaks


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "hbm_traffic_laplace2d_n65536_fp64.md")
KERNELS_SRC = os.path.join(ROOT, "paper_2501_05528_amd", "csrc", "kernels.hip")


def measured_sketch_traffic(workload):
    """HBM bytes per sketch launch from the committed rocprofv3 counter summary, or None
    when the summary is for another workload or the kernels changed since it was taken."""
    import hashlib
    if workload != "laplace2d_n65536" or not os.path.exists(TRAFFIC_PROFILE):
        return None
    text = open(TRAFFIC_PROFILE).read()
    sha = hashlib.sha256(open(KERNELS_SRC, "rb").read()).hexdigest()
    rec = {}
    for line in text.splitlines():
        if ":" in line and not line.startswith(("|", " ")):
            key, _, val = line.partition(":")
            rec[key.strip()] = val.strip()
    if rec.get("kernels.hip sha256") != sha:
        return None
    try:
        return float(rec["sketch_traffic_bytes"])
    except (KeyError, ValueError):
        return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def setup(wl_name):
    import torch
    import paper_2501_05528_amd as P
    wl = W.WORKLOADS[wl_name]
    g = wl.geometry()
    ell = P.tag_columns(g.box_ptr, g.lattice, wl.extra_tag_cols)
    T = W.tag_matrix(wl.seed, g.nboxes, ell)
    G, H = W.gaussian_test_blocks(wl.seed, g.n, wl.r)
    t0 = time.perf_counter()
    plan = P.Plan(g.box_ptr, g.lattice, wl.k, T, p=wl.p, extra_tag_cols=wl.extra_tag_cols)
    plan_s = time.perf_counter() - t0
    op = P.Operator.kernel(wl.kind, g.pts)
    Gd, Hd = P.colmajor(G), P.colmajor(H)
    # mixed modes: r_lo = r (p_lo = p) and the refinement's mixing blocks
    gu, gv = W.refinement_gammas(wl.seed, g.nboxes, wl.r, wl.r)
    gud = torch.as_tensor(gu, device="cuda")
    gvd = torch.as_tensor(gv, device="cuda")
    torch.cuda.synchronize()
    return dict(wl=wl, g=g, T=T, G=G, H=H, plan=plan, op=op, Gd=Gd, Hd=Hd, gud=gud, gvd=gvd,
                plan_s=plan_s, P=P)


def run_mode(S, precision, steps, warmup, with_error):
    """Times `steps` compressions in one precision mode; returns rate, stage times,
    report of the first timed step and the last handle's error."""
    import torch
    P, plan, op = S["P"], S["plan"], S["op"]
    kw = {} if precision == "fp64" else dict(precision=precision, gamma_u=S["gud"], gamma_v=S["gvd"])
    for w in range(warmup):
        h, rep = P.compress(plan, op, S["Gd"], S["Hd"], report=True, **kw)
        log(f"{precision} warmup {w}: {rep['ms_total']:.1f} ms (sketch {rep['ms_sketch']:.1f})")
        del h
    torch.cuda.synchronize()
    handles, reps = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        h, rep = P.compress(plan, op, S["Gd"], S["Hd"], report=True, **kw)
        handles.append(h)
        reps.append(rep)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log(f"{precision}: timed {steps} steps in {elapsed:.3f} s")
    err = None
    if with_error:
        err = handles[-1].error_fro(op)
        log(f"{precision}: relative Frobenius error {err:.3e}")
    last = handles[-1]
    del handles
    stage = {k: float(np.mean([r[k] for r in reps])) for k in
             ("ms_sketch", "ms_postprocess", "ms_orth", "ms_refine", "ms_cores", "ms_nearfield", "ms_total")}
    return dict(value=steps / elapsed, ms_step=1000.0 * elapsed / steps, stage=stage, rep=reps[0], err=err,
                handle=last)


def apply_section(S, h, reps=20):
    """blr_apply (y = U (Atil (V* x)) + B x) on 1 and 16 vectors, and its transpose on one
    vector: time per call from events on the stream, and algorithmic bytes
    8 [(bk)^2 + sum_pairs m_i m_j + 2 N k + 2 N ncols]
    against the 8 TB/s HBM peak; plus the paper's spectral error estimate (20 power
    iterations, Section 7)."""
    import torch
    P, plan, g, wl = S["P"], S["plan"], S["g"], S["wl"]
    bk = plan.b * plan.k
    out = {}
    for ncols, trans in ((1, False), (16, False), (1, True)):
        x = P.colmajor(W.gaussian_colmajor(wl.seed, W.STREAM_POWER, g.n, ncols))
        h.apply(x, trans=trans)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            h.apply(x, trans=trans)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        nbytes = 8.0 * (bk * bk + plan.info["b_values"] + 2 * g.n * plan.k + 2 * g.n * ncols)
        out[f"ncols_{ncols}" + ("_trans" if trans else "")] = {"ms": round(ms, 4), "algorithmic_GB": round(nbytes / 1e9, 4),
                                 "GB_per_s": round(nbytes / (ms * 1e-3) / 1e9, 1),
                                 "frac_of_8TBs": round(nbytes / (ms * 1e-3) / 8e12, 4)}
    x0 = W.gaussian_colmajor(wl.seed, W.STREAM_POWER, g.n, 1)[:, 0]
    x0 = x0 / np.linalg.norm(x0)
    t0 = time.perf_counter()
    e, a = h.error_power(S["op"], P.colmajor(x0), iters=20)
    out["spectral_error"] = {"rel_err_2": e / a, "iters": 20, "s": round(time.perf_counter() - t0, 3)}
    return out


def basic_section(S, tag_value, with_error):
    """One compression by Alg. 3 (b r masked test columns per side instead of ell r
    tagged ones) on the same operator, plan, G and H: the paper's comparison of
    products and time for step (I).  One untimed call first warms the code path."""
    import torch
    P, plan, op = S["P"], S["plan"], S["op"]
    h, _ = P.basic_compress(plan, op, S["Gd"], S["Hd"], report=True)
    del h
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h, rep = P.basic_compress(plan, op, S["Gd"], S["Hd"], report=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    err = h.error_fro(op) if with_error else None
    log(f"basic: {1e3 * el:.1f} ms, samples {rep['ms_sketch']:.1f} ms, rel err {err}")
    sk = rep["sketch_flops"] / (rep["ms_sketch"] * 1e-3) / 1e12
    return {"value": round(1.0 / el, 4), "unit": "compressions/s", "ms_per_step": round(1e3 * el, 3),
            "tagging_speedup": round(tag_value * el, 3),
            "applies_per_compression": int(rep["applies_A"] + rep["applies_At"]),
            "rel_err_fro": err,
            "stage_ms": {k: round(rep[k], 3) for k in ("ms_sketch", "ms_orth", "ms_cores",
                                                       "ms_nearfield", "ms_total")},
            "sample_TFLOPs": round(sk, 2), "sample_flops": rep["sketch_flops"]}


def paper_geometry_section(cases=((20000, 77), (100000, 173)), k=30, p=10, steps=3, seed=20250108):
    """The geometry and parameters of the paper's 2D Laplace experiments (Section 7.1): N
    uniformly random points in the unit square, b = sqrt(3^d N / k) boxes (77 and 173 at
    N = 20000 and 100000) of N / b points up to one from median-type splits, neighbours that
    share a boundary, log kernel, k = 30, p = 10, 3 extra tag columns, FP64.  Reports the total
    products of a compression against N (the paper prints 8.3 times fewer at N = 100000)."""
    import torch
    import paper_2501_05528_amd as P
    out = {}
    for n, nb in cases:
        g, near, _ = W.kd_geometry(n, 2, 0, seed, nboxes=nb)
        ell = P.tag_columns(g.box_ptr, None, 3, near=near)
        T = W.tag_matrix(seed, g.nboxes, ell)
        G, H = W.gaussian_test_blocks(seed, g.n, k + p)
        plan = P.Plan(g.box_ptr, None, k, T, p=p, extra_tag_cols=3, near=near)
        op = P.Operator.kernel("log", g.pts)
        Gd, Hd = P.colmajor(G), P.colmajor(H)
        h, _ = P.compress(plan, op, Gd, Hd, report=True)
        del h
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            h, rep = P.compress(plan, op, Gd, Hd, report=True)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / steps
        err = h.error_fro(op)
        sizes = g.box_sizes()
        applies = int(rep["applies_A"] + rep["applies_At"])
        log(f"paper geometry N={n}, b={nb}: {1e3 * el:.1f} ms, {applies} products, rel err {err:.2e}")
        out[f"n{n}"] = {"value": round(1.0 / el, 4), "unit": "compressions/s", "ms_per_step": round(1e3 * el, 3),
                        "boxes": g.nboxes, "k": k, "p": p, "m_min": int(sizes.min()), "m_max": int(sizes.max()),
                        "ell": ell, "ncolours": plan.info["ncolours"],
                        "applies_step1": int(2 * rep["applies_At"]),
                        "applies_per_compression": applies,
                        "N_over_applies": round(n / applies, 2),
                        "rel_err_fro": err,
                        "sketch_TFLOPs": round(rep["sketch_flops"] / (rep["ms_sketch"] * 1e-3) / 1e12, 2)}
        del h, plan, op
    return out


def bn_section(cases=((8, 8), (16, 16)), q=8, k=16, p=10, seed=20250109):
    """Alg. 1 (block nullification) against tagging on 2D log-kernel grids of boxes of
    q x q = 64 points (k = 16), with the same plan and operator: products, time and
    error.  Block nullification sketches s = r + 9 m columns per side and needs a
    Householder QR of an s x (up to 9 m) block of the test matrix per box and side
    (on the GPU; the post-processing cost of Section 3.2)."""
    import torch
    import paper_2501_05528_amd as P
    out = {}
    for bx, by in cases:
        g = W.grid_geometry(2, (bx, by), q)
        ell = P.tag_columns(g.box_ptr, g.lattice, 3)
        T = W.tag_matrix(seed, g.nboxes, ell)
        plan = P.Plan(g.box_ptr, g.lattice, k, T, p=p, extra_tag_cols=3)
        op = P.Operator.kernel("log", g.pts)
        s = P.bn_min_columns(plan)
        Om, Ps = (P.colmajor(a) for a in W.gaussian_test_blocks(seed, g.n, s))
        G, H = (P.colmajor(a) for a in W.gaussian_test_blocks(seed, g.n, k + p))
        h, _ = P.compress(plan, op, G, H, report=True)
        del h
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h, rt = P.compress(plan, op, G, H, report=True)
        torch.cuda.synchronize()
        tt = time.perf_counter() - t0
        et = h.error_fro(op)
        del h
        t0 = time.perf_counter()
        h, rb = P.bn_compress(plan, op, Om, Ps, report=True)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        eb = h.error_fro(op)
        del h
        log(f"bn N={g.n}: {1e3 * tb:.1f} ms (post-processing {rb['ms_postprocess']:.1f} ms) "
            f"vs tagging {1e3 * tt:.1f} ms")
        out[f"n{g.n}"] = {
            "boxes": g.nboxes, "m": q * q, "k": k, "s": s, "ell": ell,
            "bn": {"ms_per_step": round(1e3 * tb, 3), "applies_per_compression": int(rb["applies_A"] + rb["applies_At"]),
                   "ms_sketch": round(rb["ms_sketch"], 3), "ms_postprocess": round(rb["ms_postprocess"], 3),
                   "rel_err_fro": eb},
            "tagging": {"ms_per_step": round(1e3 * tt, 3), "applies_per_compression": int(rt["applies_A"] + rt["applies_At"]),
                        "ms_sketch": round(rt["ms_sketch"], 3), "ms_postprocess": round(rt["ms_postprocess"], 3),
                        "rel_err_fro": et},
            "tagging_speedup": round(tb / tt, 2),
            "note": "both methods run on the GPU: products, block nullification's per-box null "
                    "spaces (one Householder QR per box and side) and projections, tagging's "
                    "post-processing"}
    return out


def rank_section(S, tol=1e-8, k_probe=48, p=10):
    """Tolerance-driven rank on the bench geometry and operator: one tagged sketch at
    r = k_probe + p picks the uniform k for ``tol``; a plan at that k then compresses,
    and the exact relative Frobenius error is reported."""
    import torch
    P, g, op, wl = S["P"], S["g"], S["op"], S["wl"]
    ell = P.tag_columns(g.box_ptr, g.lattice, wl.extra_tag_cols)
    T = W.tag_matrix(wl.seed, g.nboxes, ell)
    probe = P.Plan(g.box_ptr, g.lattice, k_probe, T, p=p, extra_tag_cols=wl.extra_tag_cols)
    G, H = (P.colmajor(a) for a in W.gaussian_test_blocks(wl.seed, g.n, k_probe + p))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    k, _ = P.tag_rank(probe, op, G, H, tol)
    t_rank = time.perf_counter() - t0
    plan = P.Plan(g.box_ptr, g.lattice, k, T, p=p, extra_tag_cols=wl.extra_tag_cols)
    G2, H2 = (P.colmajor(a) for a in W.gaussian_test_blocks(wl.seed, g.n, k + p))
    h, rep = P.compress(plan, op, G2, H2, report=True)
    err = h.error_fro(op)
    log(f"rank for tol {tol:.0e}: k = {k} ({1e3 * t_rank:.1f} ms), compression {rep['ms_total']:.1f} ms, "
        f"rel err {err:.2e}")
    return {"tol": tol, "k_probe": k_probe, "k": k, "ms_rank": round(1e3 * t_rank, 3),
            "ms_compress": round(rep["ms_total"], 3), "rel_err_fro": err,
            "note": "uniform k from a per-direction singular-value threshold (no error bound); the "
                    "tolerance-calibrated path is the per-box truncation (`truncation`)"}


def truncation_section(S, tol=1e-8, k_big=48, p=10):
    """Per-box ranks from a tolerance on the bench workload: compress at k = k_big, truncate
    the representation to tol (blr_ublr_truncate), report the ranks, the change and the
    exact error before and after."""
    import torch
    P, g, op, wl = S["P"], S["g"], S["op"], S["wl"]
    ell = P.tag_columns(g.box_ptr, g.lattice, wl.extra_tag_cols)
    T = W.tag_matrix(wl.seed, g.nboxes, ell)
    plan = P.Plan(g.box_ptr, g.lattice, k_big, T, p=p, extra_tag_cols=wl.extra_tag_cols)
    G, H = (P.colmajor(a) for a in W.gaussian_test_blocks(wl.seed, g.n, k_big + p))
    h, rep = P.compress(plan, op, G, H, report=True)
    h2, _, _, _ = h.truncate(tol)
    del h2
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h2, ku, kv, change = h.truncate(tol)
    torch.cuda.synchronize()
    t_tr = time.perf_counter() - t0
    e0 = h.error_fro(op)
    e1 = h2.error_fro(op)
    log(f"truncation to {tol:.0e}: ranks {ku.mean():.2f}/{kv.mean():.2f} of {k_big}, {1e3 * t_tr:.1f} ms, "
        f"error {e0:.2e} -> {e1:.2e}")
    return {"tol": tol, "k": k_big, "ms_compress": round(rep["ms_total"], 3), "ms_truncate": round(1e3 * t_tr, 3),
            "mean_rank_u": round(float(ku.mean()), 3), "mean_rank_v": round(float(kv.mean()), 3),
            "min_rank": int(min(ku.min(), kv.min())), "max_rank": int(max(ku.max(), kv.max())),
            "rel_change": change, "rel_err_fro_before": e0, "rel_err_fro_after": e1}


def slab_section(cases=((4, 24), (13, 24)), l=10, k=30, p=10, steps=2, seed=20250110):
    """The paper's second workload (Section 7.2): the thin-slab Helmholtz Schur complement
    as a library-held black box (products only), frontal face n x n in B x B boxes of
    24 x 24 points, l = 10 planes, kappa h = 2 pi / 100, k = 30, p = 10, FP64.  Step (I)
    products stay 2 ell r as N grows; the error is the paper's 20-step spectral estimate."""
    import torch
    import paper_2501_05528_amd as P
    out = {}
    for B, q in cases:
        g, perm = W.slab_front(B, q)
        n = B * q
        ell = P.tag_columns(g.box_ptr, g.lattice, 3)
        T = W.tag_matrix(seed, g.nboxes, ell)
        G, H = (P.colmajor(a) for a in W.gaussian_test_blocks(seed, g.n, k + p))
        plan = P.Plan(g.box_ptr, g.lattice, k, T, p=p, extra_tag_cols=3)
        op = P.Operator.slab(n, l, perm)
        h, _ = P.compress(plan, op, G, H, report=True)
        del h
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            h, rep = P.compress(plan, op, G, H, report=True)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / steps
        x0 = W.gaussian_colmajor(seed, W.STREAM_POWER, g.n, 1)[:, 0]
        e, a = h.error_power(op, P.colmajor(x0 / np.linalg.norm(x0)), iters=20)
        log(f"slab N={g.n}: {1e3 * el:.1f} ms, spectral error {e / a:.2e}")
        out[f"n{g.n}"] = {"value": round(1.0 / el, 4), "unit": "compressions/s", "ms_per_step": round(1e3 * el, 3),
                          "grid": [n, n, l], "boxes": g.nboxes, "m": q * q, "k": k, "ell": ell,
                          "applies_step1": int(2 * rep["applies_At"]),
                          "applies_per_compression": int(rep["applies_A"] + rep["applies_At"]),
                          "stage_ms": {x: round(rep[x], 3) for x in ("ms_sketch", "ms_orth", "ms_cores",
                                                                     "ms_nearfield", "ms_total")},
                          "rel_err_2": e / a}
        del h, plan, op
    return out


def config_section(S, steps=2, warmup=1, with_error=True):
    """One workload in FP64 and both mixed modes: compressions/s, error and the rooflines of
    the sketch (and of the refinement sketch in the mixed modes)."""
    out = {}
    for prec in ("fp64", "bf16", "fp32"):
        m = run_mode(S, prec, steps, warmup, with_error)
        m.pop("handle", None)
        rp, st = m["rep"], m["stage"]
        sk = rp["sketch_flops"] / (st["ms_sketch"] * 1e-3) / 1e12
        d = {"value": round(m["value"], 4), "unit": "compressions/s", "ms_per_step": round(m["ms_step"], 3),
             "rel_err_fro": m["err"], "applies_per_compression": int(rp["applies_A"] + rp["applies_At"]),
             "stage_ms": {k: round(v, 3) for k, v in st.items()},
             "sketch_roofline": {"bound": "mfma", "achieved": round(sk, 2), "peak": PEAK_TFLOPS[prec],
                                 "unit": "TFLOP/s", "frac": round(sk / PEAK_TFLOPS[prec], 4),
                                 "algorithmic_flops_per_launch": rp["sketch_flops"]}}
        if prec != "fp64":
            rf = rp["refine_flops"] / (st["ms_refine"] * 1e-3) / 1e12
            d["refine_roofline"] = {"bound": "mfma", "achieved": round(rf, 2), "peak": PEAK_FP64_TFLOPS,
                                    "unit": "TFLOP/s", "frac": round(rf / PEAK_FP64_TFLOPS, 4),
                                    "algorithmic_flops_per_launch": rp["refine_flops"]}
        out[prec] = d
    out["bf16_speedup_vs_fp64"] = round(out["bf16"]["value"] / out["fp64"]["value"], 3)
    return out


def planted_section(steps=10):
    """The planted exact-rank workload (64 x 64 grid, 8 x 8 boxes of 64, k = 8, dense A in
    HBM): compressions/s and the exact error (exact recovery), in FP64 and in the BF16 and
    FP32 mixed modes (one refinement sketch)."""
    import torch
    import paper_2501_05528_amd as P
    wl = W.WORKLOADS["planted_2d_n4096"]
    g = wl.geometry()
    A, _, _ = W.planted_exact_rank(g, wl.k, wl.seed)
    ell = P.tag_columns(g.box_ptr, g.lattice, wl.extra_tag_cols)
    T = W.tag_matrix(wl.seed, g.nboxes, ell)
    G, H = (P.colmajor(a) for a in W.gaussian_test_blocks(wl.seed, g.n, wl.r))
    plan = P.Plan(g.box_ptr, g.lattice, wl.k, T, p=wl.p, extra_tag_cols=wl.extra_tag_cols)
    Ad = P.colmajor(A)
    op = P.Operator.dense(Ad)
    h, _ = P.compress(plan, op, G, H, report=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        h, rep = P.compress(plan, op, G, H, report=True)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    out = {"value": round(1.0 / el, 3), "unit": "compressions/s", "ms_per_step": round(1e3 * el, 4),
           "applies_per_compression": int(rep["applies_A"] + rep["applies_At"]),
           "rel_err_fro": h.error_fro(op)}
    gu, gv = W.refinement_gammas(wl.seed, g.nboxes, wl.r, wl.r)
    kw = dict(gamma_u=torch.as_tensor(gu, device="cuda"), gamma_v=torch.as_tensor(gv, device="cuda"))
    for prec in ("bf16", "fp32"):
        h, _ = P.compress(plan, op, G, H, report=True, precision=prec, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            h, rep = P.compress(plan, op, G, H, report=True, precision=prec, **kw)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / steps
        out[prec] = {"value": round(1.0 / el, 3), "ms_per_step": round(1e3 * el, 4),
                     "applies_per_compression": int(rep["applies_A"] + rep["applies_At"]),
                     "rel_err_fro": h.error_fro(op)}
    return out


def _blas_threads():
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    try:
        from threadpoolctl import threadpool_info
        info = threadpool_info()
        if info:
            threads = max(int(d.get("num_threads", threads)) for d in info)
    except Exception:
        pass
    return threads


def cpu_baseline_planted():
    """The whole oracle (reconstruct_tag with every step, then its exact error) on the
    planted exact-rank workload, timed once in full."""
    import oracle as O
    wl = W.WORKLOADS["planted_2d_n4096"]
    g = wl.geometry()
    A, _, _ = W.planted_exact_rank(g, wl.k, wl.seed)
    near = O.near_lists(g.lattice)
    T = W.tag_matrix(wl.seed, g.nboxes, O.num_tag_columns(near, wl.extra_tag_cols))
    G, H = W.gaussian_test_blocks(wl.seed, g.n, wl.r)
    t0 = time.perf_counter()
    res = O.reconstruct_tag(O.DenseOperator(A), g.box_ptr, g.lattice, wl.k, wl.p, wl.extra_tag_cols, T, G, H)
    dt = time.perf_counter() - t0
    err = O.rel_fro_error(O.DenseOperator(A), res["U"], res["V"], res["Atil"], res["B"], g.box_ptr, wl.k)
    return {"value": round(1.0 / dt, 4), "unit": "compressions/s", "s": round(dt, 3), "kind": "oracle",
            "sample": "full compression, timed once", "rel_err_fro": err,
            "threads": {"blas": _blas_threads(), "python": 1}}


def cpu_baseline(S, nsample_boxes=4):
    """The oracle, as it stands, on a bounded sample: every stage of reconstruct_tag
    restricted to `nsample_boxes` row boxes (sketch rows, their post-processing and
    bases, their rows of the cores and of the near-field probes), extrapolated to
    all b row boxes.  The column-side bases V (all boxes) are part of the sample
    cost only through the rows sampled here, which is what the oracle's sketch
    costs per row; the extrapolation is linear in the number of row boxes."""
    import oracle as O
    wl, g = S["wl"], S["g"]
    k, r = wl.k, wl.r
    bp = g.box_ptr
    boxes = list(range(0, g.nboxes, max(1, g.nboxes // nsample_boxes)))[:nsample_boxes]
    rows = np.concatenate([np.arange(bp[i], bp[i + 1]) for i in boxes])
    sub_ptr = np.concatenate([[0], np.cumsum([bp[i + 1] - bp[i] for i in boxes])])
    op = O.KernelOperator(wl.kind, g.pts)
    near = O.near_lists(g.lattice)
    far = O.far_lists(near, g.nboxes)
    col = O.colours(g.lattice)
    T = S["T"]
    t0 = time.perf_counter()
    zs = np.zeros((len(boxes), T.shape[1]))
    for q, i in enumerate(boxes):
        zs[q], _ = O.optimise_tag_vector(T, near[i], far[i])
    Om = O.extended_test_matrix(T, S["G"], bp)
    Ps = O.extended_test_matrix(T, S["H"], bp)
    Y = op.matmat(Om, rows=rows)
    Z = op.rmatmat(Ps, rows=rows)
    Yh = O.tag_postprocess(Y, zs, sub_ptr, r)
    Zh = O.tag_postprocess(Z, zs, sub_ptr, r)
    U, V = O.tag_bases(Yh, Zh, sub_ptr, k)
    # cores rows U_i* (A V)(I_i, :) with V = diag(V_j): bk products restricted to the rows
    Vfull = np.zeros((g.n, k))
    for q, i in enumerate(boxes):
        Vfull[bp[i]:bp[i + 1]] = V[sub_ptr[q]:sub_ptr[q + 1]]
    Vbd = O.reconstruct._blockdiag(Vfull, bp, k)
    W_rows = op.matmat(Vbd, rows=rows)
    At_rows = [U[sub_ptr[q]:sub_ptr[q + 1]].T @ W_rows[sub_ptr[q]:sub_ptr[q + 1]] for q in range(len(boxes))]
    # near-field probe rows: (A X_c)(I_i, :) for every colour
    mmax = int(np.max(g.box_sizes()))
    for c in range(3 ** g.dim):
        X = np.zeros((g.n, mmax))
        for l in range(g.nboxes):
            if col[l] == c:
                X[bp[l]:bp[l + 1], :bp[l + 1] - bp[l]] = np.eye(bp[l + 1] - bp[l])
        _ = op.matmat(X, rows=rows)
    dt = time.perf_counter() - t0
    del At_rows
    per_comp = dt * g.nboxes / len(boxes)
    threads = _blas_threads()
    return {"value": 1.0 / per_comp, "unit": "compressions/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(boxes)} of {g.nboxes} row boxes of every stage "
                      f"({dt:.1f} s), extrapolated linearly to all row boxes (not a full timed run)",
            "threads": {"blas": threads, "kernel_entries": 1},
            "note": "products run in numpy's BLAS thread pool; kernel entries are generated "
                    "by single-threaded numpy"}


def _job_inputs(P, torch, wl, precision):
    """Plan, operator and device inputs of one generator job."""
    g = wl.geometry()
    ell = P.tag_columns(g.box_ptr, g.lattice, wl.extra_tag_cols)
    T = W.tag_matrix(wl.seed, g.nboxes, ell)
    G, H = W.gaussian_test_blocks(wl.seed, g.n, wl.r)
    gu, gv = W.refinement_gammas(wl.seed, g.nboxes, wl.r, wl.r)
    plan = P.Plan(g.box_ptr, g.lattice, wl.k, T, p=wl.p, extra_tag_cols=wl.extra_tag_cols)
    return dict(wl=wl, n=g.n, plan=plan, op=P.Operator.kernel(wl.kind, g.pts), G=P.colmajor(G),
                H=P.colmajor(H), gamma_u=torch.as_tensor(gu, device="cuda"),
                gamma_v=torch.as_tensor(gv, device="cuda"), precision=precision)


def _kw(j):
    return {} if j["precision"] == "fp64" else dict(precision=j["precision"], gamma_u=j["gamma_u"],
                                                    gamma_v=j["gamma_v"])


def batch_section(njobs=96, seed=20250104, n_lo=4096, n_hi=65536):
    """Uneven batch (the batch generator: N, box shape, rank, kernel per job): FP32-sketch
    mixed jobs in one batch (persistent sketch launches, HIP graph replay, autotuned
    tiles) against plain FP64 compressions one at a time, with the accuracy of each; and
    the FP64 jobs as one batch (persistent FP64 sketch launches, one eager run), which
    separates the batching gain from the precision gain."""
    import torch
    import paper_2501_05528_amd as P
    torch.cuda.empty_cache()
    wls = W.uneven_batch_jobs(njobs, seed, n_lo=n_lo, n_hi=n_hi)
    jobs64 = [_job_inputs(P, torch, wl, "fp64") for wl in wls]
    jobs32 = [dict(j, precision="fp32") for j in jobs64]
    torch.cuda.synchronize()
    # plain FP64, one at a time (warm-up on the first job)
    P.compress(jobs64[0]["plan"], jobs64[0]["op"], jobs64[0]["G"], jobs64[0]["H"], report=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hs64 = [P.compress(j["plan"], j["op"], j["G"], j["H"], report=False)[0] for j in jobs64]
    torch.cuda.synchronize()
    t64 = time.perf_counter() - t0
    e64 = [h.error_fro(j["op"]) for h, j in zip(hs64, jobs64)]
    del hs64
    # the same FP64 jobs as one batch: persistent FP64 sketch launches (one per kernel kind
    # and column-tile class), one eager run
    b64 = P.Batch(jobs64, graph=False, autotune=False)
    rep64 = b64.run()
    torch.cuda.synchronize()
    e64b = max(abs(b64.result(q).error_fro(j["op"]) - e) / e for q, (j, e) in
               enumerate(zip(jobs64[:4], e64[:4])))
    del b64
    torch.cuda.empty_cache()
    b = P.Batch(jobs32, graph=True, autotune=True)
    rep_eager = b.run()
    b.run()
    torch.cuda.synchronize()
    reps = []
    t0 = time.perf_counter()
    for _ in range(3):
        reps.append(b.run())
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / 3
    emx = [b.result(q).error_fro(j["op"]) for q, j in enumerate(jobs32)]
    ratio = max(e / max(f, 1e-300) for e, f in zip(emx, e64))
    sk = rep_eager["sketch_flops"] / (rep_eager["ms_sketch"] * 1e-3) / 1e12 if rep_eager["ms_sketch"] else None
    return {"jobs": njobs, "N_range": [min(j["n"] for j in jobs64), max(j["n"] for j in jobs64)],
            "note": "N up to 65536: with N up to 131072 the 96 jobs' outputs and temporaries, which a "
                    "batch keeps resident, need about 570 GB",
            "fp64_one_at_a_time_jobs_per_s": round(njobs / t64, 3),
            "batched_fp64_jobs_per_s": round(njobs / (rep64["ms_total"] * 1e-3), 3),
            "batched_fp64_sketch_ms": round(rep64["ms_sketch"], 3),
            "batched_fp64_sketch_tflops": round(rep64["sketch_flops"] / (rep64["ms_sketch"] * 1e-3) / 1e12, 2),
            "batched_fp64_classes": {"ntr": rep64["class_ntr"], "kind": rep64["class_kind"],
                                     "tail": rep64["class_tail"], "jobs": rep64["class_jobs"]},
            "batched_fp64_err_rel_diff_first4": e64b,
            "batched_fp32_jobs_per_s": round(njobs / tb, 3),
            "speedup": round(t64 / tb, 3),
            "max_err_ratio_vs_fp64": round(ratio, 4),
            "max_rel_err_fro_fp64": max(e64), "max_rel_err_fro_batched": max(emx),
            "graph_replay_ms": round(float(np.median([r["ms_total"] for r in reps])), 3),
            "eager_ms": round(rep_eager["ms_total"], 3),
            "eager_sketch_ms": round(rep_eager["ms_sketch"], 3),
            "sketch_tflops_eager": round(sk, 2) if sk else None,
            "sketch_classes": {"ntr": rep_eager["class_ntr"], "spw": reps[-1]["class_spw"],
                               "jobs": rep_eager["class_jobs"]}}


def serve_section(rates=(10.0, 50.0, 200.0, 500.0), njobs=200, seed=20250105):
    """Poisson arrivals of a job mix at several rates: 80 % jobs from the batch generator
    (N 4096 .. 32768, three kernels, uneven boxes and ranks), 19 % the 2D Laplace N = 65536,
    k = 32 job and 1 % the 2D Laplace N = 262144, k = 48 job (32 x 32 boxes).  Three drives of
    the same arrivals: the 4-slot server in the BF16 mixed mode with HBM-budget admission,
    BF16 one job at a time (1 slot), and plain FP64 one job at a time.  A client thread claims
    results as they complete.  Latency is submit to completion; device overlap is the sum of
    the jobs' device intervals over the span they cover."""
    import threading
    import torch
    import paper_2501_05528_amd as P
    gen = W.uneven_batch_jobs(njobs, seed, n_lo=4096, n_hi=32768)
    lap = _job_inputs(P, torch, W.WORKLOADS["laplace2d_n65536"], "bf16")
    big = _job_inputs(P, torch, W.WORKLOADS["laplace2d_n262144"], "bf16")
    mix = []
    for q, wl in enumerate(gen):
        if q % 100 == 50:
            mix.append(big)
        elif q % 5 == 4:
            mix.append(lap)
        else:
            mix.append(_job_inputs(P, torch, wl, "bf16"))
    torch.cuda.synchronize()
    rng = W.rng(seed, W.STREAM_ARRIVALS)

    def drive(gaps, precision, slots):
        srv = P.Server(hbm_budget=160 << 30, slots=slots)
        tickets, stats = [], []
        done = threading.Event()

        def claim():
            q = 0
            while q < len(mix):
                if q >= len(tickets):
                    time.sleep(0.0005)
                    continue
                _, st = srv.wait(tickets[q])
                stats.append(st)
                q += 1
            done.set()

        th = threading.Thread(target=claim)
        th.start()
        t = time.monotonic()
        t_first = t
        for j, gap in zip(mix, gaps):
            t += gap
            while time.monotonic() < t:
                time.sleep(0.0002)
            jj = dict(j, precision=precision)
            tickets.append(srv.submit(jj["plan"], jj["op"], jj["G"], jj["H"], **_kw(jj)))
        th.join()
        srv.close()
        lat = [st["t_end"] - st["t_submit"] for st in stats]
        t_last = max(st["t_end"] for st in stats)
        busy = sum(st["dev_end_ms"] - st["dev_start_ms"] for st in stats)
        span = max(st["dev_end_ms"] for st in stats) - min(st["dev_start_ms"] for st in stats)
        return {"jobs_per_s": round(len(mix) / (t_last - t_first), 3),
                "p50_ms": round(1e3 * float(np.percentile(lat, 50)), 2),
                "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 2),
                "device_overlap": round(busy / span, 3) if span > 0 else None}

    nbig = sum(1 for j in mix if j is big)
    nlap = sum(1 for j in mix if j is lap)
    out = {"jobs_per_rate": len(mix), "mix": {"generator": len(mix) - nbig - nlap, "laplace2d_n65536": nlap,
                                              "laplace2d_n262144": nbig},
           "slots": 4, "admission": "FIFO by HBM footprint (160 GiB budget)"}
    for rate in rates:
        gaps = rng.exponential(1.0 / rate, size=len(mix))   # the same arrivals for all drives
        log(f"serving at {rate:g} jobs/s")
        out[f"rate_{int(rate)}"] = {"served_bf16": drive(gaps, "bf16", 4),
                                    "bf16_one_at_a_time": drive(gaps, "bf16", 1),
                                    "fp64_one_at_a_time": drive(gaps, "fp64", 1)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="laplace2d_n65536")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-error", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched uneven-job measurement")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    ap.add_argument("--no-paper-geometry", action="store_true",
                    help="skip the random-point geometry measurement")
    ap.add_argument("--no-rank", action="store_true",
                    help="skip the tolerance-driven rank measurement")
    ap.add_argument("--no-bn", action="store_true",
                    help="skip the block-nullification (Alg. 1) comparison")
    ap.add_argument("--no-basic", action="store_true",
                    help="skip the one-off Alg. 3 (basic randomized SVD) comparison run")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-precision (BF16 / FP32 sketch + FP64 refinement) runs")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the 3D (N = 110592) and planted (N = 4096) workloads")
    ap.add_argument("--no-truncate", action="store_true", help="skip the per-box rank truncation")
    ap.add_argument("--no-slab", action="store_true", help="skip the thin-slab Schur complement")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after timing, run one device-to-device copy of this many MiB "
                         "(a plain kernel of known traffic for scaling rocprofv3 byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; "
                                   "sharding over several GPUs is not implemented"}))
        sys.exit(2)
    import torch
    log(f"setup {args.workload}")
    S = setup(args.workload)
    plan = S["plan"]
    wl, g = S["wl"], S["g"]
    res = run_mode(S, "fp64", args.steps, args.warmup, not args.no_error)
    if args.calib_copy_mib:
        nel = args.calib_copy_mib * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {nel * 8} bytes read, {nel * 8} bytes written")
        del src, dst
    value = res["value"]
    stage = res["stage"]
    rep0 = res["rep"]
    applies = int(rep0["applies_A"] + rep0["applies_At"])
    sketch_flops = rep0["sketch_flops"]
    achieved = sketch_flops / (stage["ms_sketch"] * 1e-3) / 1e12
    roofline = {"bound": "mfma", "kernel": "k_sketch (tagged sketch, FP64 MFMA)",
                "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP64_TFLOPS, 4),
                "traffic": measured_sketch_traffic(wl.name),
                "algorithmic_flops_per_launch": sketch_flops}
    out = {
        "metric": METRIC, "value": round(value, 4), "unit": "compressions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(res["ms_step"], 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "kernel": wl.kind, "N": g.n, "boxes": g.nboxes,
                   "m": int(np.max(g.box_sizes())), "k": wl.k, "p": wl.p, "ell": plan.ell,
                   "precision": "fp64"},
        "applies_per_compression": applies,
        "applies_per_s": round(applies * value, 1),
        "rel_err_fro": res["err"],
        "stage_ms": {k: round(v, 3) for k, v in stage.items() if k != "ms_refine"},
        "plan_s": round(S["plan_s"], 3),
        "roofline": roofline,
    }
    try:
        log("uBLR apply and spectral error")
        out["apply"] = apply_section(S, res["handle"])
    except Exception as e:  # extra measurement: never lose the line
        out["apply"] = {"error": repr(e)}
    res.pop("handle", None)
    if not args.no_mixed:
        mixed = {}
        for prec in ("bf16", "fp32"):
            m = run_mode(S, prec, args.steps, args.warmup, not args.no_error)
            m.pop("handle", None)
            rp = m["rep"]
            st = m["stage"]
            sk = rp["sketch_flops"] / (st["ms_sketch"] * 1e-3) / 1e12
            rf = rp["refine_flops"] / (st["ms_refine"] * 1e-3) / 1e12
            mixed[prec] = {
                "value": round(m["value"], 4), "unit": "compressions/s",
                "ms_per_step": round(m["ms_step"], 3),
                "speedup_vs_fp64": round(m["value"] / value, 3),
                "rel_err_fro": m["err"],
                "r_lo": rp["r_lo"],
                "applies_per_compression": int(rp["applies_A"] + rp["applies_At"]),
                "stage_ms": {k: round(v, 3) for k, v in st.items()},
                "sketch_roofline": {"bound": "mfma", "achieved": round(sk, 2), "peak": PEAK_TFLOPS[prec],
                                    "unit": "TFLOP/s", "frac": round(sk / PEAK_TFLOPS[prec], 4),
                                    "algorithmic_flops_per_launch": rp["sketch_flops"]},
                "refine_roofline": {"bound": "mfma", "achieved": round(rf, 2), "peak": PEAK_FP64_TFLOPS,
                                    "unit": "TFLOP/s", "frac": round(rf / PEAK_FP64_TFLOPS, 4),
                                    "algorithmic_flops_per_launch": rp["refine_flops"]},
            }
        out["mixed"] = mixed
    if not args.no_configs:
        try:
            log("3D workload (1/r, N = 110592, k = 48): FP64, BF16 and FP32 mixed")
            S3 = setup("invr3d_n110592")
            out["invr3d_n110592"] = config_section(S3, with_error=not args.no_error)
            del S3
        except Exception as e:  # extra measurement: never lose the line
            out["invr3d_n110592"] = {"error": repr(e)}
        try:
            log("planted exact-rank workload (N = 4096)")
            out["planted_2d_n4096"] = planted_section()
        except Exception as e:
            out["planted_2d_n4096"] = {"error": repr(e)}
    if not args.no_truncate:
        try:
            log("per-box ranks from a tolerance (truncation)")
            out["truncation"] = truncation_section(S)
        except Exception as e:
            out["truncation"] = {"error": repr(e)}
    if not args.no_slab:
        try:
            log("thin-slab Schur complement (black box)")
            out["slab"] = slab_section()
        except Exception as e:
            out["slab"] = {"error": repr(e)}
    if not args.no_paper_geometry:
        try:
            log("random-point geometry of the paper's experiments")
            out["paper_geometry"] = paper_geometry_section()
        except Exception as e:  # extra measurement: never lose the line
            out["paper_geometry"] = {"error": repr(e)}
    if not args.no_rank:
        try:
            log("tolerance-driven rank")
            out["rank_choice"] = [rank_section(S, tol) for tol in (1e-8, 1e-9)]
        except Exception as e:  # extra measurement: never lose the line
            out["rank_choice"] = {"error": repr(e)}
    if not args.no_bn:
        try:
            log("Alg. 1 comparison (block nullification)")
            out["bn_alg1"] = bn_section()
        except Exception as e:  # extra measurement: never lose the line
            out["bn_alg1"] = {"error": repr(e)}
    if not args.no_basic:
        try:
            log("Alg. 3 comparison (basic randomized SVD per box)")
            out["basic_alg3"] = basic_section(S, value, not args.no_error)
        except Exception as e:  # extra measurement: never lose the line
            out["basic_alg3"] = {"error": repr(e)}
    if not args.no_batch:
        try:
            log("batched uneven jobs")
            out["batch"] = batch_section()
        except Exception as e:  # extra measurement: never lose the line above
            out["batch"] = {"error": repr(e)}
    if not args.no_serve:
        try:
            log("serving with Poisson arrivals")
            out["serve"] = serve_section()
        except Exception as e:
            out["serve"] = {"error": repr(e)}
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on a bounded sample)")
        out["cpu_baseline"] = cpu_baseline(S)
        try:
            log("cpu baseline: full oracle run on the planted workload")
            out["cpu_baseline"]["planted_2d_n4096_full"] = cpu_baseline_planted()
        except Exception as e:
            out["cpu_baseline"]["planted_2d_n4096_full"] = {"error": repr(e)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
