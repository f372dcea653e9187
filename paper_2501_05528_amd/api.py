"""Thin Python binding over the C ABI (argument marshalling only).

Device matrices are torch CUDA float64 tensors of shape (rows, cols) in
column-major layout (strides (1, rows)); ``colmajor`` builds them.  Every
computation runs in the HIP library; there is no CPU path.
"""
from __future__ import annotations

import ctypes
from ctypes import byref, c_double, c_int32, c_int64, c_void_p

import numpy as np

from . import _lib
from ._lib import BlrError, check, lib  # noqa: F401

KERNELS = {"log": 0, "inv_r": 1, "exp": 2, "cos": 3}
PARTS = {"U": 0, "V": 1, "Atil": 2, "B": 3, "Y": 4, "Z": 5, "Yhat": 6, "Zhat": 7,
         "Y0": 8, "Z0": 9, "U0": 10, "V0": 11, "SY": 12, "SZ": 13}
PRECISIONS = dict(_lib.PRECISION)


def _torch():
    import torch
    return torch


def colmajor_empty(rows: int, cols: int, device=None, dtype=None):
    torch = _torch()
    return torch.empty((cols, rows), dtype=dtype or torch.float64, device=device or "cuda").t()


def colmajor(a, device=None):
    """Copy a 2-D array (numpy or torch) to a column-major CUDA float64 tensor."""
    torch = _torch()
    t = torch.as_tensor(np.asarray(a) if not isinstance(a, torch.Tensor) else a)
    if t.dim() == 1:
        t = t[:, None]
    out = colmajor_empty(t.shape[0], t.shape[1], device)
    out.copy_(t.to(torch.float64))
    return out


class _DeviceView:
    """Column-major (rows x cols) float64 (or float32) device memory owned by the library."""

    def __init__(self, ptr: int, rows: int, cols: int, itemsize: int = 8, ld: int = 0):
        self.__cuda_array_interface__ = {"shape": (rows, cols), "typestr": f"<f{itemsize}",
                                         "data": (ptr, False), "version": 2,
                                         "strides": (itemsize, itemsize * max(ld, rows))}


def colmajor_copy(t):
    out = colmajor_empty(t.shape[0], t.shape[1], t.device, t.dtype)
    out.copy_(t)
    return out


def _ptr(t):
    return c_void_p(t.data_ptr()) if t is not None else c_void_p(0)


def _ld(t):
    """Leading dimension of a column-major (rows, cols) tensor."""
    if t.dim() != 2:
        raise ValueError("expected a 2-D tensor")
    if t.stride(0) != 1 and t.shape[1] > 1:
        raise ValueError("expected a column-major tensor (stride(0) == 1)")
    return max(t.stride(1), t.shape[0]) if t.shape[1] > 1 else t.shape[0]


def _stream(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return c_void_p(s.cuda_stream)


def near_csr(near):
    """(near_ptr, near_idx) int32 arrays from neighbour lists (a list of index lists, or a
    (ptr, idx) pair)."""
    if isinstance(near, tuple) and len(near) == 2 and not isinstance(near[0], (list, tuple)):
        return np.ascontiguousarray(near[0], np.int32), np.ascontiguousarray(near[1], np.int32)
    ptr = np.zeros(len(near) + 1, np.int32)
    ptr[1:] = np.cumsum([len(n) for n in near])
    idx = np.ascontiguousarray(np.concatenate([np.asarray(n, np.int32) for n in near]), np.int32)
    return ptr, idx


def _geometry(box_ptr, lattice, near=None):
    """blr_geometry for box_ptr and a lattice (b x d) and/or explicit neighbour lists."""
    bp = np.ascontiguousarray(box_ptr, dtype=np.int64)
    b = len(bp) - 1
    keep = [bp]
    if lattice is not None:
        lat = np.ascontiguousarray(lattice, dtype=np.int32)
        if lat.ndim != 2 or lat.shape[0] != b:
            raise ValueError("lattice must be b x d")
        dim, latp = lat.shape[1], lat.ctypes.data_as(_lib.P_i32)
        keep.append(lat)
    elif near is not None:
        dim, latp = 1, ctypes.cast(None, _lib.P_i32)
    else:
        raise ValueError("need a lattice or explicit neighbour lists")
    if near is not None:
        nptr, nidx = near_csr(near)
        keep += [nptr, nidx]
        np_p, ni_p = nptr.ctypes.data_as(_lib.P_i32), nidx.ctypes.data_as(_lib.P_i32)
    else:
        np_p = ni_p = ctypes.cast(None, _lib.P_i32)
    g = _lib.Geometry(dim, b, bp.ctypes.data_as(_lib.P_i64), latp, np_p, ni_p)
    return g, keep


def tag_columns(box_ptr, lattice, extra_tag_cols: int = 3, near=None) -> int:
    g, keep = _geometry(box_ptr, lattice, near)
    ell = c_int32()
    check(lib().blr_tag_columns(byref(g), extra_tag_cols, byref(ell)))
    return ell.value


class Plan:
    """Host plan: lists, colours, tag vectors z and aspect ratios rho."""

    def __init__(self, box_ptr, lattice, k: int, T, p: int = 10, extra_tag_cols: int = 3,
                 aspect_opt: bool = True, near=None):
        g, keep = _geometry(box_ptr, lattice, near)
        Tf = np.asfortranarray(T, dtype=np.float64)
        prm = _lib.TagParams(k, p, extra_tag_cols, 1 if aspect_opt else 0,
                             Tf.ctypes.data_as(_lib.P_f64))
        h = c_void_p()
        ell = tag_columns(box_ptr, lattice, extra_tag_cols, near)
        if Tf.shape != (g.nboxes, ell):
            raise ValueError(f"T must be {g.nboxes} x {ell}, got {Tf.shape}")
        check(lib().blr_tag_plan(byref(g), byref(prm), byref(h)))
        self._h = h
        self._lib = lib()      # kept so that destruction at interpreter exit needs no module globals
        info = _lib.PlanInfo()
        check(lib().blr_plan_query(h, byref(info)))
        self.info = {f: getattr(info, f) for f, _ in _lib.PlanInfo._fields_}
        self.n = info.n
        self.b = info.nboxes
        self.k, self.r, self.ell = info.k, info.r, info.ell

    def lists(self):
        i = self.info
        near_ptr = np.zeros(self.b + 1, np.int32)
        near_idx = np.zeros(i["near_nnz"], np.int32)
        colour = np.zeros(self.b, np.int32)
        boff = np.zeros(i["near_nnz"], np.int64)
        check(lib().blr_plan_lists(self._h, near_ptr.ctypes.data_as(_lib.P_i32),
                                   near_idx.ctypes.data_as(_lib.P_i32),
                                   colour.ctypes.data_as(_lib.P_i32),
                                   boff.ctypes.data_as(_lib.P_i64)))
        return near_ptr, near_idx, colour, boff

    def tags(self):
        z = np.zeros((self.b, self.ell), order="F")
        rho = np.zeros(self.b)
        check(lib().blr_plan_tags(self._h, z.ctypes.data_as(_lib.P_f64), rho.ctypes.data_as(_lib.P_f64)))
        return z, rho

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and getattr(self, "_lib", None) is not None:
            self._lib.blr_plan_destroy(h)
            self._h = None


class Operator:
    """A black-box operator held by the library (dense or kernel matrix)."""

    def __init__(self, handle, n, keep=None):
        self._h = handle
        self._lib = lib()      # kept so that destruction at interpreter exit needs no module globals
        self.n = n
        self._keep = keep

    @classmethod
    def dense(cls, A):
        """A: column-major CUDA float64 tensor n x n (borrowed; kept alive here)."""
        h = c_void_p()
        check(lib().blr_op_dense_create(A.shape[0], _ptr(A), _ld(A), byref(h)))
        return cls(h, A.shape[0], keep=A)

    @classmethod
    def kernel(cls, kind: str, pts):
        p = np.ascontiguousarray(pts, dtype=np.float64)
        h = c_void_p()
        check(lib().blr_op_kernel_create(KERNELS[kind], p.shape[1], p.shape[0],
                                         p.ctypes.data_as(_lib.P_f64), byref(h)))
        return cls(h, p.shape[0])

    @classmethod
    def slab(cls, n: int, l: int, perm, kappa_h: float = 2.0 * np.pi / 100.0):
        """Thin-slab Schur complement (blr_op_slab_create): n x n x l grid, frontal face
        z = l - 1, perm[row] = plane index x + n y of operator row ``row``."""
        pm = np.ascontiguousarray(perm, dtype=np.int64)
        h = c_void_p()
        check(lib().blr_op_slab_create(int(n), int(l), float(kappa_h), pm.ctypes.data_as(_lib.P_i64), byref(h)))
        return cls(h, int(n) * int(n))

    @classmethod
    def from_matmat(cls, n: int, matmat, matmat_lp=None):
        """A black-box operator from the caller's products: ``matmat(X, trans)`` gets a
        column-major CUDA float64 tensor X (n x ncols) and returns A X (or A* X when
        ``trans``) as a tensor of the same shape.  The library calls it on its stream
        (made current here) for every product it needs.  ``matmat_lp(X, trans, precision)``
        (optional, mixed modes) gets and returns float32 tensors, precision "fp32" or "bf16"."""
        torch = _torch()

        def _apply(ctx, trans, ncols, xp, ldx, yp, ldy, stream):
            try:
                X = torch.as_tensor(_DeviceView(xp, n, ncols, 8, ldx), device="cuda")
                Y = torch.as_tensor(_DeviceView(yp, n, ncols, 8, ldy), device="cuda")
                if stream:
                    with torch.cuda.stream(torch.cuda.ExternalStream(stream)):
                        Y.copy_(matmat(X, bool(trans)))
                else:
                    # the library runs on the null stream: torch's work on its default
                    # stream is not ordered before the library's next step, so wait here
                    Y.copy_(matmat(X, bool(trans)))
                    torch.cuda.synchronize()
                return 0
            except Exception:  # reported to the caller as BLR_ERR_OPERATOR
                return 1

        fn = _lib.APPLY_FN(_apply)
        h = c_void_p()
        check(lib().blr_op_callback_create(n, fn, None, byref(h)))
        if matmat_lp is None:
            return cls(h, n, keep=fn)
        names = {v: k for k, v in PRECISIONS.items()}

        def _apply_lp(ctx, trans, precision, ncols, xp, ldx, yp, ldy, stream):
            try:
                X = torch.as_tensor(_DeviceView(xp, n, ncols, 4, ldx), device="cuda")
                Y = torch.as_tensor(_DeviceView(yp, n, ncols, 4, ldy), device="cuda")
                prec = names[int(precision)]
                if stream:
                    with torch.cuda.stream(torch.cuda.ExternalStream(stream)):
                        Y.copy_(matmat_lp(X, bool(trans), prec))
                else:
                    Y.copy_(matmat_lp(X, bool(trans), prec))
                    torch.cuda.synchronize()
                return 0
            except Exception:  # reported to the caller as BLR_ERR_OPERATOR
                return 1

        fn_lp = _lib.APPLY_LP_FN(_apply_lp)
        op = cls(h, n, keep=(fn, fn_lp))
        check(lib().blr_op_callback_set_lp(h, fn_lp))
        return op

    def apply(self, X, trans: bool = False, stream=None):
        Y = colmajor_empty(self.n, X.shape[1], X.device)
        check(lib().blr_op_apply(self._h, 1 if trans else 0, X.shape[1], _ptr(X), _ld(X), _ptr(Y),
                                 _ld(Y), _stream(stream)))
        return Y

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and getattr(self, "_lib", None) is not None:
            self._lib.blr_op_destroy(h)
            self._h = None


class UBLR:
    """Compressed A ~ U Atil V* + B owned by the library."""

    def __init__(self, handle, plan: Plan, precision: str = "fp64", r_lo: int = 0, owner=None):
        self._h = handle
        self._lib = lib()      # kept so that destruction at interpreter exit needs no module globals
        self.plan = plan
        self.precision = precision
        self.r_lo = r_lo or plan.r
        self._owner = owner        # a Batch that owns the handle (then it is not destroyed here)

    def part_ptr(self, name: str):
        ptr = c_void_p()
        cnt = c_int64()
        check(lib().blr_ublr_part_ptr(self._h, PARTS[name], byref(ptr), byref(cnt)))
        return ptr.value, cnt.value

    def part(self, name: str):
        """A copy of one part as a torch CUDA tensor (matrices column-major)."""
        torch = _torch()
        ptr, cnt = self.part_ptr(name)
        n, k, r, ell, b = self.plan.n, self.plan.k, self.plan.r, self.plan.ell, self.plan.b
        rs = self.r_lo if self.precision != "fp64" else r
        shapes = {"U": (n, k), "V": (n, k), "Atil": (b * k, b * k), "B": (cnt, 1),
                  "Y": (n, ell * r), "Z": (n, ell * r), "Yhat": (n, rs), "Zhat": (n, rs),
                  "Y0": (n, ell * rs), "Z0": (n, ell * rs), "U0": (n, rs), "V0": (n, rs),
                  "SY": (n, r), "SZ": (n, r)}
        rows, cols = shapes[name]
        itemsize = 4 if name in ("Y0", "Z0") else 8
        view = torch.as_tensor(_DeviceView(ptr, rows, cols, itemsize), device="cuda")
        return view.clone(memory_format=torch.preserve_format) if cols == 1 else \
            colmajor_copy(view)

    def export(self, name: str, stream=None):
        """A host (numpy) copy of one part, matrices column-major (Fortran order)."""
        _, cnt = self.part_ptr(name)
        dt = np.float32 if name in ("Y0", "Z0") else np.float64
        out = np.empty(cnt, dtype=dt)
        check(lib().blr_ublr_export(self._h, PARTS[name], out.ctypes.data_as(c_void_p), cnt, _stream(stream)))
        return out

    def apply(self, x, trans: bool = False, stream=None, out=None, noalloc: bool = False):
        """y = A_uBLR x (or A_uBLR* x).  ``out``: optional column-major N x ncols result
        buffer; ``noalloc``: use blr_apply_noalloc (library-held workspace, no allocation)."""
        y = colmajor_empty(self.plan.n, x.shape[1], x.device) if out is None else out
        fn = lib().blr_apply_noalloc if noalloc else lib().blr_apply
        check(fn(self._h, 1 if trans else 0, x.shape[1], _ptr(x), _ld(x), _ptr(y), _ld(y), _stream(stream)))
        return y

    def truncate(self, tol: float, stream=None):
        """Per-box ranks from a tolerance (blr_ublr_truncate): (UBLR, ranks_u, ranks_v,
        rel_change) with the ranks as numpy int32 arrays of b."""
        b = self.plan.b
        ku = np.zeros(b, dtype=np.int32)
        kv = np.zeros(b, dtype=np.int32)
        ch = c_double()
        h = c_void_p()
        check(lib().blr_ublr_truncate(self._h, float(tol), _stream(stream), byref(h),
                                      ku.ctypes.data_as(_lib.P_i32), kv.ctypes.data_as(_lib.P_i32), byref(ch)))
        return UBLR(h, self.plan, self.precision, self.r_lo), ku, kv, ch.value

    def ranks(self):
        """(ranks_u, ranks_v): per-box ranks (k everywhere unless truncated)."""
        b = self.plan.b
        ku = np.zeros(b, dtype=np.int32)
        kv = np.zeros(b, dtype=np.int32)
        check(lib().blr_ublr_ranks(self._h, ku.ctypes.data_as(_lib.P_i32), kv.ctypes.data_as(_lib.P_i32)))
        return ku, kv

    def error_fro(self, op: Operator, stream=None) -> float:
        e = c_double()
        check(lib().blr_error_fro(self._h, op._h, _stream(stream), byref(e)))
        return e.value

    def error_power(self, op: Operator, x0, iters: int = 20, stream=None):
        e, a = c_double(), c_double()
        check(lib().blr_error_power(self._h, op._h, _ptr(x0), iters, _stream(stream), byref(e), byref(a)))
        return e.value, a.value

    def __del__(self):
        h = getattr(self, "_h", None)
        owned = getattr(self, "_owner", None) is None
        if h is not None and h.value and owned and getattr(self, "_lib", None) is not None:
            self._lib.blr_ublr_destroy(h)
            self._h = None


def footprint(plan: Plan, precision: str = "fp64", r_lo: int = 0) -> int:
    """Device bytes of one compression on this plan (outputs and temporaries)."""
    b = c_int64()
    check(lib().blr_plan_footprint(plan._h, PRECISIONS[precision], r_lo, byref(b)))
    return b.value


class Batch:
    """Many compressions in one object: persistent low-precision sketch launches across
    jobs, optional HIP-graph replay and autotuned sketch tiles (blr_batch_*).

    jobs: list of dicts with keys plan, op, G, H and, for mixed jobs, precision
    ("bf16"/"fp32"), gamma_u, gamma_v (CUDA float64 tensors; kept alive here)."""

    def __init__(self, jobs, graph: bool = False, autotune: bool = True):
        arr = (_lib.BatchJob * len(jobs))()
        self._keep = []
        self._meta = []
        for q, jb in enumerate(jobs):
            prec = jb.get("precision", "fp64")
            mixed = prec != "fp64"
            G, H = jb["G"], jb["H"]
            r_lo = G.shape[1] if mixed else 0
            gu, gv = jb.get("gamma_u"), jb.get("gamma_v")
            opts = _lib.CompressOpts(PRECISIONS[prec], 0, r_lo, 0, _ptr(gu).value if mixed else None,
                                     _ptr(gv).value if mixed else None)
            arr[q] = _lib.BatchJob(jb["plan"]._h.value, jb["op"]._h.value, _ptr(G).value, _ptr(H).value, opts)
            self._keep.append((jb["plan"], jb["op"], G, H, gu, gv))
            self._meta.append((jb["plan"], prec, r_lo))
        flags = (_lib.BATCH_GRAPH if graph else 0) | (_lib.BATCH_AUTOTUNE if autotune else 0)
        h = c_void_p()
        check(lib().blr_batch_create(len(jobs), arr, flags, byref(h)))
        self._h = h
        self._lib = lib()      # kept so that destruction at interpreter exit needs no module globals
        self.njobs = len(jobs)

    def run(self, stream=None):
        rep = _lib.BatchReport()
        check(lib().blr_batch_run(self._h, _stream(stream), byref(rep)))
        out = {f: getattr(rep, f) for f, _ in _lib.BatchReport._fields_}
        nc = rep.nclasses
        for f in ("class_precision", "class_ntr", "class_spw", "class_jobs", "class_kind", "class_tail"):
            out[f] = list(getattr(rep, f))[:nc]
        return out

    def result(self, j: int) -> UBLR:
        h = c_void_p()
        check(lib().blr_batch_result(self._h, j, byref(h)))
        plan, prec, r_lo = self._meta[j]
        return UBLR(h, plan, prec, r_lo, owner=self)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and getattr(self, "_lib", None) is not None:
            self._lib.blr_batch_destroy(h)
            self._h = None


class Server:
    """Request loop for compression jobs (blr_server_*): FIFO admission by free slot and
    HBM budget, concurrent slots on their own streams."""

    def __init__(self, hbm_budget: int, slots: int = 4):
        h = c_void_p()
        check(lib().blr_server_create(int(hbm_budget), slots, byref(h)))
        self._h = h
        self._lib = lib()      # kept so that destruction at interpreter exit needs no module globals
        self._pending = {}

    def submit(self, plan: Plan, op: Operator, G, H, precision: str = "fp64", gamma_u=None,
               gamma_v=None) -> int:
        mixed = precision != "fp64"
        r_lo = G.shape[1] if mixed else 0
        opts = _lib.CompressOpts(PRECISIONS[precision], 0, r_lo, 0, _ptr(gamma_u).value if mixed else None,
                                 _ptr(gamma_v).value if mixed else None)
        t = ctypes.c_uint64()
        check(lib().blr_server_submit(self._h, plan._h, op._h, _ptr(G), _ptr(H), byref(opts), byref(t)))
        self._pending[t.value] = (plan, op, G, H, gamma_u, gamma_v, precision, r_lo)
        return t.value

    def done(self, ticket: int) -> bool:
        d = c_int32()
        check(lib().blr_server_poll(self._h, ticket, byref(d)))
        return bool(d.value)

    def wait(self, ticket: int):
        """(UBLR, stats dict); raises BlrError if the job failed."""
        h = c_void_p()
        st = _lib.ServerJobStats()
        status = lib().blr_server_wait(self._h, ticket, byref(h), byref(st))
        plan, op, G, H, gu, gv, prec, r_lo = self._pending.pop(ticket)
        stats = {f: getattr(st, f) for f, _ in _lib.ServerJobStats._fields_}
        check(status)
        return UBLR(h, plan, prec, r_lo), stats

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and getattr(self, "_lib", None) is not None:
            self._lib.blr_server_destroy(h)
            self._h = None
        self._pending = {}

    def __del__(self):
        self.close()


def compress(plan: Plan, op: Operator, G, H, keep_intermediates: bool = False, report: bool = True,
             stream=None, precision: str = "fp64", gamma_u=None, gamma_v=None):
    """reconstruct_tag (Table 1).  Returns (UBLR, report dict or None).

    precision "fp32" / "bf16" selects a mixed mode: G and H are N x r_lo (r_lo =
    their column count) and gamma_u, gamma_v are C-contiguous CUDA float64 tensors
    b x r_lo x r for the refinement sketch."""
    mixed = precision != "fp64"
    r_lo = G.shape[1] if mixed else 0
    if mixed:
        for g in (gamma_u, gamma_v):
            if g is None or not g.is_contiguous() or tuple(g.shape) != (plan.b, r_lo, plan.r):
                raise ValueError(f"gamma blocks must be contiguous {plan.b} x {r_lo} x {plan.r}")
    opts = _lib.CompressOpts(PRECISIONS[precision], 1 if keep_intermediates else 0, r_lo, 0,
                             _ptr(gamma_u).value if mixed else None,
                             _ptr(gamma_v).value if mixed else None)
    h = c_void_p()
    rep = _lib.Report()
    check(lib().blr_tag_compress(plan._h, op._h, _ptr(G), _ptr(H), byref(opts), _stream(stream),
                                 byref(h), byref(rep) if report else None))
    out = UBLR(h, plan, precision, r_lo)
    rd = {f: getattr(rep, f) for f, _ in _lib.Report._fields_} if report else None
    return out, rd


def basic_compress(plan: Plan, op: Operator, G, H, keep_samples: bool = False, report: bool = True,
                   stream=None):
    """Alg. 3 (basic randomized SVD per box) for step (I), then steps (II)-(III) of
    Table 1.  G and H: N x r column-major CUDA float64, masked per box inside the
    library.  Returns (UBLR, report dict or None); keep_samples keeps parts "SY",
    "SZ" (each box's own rows of its two products)."""
    h = c_void_p()
    rep = _lib.Report()
    check(lib().blr_basic_compress(plan._h, op._h, _ptr(G), _ptr(H), 1 if keep_samples else 0,
                                   _stream(stream), byref(h), byref(rep) if report else None))
    out = UBLR(h, plan)
    rd = {f: getattr(rep, f) for f, _ in _lib.Report._fields_} if report else None
    return out, rd


def bn_min_columns(plan: Plan) -> int:
    """The smallest test-matrix width s for block nullification (Alg. 1) on ``plan``."""
    v = ctypes.c_int64()
    check(lib().blr_bn_min_columns(plan._h, byref(v)))
    return v.value


def bn_compress(plan: Plan, op: Operator, Omega, Psi, keep_samples: bool = False, report: bool = True,
                stream=None):
    """Alg. 1 (block nullification) for step (I), then steps (II)-(III) of Table 1.
    Omega and Psi: N x s column-major CUDA float64 with s >= bn_min_columns(plan).
    Returns (UBLR, report dict or None); keep_samples keeps parts "SY", "SZ"."""
    h = c_void_p()
    rep = _lib.Report()
    check(lib().blr_bn_compress(plan._h, op._h, Omega.shape[1], _ptr(Omega), _ptr(Psi),
                                1 if keep_samples else 0, _stream(stream), byref(h),
                                byref(rep) if report else None))
    out = UBLR(h, plan)
    rd = {f: getattr(rep, f) for f, _ in _lib.Report._fields_} if report else None
    return out, rd


def tag_rank(plan: Plan, op: Operator, G, H, tol: float, stream=None):
    """Tolerance-driven uniform rank from one tagged sketch at the plan's r columns.
    Returns (k, sigma) with sigma a 2 x b x r numpy array (Y side, Z side)."""
    k = c_int32()
    sig = np.zeros((2, plan.b, plan.r))
    check(lib().blr_tag_rank(plan._h, op._h, _ptr(G), _ptr(H), float(tol), _stream(stream), byref(k),
                             sig.ctypes.data_as(ctypes.POINTER(c_double))))
    return k.value, sig


# ---------------------------------------------------------------- stages
def sketch(plan: Plan, op: Operator, G, H, stream=None):
    LR = plan.ell * plan.r
    Y = colmajor_empty(plan.n, LR, G.device)
    Z = colmajor_empty(plan.n, LR, G.device)
    check(lib().blr_sketch(plan._h, op._h, _ptr(G), _ptr(H), _ptr(Y), _ptr(Z), _stream(stream)))
    return Y, Z


def postprocess(plan: Plan, Y, Z, stream=None):
    Yh = colmajor_empty(plan.n, plan.r, Y.device)
    Zh = colmajor_empty(plan.n, plan.r, Z.device)
    check(lib().blr_tag_postprocess(plan._h, _ptr(Y), _ptr(Z), _ptr(Yh), _ptr(Zh), _stream(stream)))
    return Yh, Zh


def orthonormalize(plan: Plan, S, stream=None):
    """Q (N x k) and sigma (b x r) from the per-box samples in S (S is consumed)."""
    torch = _torch()
    Q = colmajor_empty(plan.n, plan.k, S.device)
    sig = torch.empty((plan.b, plan.r), dtype=torch.float64, device=S.device)
    check(lib().blr_orthonormalize(plan._h, _ptr(S), _ptr(Q), _ptr(sig), _stream(stream)))
    return Q, sig


def cores(plan: Plan, op: Operator, U, V, stream=None):
    bk = plan.b * plan.k
    At = colmajor_empty(bk, bk, U.device)
    check(lib().blr_cores(plan._h, op._h, _ptr(U), _ptr(V), _ptr(At), _stream(stream)))
    return At


def nearfield(plan: Plan, op: Operator, U, V, Atil, stream=None):
    torch = _torch()
    Bv = torch.empty(plan.info["b_values"], dtype=torch.float64, device=U.device)
    check(lib().blr_nearfield(plan._h, op._h, _ptr(U), _ptr(V), _ptr(Atil), _ptr(Bv), _stream(stream)))
    return Bv


# ---------------------------------------------------------------- mixed-precision stages
def sketch_lowp(plan: Plan, op: Operator, precision: str, G, H, stream=None):
    """Low-precision tagged sketches (FP32 results, N x ell r_lo each)."""
    torch = _torch()
    r_lo = G.shape[1]
    LR = plan.ell * r_lo
    Y = colmajor_empty(plan.n, LR, G.device, torch.float32)
    Z = colmajor_empty(plan.n, LR, G.device, torch.float32)
    check(lib().blr_sketch_lowp(plan._h, op._h, PRECISIONS[precision], r_lo, _ptr(G), _ptr(H),
                                _ptr(Y), _ptr(Z), _stream(stream)))
    return Y, Z


def postprocess_lowp(plan: Plan, r_lo: int, Y0, Z0, stream=None):
    Yh = colmajor_empty(plan.n, r_lo, Y0.device)
    Zh = colmajor_empty(plan.n, r_lo, Z0.device)
    check(lib().blr_tag_postprocess_lowp(plan._h, r_lo, _ptr(Y0), _ptr(Z0), _ptr(Yh), _ptr(Zh),
                                         _stream(stream)))
    return Yh, Zh


def sample_bases(plan: Plan, S, stream=None):
    """Per-box Householder Q of the N x c samples in S (S is consumed)."""
    Q = colmajor_empty(plan.n, S.shape[1], S.device)
    check(lib().blr_sample_bases(plan._h, S.shape[1], _ptr(S), _ptr(Q), _stream(stream)))
    return Q


def refine_sketch(plan: Plan, op: Operator, U0, V0, gamma_u, gamma_v, stream=None):
    """Far-field refinement samples SY, SZ (N x r) on the mixed sample bases."""
    SY = colmajor_empty(plan.n, plan.r, U0.device)
    SZ = colmajor_empty(plan.n, plan.r, U0.device)
    check(lib().blr_refine_sketch(plan._h, op._h, U0.shape[1], _ptr(U0), _ptr(V0), _ptr(gamma_u),
                                  _ptr(gamma_v), _ptr(SY), _ptr(SZ), _stream(stream)))
    return SY, SZ
