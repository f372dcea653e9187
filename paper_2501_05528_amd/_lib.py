"""ctypes declarations of the C ABI in include/blr_tag.h.

Loading fails loudly (ImportError) when ``libblrtag.so`` has not been built:
there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_void_p

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libblrtag.so")

P_i32 = POINTER(c_int32)
P_i64 = POINTER(c_int64)
P_f64 = POINTER(c_double)


class Geometry(ctypes.Structure):
    _fields_ = [("dim", c_int32), ("nboxes", c_int32), ("box_ptr", P_i64), ("box_lattice", P_i32),
                ("near_ptr", P_i32), ("near_idx", P_i32)]


class TagParams(ctypes.Structure):
    _fields_ = [("k", c_int32), ("p", c_int32), ("extra_tag_cols", c_int32),
                ("aspect_opt", c_int32), ("T", P_f64)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("n", c_int64), ("nboxes", c_int32), ("dim", c_int32), ("k", c_int32),
                ("p", c_int32), ("r", c_int32), ("ell", c_int32), ("m_max", c_int32),
                ("m_min", c_int32), ("ncolours", c_int32), ("near_nnz", c_int64),
                ("b_values", c_int64)]


class CompressOpts(ctypes.Structure):
    _fields_ = [("precision", c_int32), ("keep_intermediates", c_int32), ("r_lo", c_int32),
                ("reserved", c_int32), ("gamma_u", c_void_p), ("gamma_v", c_void_p)]


class Report(ctypes.Structure):
    _fields_ = [("ms_sketch", c_double), ("ms_postprocess", c_double), ("ms_orth", c_double),
                ("ms_cores", c_double), ("ms_nearfield", c_double), ("ms_total", c_double),
                ("applies_A", c_int64), ("applies_At", c_int64), ("sketch_flops", c_double),
                ("rho_min", c_double), ("rho_median", c_double), ("rho_max", c_double),
                ("ms_refine", c_double), ("refine_flops", c_double), ("precision", c_int32),
                ("r_lo", c_int32)]


PRECISION = {"fp64": 0, "fp32": 1, "bf16": 2}
BATCH_MAX_CLASSES = 32   # BLR_BATCH_MAX_CLASSES


class BatchJob(ctypes.Structure):
    _fields_ = [("plan", c_void_p), ("op", c_void_p), ("G", c_void_p), ("H", c_void_p),
                ("opts", CompressOpts)]


class BatchReport(ctypes.Structure):
    _fields_ = [("ms_total", c_double), ("ms_sketch", c_double), ("sketch_flops", c_double),
                ("refine_flops", c_double), ("applies", c_int64), ("graph_replayed", c_int32),
                ("nclasses", c_int32), ("class_precision", c_int32 * BATCH_MAX_CLASSES),
                ("class_ntr", c_int32 * BATCH_MAX_CLASSES), ("class_spw", c_int32 * BATCH_MAX_CLASSES),
                ("class_jobs", c_int32 * BATCH_MAX_CLASSES), ("class_kind", c_int32 * BATCH_MAX_CLASSES),
                ("class_tail", c_int32 * BATCH_MAX_CLASSES)]


class ServerJobStats(ctypes.Structure):
    _fields_ = [("t_submit", c_double), ("t_start", c_double), ("t_end", c_double),
                ("ms_device", c_double), ("dev_start_ms", c_double), ("dev_end_ms", c_double),
                ("footprint", c_int64), ("slot", c_int32), ("status", c_int32)]


BATCH_GRAPH = 1
BATCH_AUTOTUNE = 2


# int32 apply(ctx, trans, ncols, X, ldx, Y, ldy, stream): the black-box operator callback
APPLY_FN = ctypes.CFUNCTYPE(c_int32, c_void_p, c_int32, c_int64, c_void_p, c_int64, c_void_p, c_int64,
                            c_void_p)
APPLY_LP_FN = ctypes.CFUNCTYPE(c_int32, c_void_p, c_int32, c_int32, c_int64, c_void_p, c_int64, c_void_p,
                               c_int64, c_void_p)

# name -> (restype, argtypes); every symbol declared in include/blr_tag.h
SIGNATURES = {
    "blr_status_string": (c_char_p, [c_int32]),
    "blr_last_error_message": (c_char_p, []),
    "blr_version": (c_char_p, []),
    "blr_tag_columns": (c_int32, [POINTER(Geometry), c_int32, P_i32]),
    "blr_tag_plan": (c_int32, [POINTER(Geometry), POINTER(TagParams), POINTER(c_void_p)]),
    "blr_plan_destroy": (None, [c_void_p]),
    "blr_plan_query": (c_int32, [c_void_p, POINTER(PlanInfo)]),
    "blr_plan_lists": (c_int32, [c_void_p, P_i32, P_i32, P_i32, P_i64]),
    "blr_plan_tags": (c_int32, [c_void_p, P_f64, P_f64]),
    "blr_op_dense_create": (c_int32, [c_int64, c_void_p, c_int64, POINTER(c_void_p)]),
    "blr_op_kernel_create": (c_int32, [c_int32, c_int32, c_int64, P_f64, POINTER(c_void_p)]),
    "blr_op_slab_create": (c_int32, [c_int32, c_int32, c_double, P_i64, POINTER(c_void_p)]),
    "blr_op_callback_create": (c_int32, [c_int64, APPLY_FN, c_void_p, POINTER(c_void_p)]),
    "blr_op_callback_set_lp": (c_int32, [c_void_p, APPLY_LP_FN]),
    "blr_op_destroy": (None, [c_void_p]),
    "blr_op_apply": (c_int32, [c_void_p, c_int32, c_int64, c_void_p, c_int64, c_void_p, c_int64,
                               c_void_p]),
    "blr_sketch": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "blr_tag_postprocess": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "blr_orthonormalize": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "blr_cores": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "blr_nearfield": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                c_void_p]),
    "blr_sketch_lowp": (c_int32, [c_void_p, c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_void_p,
                                  c_void_p, c_void_p]),
    "blr_tag_postprocess_lowp": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p,
                                           c_void_p]),
    "blr_sample_bases": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p]),
    "blr_refine_sketch": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_void_p,
                                    c_void_p, c_void_p, c_void_p, c_void_p]),
    "blr_tag_compress": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, POINTER(CompressOpts),
                                   c_void_p, POINTER(c_void_p), POINTER(Report)]),
    "blr_basic_compress": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_void_p,
                                     POINTER(c_void_p), POINTER(Report)]),
    "blr_bn_min_columns": (c_int32, [c_void_p, P_i64]),
    "blr_bn_compress": (c_int32, [c_void_p, c_void_p, c_int64, c_void_p, c_void_p, c_int32, c_void_p,
                                  POINTER(c_void_p), POINTER(Report)]),
    "blr_tag_rank": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_void_p, P_i32,
                               POINTER(c_double)]),
    "blr_ublr_destroy": (None, [c_void_p]),
    "blr_ublr_part_ptr": (c_int32, [c_void_p, c_int32, POINTER(c_void_p), P_i64]),
    "blr_ublr_export": (c_int32, [c_void_p, c_int32, c_void_p, c_int64, c_void_p]),
    "blr_plan_footprint": (c_int32, [c_void_p, c_int32, c_int32, P_i64]),
    "blr_batch_create": (c_int32, [c_int32, POINTER(BatchJob), c_int32, POINTER(c_void_p)]),
    "blr_batch_run": (c_int32, [c_void_p, c_void_p, POINTER(BatchReport)]),
    "blr_batch_result": (c_int32, [c_void_p, c_int32, POINTER(c_void_p)]),
    "blr_batch_destroy": (None, [c_void_p]),
    "blr_server_create": (c_int32, [c_int64, c_int32, POINTER(c_void_p)]),
    "blr_server_submit": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, POINTER(CompressOpts),
                                    POINTER(ctypes.c_uint64)]),
    "blr_server_poll": (c_int32, [c_void_p, ctypes.c_uint64, P_i32]),
    "blr_server_wait": (c_int32, [c_void_p, ctypes.c_uint64, POINTER(c_void_p), POINTER(ServerJobStats)]),
    "blr_server_destroy": (None, [c_void_p]),
    "blr_apply": (c_int32, [c_void_p, c_int32, c_int64, c_void_p, c_int64, c_void_p, c_int64,
                            c_void_p]),
    "blr_apply_noalloc": (c_int32, [c_void_p, c_int32, c_int64, c_void_p, c_int64, c_void_p, c_int64,
                                    c_void_p]),
    "blr_ublr_truncate": (c_int32, [c_void_p, c_double, c_void_p, POINTER(c_void_p), P_i32, P_i32, P_f64]),
    "blr_ublr_ranks": (c_int32, [c_void_p, P_i32, P_i32]),
    "blr_error_fro": (c_int32, [c_void_p, c_void_p, c_void_p, P_f64]),
    "blr_error_power": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_void_p, P_f64, P_f64]),
}

STATUS = {0: "BLR_OK", 1: "BLR_ERR_INVALID_ARG", 2: "BLR_ERR_GEOMETRY", 3: "BLR_ERR_OOM",
          4: "BLR_ERR_DEVICE", 5: "BLR_ERR_OPERATOR", 6: "BLR_ERR_NUMERICAL", 7: "BLR_ERR_BUSY",
          8: "BLR_ERR_UNSUPPORTED"}

_LIB = None


class BlrError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.name = STATUS.get(status, str(status))


def lib():
    """The loaded library; raises ImportError if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              f"`python -m paper_2501_05528_amd.build` (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def check(status: int):
    if status != 0:
        msg = lib().blr_last_error_message()
        raise BlrError(status, msg.decode() if msg else "")
