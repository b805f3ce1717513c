"""ctypes declarations of the C ABI in include/ifgf.h."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libifgf.so")
MAX_LEVELS = 12
BATCH_MAX = 64

OK, EINVAL, EDUPLICATE, ENOMEM, EHIP, EUNSUPPORTED, EBUSY, EINTERNAL = range(8)
PREC_FP64, PREC_FP32_INTERP = 0, 1
C64, C128 = 0, 1
KERNEL_COMBINED, KERNEL_CONSTANT = 0, 1
PROP_AUTO, PROP_NODE, PROP_CONE, PROP_PAIRS = 0, 1, 2, 3
TARGET_AUTO, TARGET_WAVE, TARGET_ROWS, TARGET_PAIRS = 0, 1, 2, 3
STAGES = ["gather", "near", "leaf", "coeffs", "prop", "targets", "adj_targets", "adj_prop", "adj_coeffs",
          "adj_leaf", "adj_near", "adj_out", "prop_cone"]


class Options(ctypes.Structure):
    _fields_ = [
        ("p_s", ctypes.c_int32),
        ("p_ang", ctypes.c_int32),
        ("ns0", ctypes.c_int32),
        ("nc0", ctypes.c_int32),
        ("depth", ctypes.c_int32),
        ("leaf_h_lambda", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("max_rhs", ctypes.c_int32),
        ("kernel", ctypes.c_int32),
        ("prop_kernel", ctypes.c_int32),
        ("target_kernel", ctypes.c_int32),
        ("far_field", ctypes.c_int32),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("depth", ctypes.c_int32),
        ("n", ctypes.c_int64),
        ("root_side", ctypes.c_double),
        ("root_corner", ctypes.c_double * 3),
        ("p_s", ctypes.c_int32),
        ("p_ang", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("boxes", ctypes.c_int64 * MAX_LEVELS),
        ("ns", ctypes.c_int32 * MAX_LEVELS),
        ("nc", ctypes.c_int32 * MAX_LEVELS),
        ("cones", ctypes.c_int64 * MAX_LEVELS),
        ("cousin_pairs", ctypes.c_int64 * MAX_LEVELS),
        ("near_pairs", ctypes.c_int64),
        ("prop_evals", ctypes.c_int64 * MAX_LEVELS),
        ("device_bytes", ctypes.c_int64),
        ("prop_kernel", ctypes.c_int32 * MAX_LEVELS),
        ("pair_rows", ctypes.c_int64 * MAX_LEVELS),
        ("pair_row_cones", ctypes.c_int64 * MAX_LEVELS),
    ]


class GmresOptions(ctypes.Structure):
    _fields_ = [
        ("restart", ctypes.c_int32),
        ("max_iter", ctypes.c_int32),
        ("tol", ctypes.c_double),
        ("alpha_re", ctypes.c_double),
        ("alpha_im", ctypes.c_double),
        ("use_guess", ctypes.c_int32),
    ]


class TuneReport(ctypes.Structure):
    _fields_ = [
        ("nlevels", ctypes.c_int32),
        ("parent_level", ctypes.c_int32 * MAX_LEVELS),
        ("choice", ctypes.c_int32 * MAX_LEVELS),
        ("ms", (ctypes.c_double * 5) * MAX_LEVELS),
        ("target_choice", ctypes.c_int32),
        ("target_ms", ctypes.c_double * 3),
    ]


VP = ctypes.c_void_p
I32, I64, F64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double

# name -> (restype, argtypes)
SIGNATURES = {
    "ifgf_options_default": (None, [ctypes.POINTER(Options)]),
    "ifgf_plan_create": (I32, [ctypes.POINTER(VP), I64, VP, VP, VP, F64, F64, ctypes.POINTER(Options), VP]),
    "ifgf_plan_create_targets": (I32, [ctypes.POINTER(VP), I64, VP, VP, VP, I64, VP, F64, F64,
                                       ctypes.POINTER(Options), VP]),
    "ifgf_apply": (I32, [VP, VP, VP, I32, I32, VP]),
    "ifgf_apply_adjoint": (I32, [VP, VP, VP, I32, I32, I32, VP]),
    "ifgf_apply_stages": (I32, [VP, VP, VP, I32, I32, I32, I32, I32, VP]),
    "ifgf_plan_get_stats": (I32, [VP, ctypes.POINTER(Stats)]),
    "ifgf_plan_export_order": (I32, [VP, VP, VP]),
    "ifgf_plan_export_boxes": (I32, [VP, I32, VP, VP]),
    "ifgf_plan_export_lists": (I32, [VP, I32, I32, VP, VP, ctypes.POINTER(I64)]),
    "ifgf_plan_export_cones": (I32, [VP, I32, VP, VP]),
    "ifgf_plan_export_field": (I32, [VP, I32, I32, VP]),
    "ifgf_plan_check": (I32, [VP, ctypes.POINTER(I32)]),
    "ifgf_plan_set_profiling": (I32, [VP, I32]),
    "ifgf_plan_read_profile": (I32, [VP, VP, VP]),
    "ifgf_plan_destroy": (None, [VP]),
    "ifgf_far_field": (I32, [VP, VP, I64, VP, VP, I32, VP]),
    "ifgf_plan_autotune": (I32, [VP, I32, ctypes.POINTER(TuneReport), VP]),
    "ifgf_gmres_options_default": (None, [ctypes.POINTER(GmresOptions)]),
    "ifgf_gmres_solve": (I32, [VP, VP, VP, ctypes.POINTER(GmresOptions), ctypes.POINTER(I32),
                               ctypes.POINTER(F64), VP, VP]),
    "ifgf_batch_create": (I32, [ctypes.POINTER(VP), I32, ctypes.POINTER(VP)]),
    "ifgf_batch_apply": (I32, [VP, ctypes.POINTER(VP), ctypes.POINTER(VP), I32, VP]),
    "ifgf_batch_apply_noalloc": (I32, [VP, ctypes.POINTER(VP), ctypes.POINTER(VP), I32, VP]),
    "ifgf_batch_check": (I32, [VP, ctypes.POINTER(I32)]),
    "ifgf_batch_set_spin_limit": (I32, [VP, I32]),
    "ifgf_batch_get_info": (I32, [VP, ctypes.POINTER(I64), ctypes.POINTER(I32), ctypes.POINTER(I32),
                                  ctypes.POINTER(I32)]),
    "ifgf_batch_destroy": (None, [VP]),
    "ifgf_status_string": (ctypes.c_char_p, [I32]),
    "ifgf_last_error": (ctypes.c_char_p, []),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load libifgf.so and declare its signatures; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class IFGFError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: status {status} ({msg})")
        self.status = status


def check(status: int, where: str):
    if status != OK:
        lib = load()
        msg = lib.ifgf_last_error().decode() or lib.ifgf_status_string(status).decode()
        raise IFGFError(status, where, msg)
