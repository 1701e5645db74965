"""ctypes declarations of the hspmm C ABI (include/hspmm.h).

The library is loaded from this package directory only; there is no
fallback: a missing or unloadable library raises at import of the product
entry points.
"""
from __future__ import annotations

import ctypes
from pathlib import Path

LIB_PATH = Path(__file__).resolve().parent / "libhspmm.so"

F64, F32, F16, BF16 = 0, 1, 2, 3
SPLIT = {"auto": 0, "csr": 1, "csr_only": 1, "bcsr": 2, "bcsr_only": 2, "boundary": 3, "eq1": 3}
R_MEASURED = -2  # BOUNDARY with Eq. 1 solved on throughputs measured at plan time

FIELDS = {
    "rb_class": 0, "rb_nnz": 1, "rb_nblk": 2, "csr_rows": 3, "csr_ptr": 4, "csr_col": 5,
    "csr_val": 6, "bcsr_rb": 7, "blk_ptr": 8, "blk_col": 9, "blk_val": 10, "rb_scale": 11,
    "grp_ptr": 12, "grp_rb": 13, "grp_uptr": 14, "grp_ucol": 15, "blk_bsrc": 16,
}

STATUS = {
    0: "OK", -1: "ERR_ARG", -2: "ERR_CSR", -3: "ERR_DTYPE", -4: "ERR_NO_BACKWARD",
    -5: "ERR_HIP", -6: "ERR_OOM", -7: "ERR_OVERFLOW",
}


class PlanOpts(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("compute", ctypes.c_int32),
        ("split", ctypes.c_int32),
        ("block_rows", ctypes.c_int32),
        ("r_boundary", ctypes.c_int64),
        ("n_hint", ctypes.c_int32),
        ("want_backward", ctypes.c_int32),
        ("max_workspace_bytes", ctypes.c_uint64),
    ]


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("compute", ctypes.c_int32),
        ("m", ctypes.c_int64), ("k", ctypes.c_int64),
        ("nnz_input", ctypes.c_int64), ("nnz", ctypes.c_int64),
        ("block_rows", ctypes.c_int32),
        ("canonical_input", ctypes.c_int32),
        ("rows_csr", ctypes.c_int64),
        ("nnz_csr", ctypes.c_int64),
        ("long_rows", ctypes.c_int64),
        ("rb_bcsr", ctypes.c_int64),
        ("nblk", ctypes.c_int64),
        ("nblk_padded", ctypes.c_int64),
        ("nnz_bcsr", ctypes.c_int64),
        ("fill", ctypes.c_double),
        ("pred_us_csr", ctypes.c_double), ("pred_us_bcsr", ctypes.c_double),
        ("r_boundary", ctypes.c_int64),
        ("bytes_device", ctypes.c_int64),
        ("plan_ms", ctypes.c_double),
        ("has_backward", ctypes.c_int32),
        ("t_rows_csr", ctypes.c_int64), ("t_rb_bcsr", ctypes.c_int64), ("t_nblk", ctypes.c_int64),
        ("pred_us_csr_all", ctypes.c_double), ("pred_us_bcsr_all", ctypes.c_double),
        ("ngroups", ctypes.c_int64), ("grp_staged_tiles", ctypes.c_int64), ("grp_stage_rows", ctypes.c_int64),
        ("meas_us_csr_all", ctypes.c_double), ("meas_us_bcsr_all", ctypes.c_double),
    ]


CALIB_MAX = 32


class CalibInfo(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("T", ctypes.c_int32),
        ("x_max", ctypes.c_int32), ("y_max", ctypes.c_int32),
        ("n_candidates", ctypes.c_int32),
        ("cand_x", ctypes.c_int32 * CALIB_MAX),
        ("cand_y", ctypes.c_int32 * CALIB_MAX),
        ("cand_gflops", ctypes.c_double * CALIB_MAX),
        ("coef", ctypes.c_double * 5),
        ("best_x", ctypes.c_int32), ("best_y", ctypes.c_int32),
        ("best_gflops", ctypes.c_double),
        ("default_gflops", ctypes.c_double),
        ("applied", ctypes.c_int32),
    ]


EXPORTED = [
    "hybrid_spmm_plan", "hybrid_spmm_run", "hybrid_spmm_backward", "hybrid_spmm_update_values",
    "hybrid_spmm_plan_info", "hybrid_spmm_export", "hybrid_spmm_destroy",
    "hybrid_spmm_last_error", "hybrid_spmm_version", "hybrid_spmm_calibrate", "hybrid_spmm_run_noalloc",
    "hybrid_spmm_set_timing_events", "hybrid_spmm_backward_fused",
]

_lib = None


def load():
    """Load libhspmm.so and declare every entry point's signature."""
    global _lib
    if _lib is not None:
        return _lib
    if not LIB_PATH.exists():
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2511_08158_amd.build`")
    L = ctypes.CDLL(str(LIB_PATH))
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    L.hybrid_spmm_plan.argtypes = [ctypes.POINTER(vp), i64, i64, i64, vp, vp, vp, i32,
                                   ctypes.POINTER(PlanOpts), vp]
    L.hybrid_spmm_run.argtypes = [vp, i64, vp, i64, vp, i64, vp]
    L.hybrid_spmm_run_noalloc.argtypes = [vp, i64, vp, i64, vp, i64, vp]
    L.hybrid_spmm_backward.argtypes = [vp, i64, vp, i64, vp, i64, vp, i64, vp, vp]
    L.hybrid_spmm_update_values.argtypes = [vp, vp, i32, vp]
    L.hybrid_spmm_plan_info.argtypes = [vp, ctypes.POINTER(PlanInfo)]
    L.hybrid_spmm_export.argtypes = [vp, i32, i32, vp, i64, ctypes.POINTER(i64)]
    L.hybrid_spmm_calibrate.argtypes = [vp, i64, vp, i64, vp, i64, i32, ctypes.POINTER(CalibInfo), vp]
    L.hybrid_spmm_backward_fused.argtypes = [vp, i64, vp, i64, vp, i64, vp, i64, ctypes.POINTER(ctypes.c_int32)]
    L.hybrid_spmm_backward_fused.restype = ctypes.c_int
    L.hybrid_spmm_set_timing_events.argtypes = [vp, vp]
    L.hybrid_spmm_set_timing_events.restype = ctypes.c_int
    L.hybrid_spmm_destroy.argtypes = [vp]
    L.hybrid_spmm_destroy.restype = None
    for f in (L.hybrid_spmm_plan, L.hybrid_spmm_run, L.hybrid_spmm_run_noalloc, L.hybrid_spmm_backward,
              L.hybrid_spmm_update_values, L.hybrid_spmm_plan_info, L.hybrid_spmm_export,
              L.hybrid_spmm_calibrate):
        f.restype = ctypes.c_int
    L.hybrid_spmm_last_error.restype = ctypes.c_char_p
    L.hybrid_spmm_version.restype = ctypes.c_char_p
    _lib = L
    return L
