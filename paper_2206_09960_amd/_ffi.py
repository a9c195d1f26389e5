"""ctypes declarations of the C ABI in include/psi.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpsi.so")

# status codes
PSI_OK, PSI_EINVAL, PSI_ENOTCONV, PSI_ESTAGNATED, PSI_ENUMERIC, PSI_EDEVICE, PSI_ENOSPACE = range(7)
STATUS_NAMES = {0: "PSI_OK", 1: "PSI_EINVAL", 2: "PSI_ENOTCONV", 3: "PSI_ESTAGNATED",
                4: "PSI_ENUMERIC", 5: "PSI_EDEVICE", 6: "PSI_ENOSPACE"}
# build flags
PSI_INPUT_HOST = 0x1
PSI_STRICT = 0x2
PSI_WEIGHTED_FP64 = 0x4
# tolerance modes
PSI_TOL_ABS_L1, PSI_TOL_BNORM, PSI_TOL_REL_L1 = 0, 1, 2
# precisions
PSI_PREC_FP64, PSI_PREC_FP64_WEIGHTED, PSI_PREC_MIXED, PSI_PREC_FP32 = 0, 1, 2, 3
# solve flags
PSI_NO_FALLBACK = 0x1
# partial pass of a column-segmented pass
PSI_SEG_TILES, PSI_SEG_SLICES, PSI_SEG_BANDS, PSI_SEG_BINS = 1, 2, 3, 4
# pass kinds
PSI_PASS_STEP64, PSI_PASS_STEP64_W, PSI_PASS_FINAL64, PSI_PASS_STEP32 = 0, 1, 2, 3
PSI_PASS_PART64, PSI_PASS_PART32 = 4, 5

i32, i64, u32, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_double
vp, sz = ctypes.c_void_p, ctypes.c_size_t


class OperatorStats(ctypes.Structure):
    _fields_ = [("n_users", i64), ("n_edges_in", i64), ("n_edges", i64), ("n_self_loops", i64),
                ("n_duplicates", i64), ("n_no_leaders", i64), ("max_followers", i64),
                ("n_graphs", i32), ("flags", i32), ("b_norm", f64), ("kappa", f64)]


class Params(ctypes.Structure):
    _fields_ = [("tol", f64), ("tol_mode", i32), ("max_iter", i32), ("precision", i32),
                ("check_every", i32), ("flags", u32), ("tile_items", i32), ("col_segments", i32),
                ("seg_form", i32),
                ("inner_tol", f64), ("band_col_log", i32), ("band_rows", i32),
                ("batch_tile", i32), ("batch_items", i32), ("hub_chunk", i32)]


class Info(ctypes.Structure):
    _fields_ = [("status", i32), ("iterations", i32), ("spmv_passes", i32), ("fp32_passes", i32),
                ("refinements", i32), ("used_s0", i32), ("col_segments", i32),
                ("tile_items", i32), ("final_gap", f64),
                ("final_l1_step", f64), ("b_norm", f64), ("kappa", f64), ("err_bound_s", f64),
                ("psi_gap_bound", f64), ("device_ms", f64), ("seg_form", i32),
                ("batch_tile", i32), ("hub_chunk", i32)]


def struct_dict(s: ctypes.Structure) -> dict:
    return {name: getattr(s, name) for name, _ in s._fields_}


# (name, restype, argtypes) of every exported entry point
SIGNATURES = [
    ("psi_version", ctypes.c_char_p, []),
    ("psi_last_error", ctypes.c_char_p, []),
    ("psi_operator_workspace_size", i32, [i64, i64, i32, u32, ctypes.POINTER(sz), ctypes.POINTER(sz)]),
    ("psi_build_operator", i32, [i64, i64, vp, vp, vp, vp, i32, vp, u32, vp, sz, vp, sz, vp,
                                 ctypes.POINTER(vp)]),
    ("psi_operator_destroy", i32, [vp]),
    ("psi_operator_get_stats", i32, [vp, ctypes.POINTER(OperatorStats)]),
    ("psi_operator_views", i32, [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                 ctypes.POINTER(vp), ctypes.POINTER(vp)]),
    ("psi_params_default", i32, [ctypes.POINTER(Params)]),
    ("psi_solve", i32, [vp, ctypes.POINTER(Params), vp, vp, vp, ctypes.POINTER(Info), vp]),
    ("psi_solve_async", i32, [vp, ctypes.POINTER(Params), vp, vp, vp, ctypes.POINTER(Info), vp]),
    ("psi_pagerank", i32, [vp, f64, ctypes.POINTER(Params), i32, vp, vp, ctypes.POINTER(Info),
                           vp]),
    ("psi_step", i32, [vp, i32, vp, vp, vp, i32, i32, i32, vp]),
    ("psi_final", i32, [vp, vp, vp, vp]),
    ("psi_debug_force_slot_timeout", i32, [vp, i32]),
    ("psi_operator_band_info", i32, [vp] + [ctypes.POINTER(i32)] * 6),
    ("psi_operator_bins_info", i32, [vp] + [ctypes.POINTER(i32)] * 5 + [ctypes.POINTER(i64)]),
    ("psi_pass_time", i32, [vp, i32, i32, i32, i32, i32, ctypes.POINTER(f64), vp]),
    ("psi_autotune_batched", i32, [vp, i32, i32, vp, sz, i32, ctypes.POINTER(i32),
                                   ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(f64),
                                   vp]),
    ("psi_autotune_graphs", i32, [vp, i32, f64, i32, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                  ctypes.POINTER(i32), ctypes.POINTER(f64), vp]),
    ("psi_batched_workspace_size", i32, [vp, i32, i32, ctypes.POINTER(sz)]),
    ("psi_solve_batched", i32, [vp, ctypes.POINTER(Params), i32, vp, vp, vp, ctypes.POINTER(Info),
                                vp, sz, vp]),
    ("psi_gather_probe", i32, [vp, i64, i32, vp, i64, vp, i32, i32, ctypes.POINTER(f64), vp]),
    ("psi_anderson_workspace_size", i32, [vp, i32, ctypes.POINTER(sz)]),
    ("psi_solve_anderson_noalloc", i32, [vp, ctypes.POINTER(Params), i32, vp, vp, vp,
                                     ctypes.POINTER(Info), vp]),
    ("psi_solve_anderson", i32, [vp, ctypes.POINTER(Params), i32, vp, vp, vp,
                                 ctypes.POINTER(Info), vp, sz, vp]),
    ("psi_solve_origins", i32, [vp, ctypes.POINTER(Params), i32, vp, vp, vp,
                                ctypes.POINTER(Info), vp, sz, vp]),
    ("psi_autotune", i32, [vp, i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i32),
                           ctypes.POINTER(i32), ctypes.POINTER(f64), vp]),
    ("psi_mpnn_param_count", i64, []),
    ("psi_model_state_size", i32, [ctypes.POINTER(sz)]),
    ("psi_model_create", i32, [vp, i64, u32, vp, sz, vp, ctypes.POINTER(vp)]),
    ("psi_model_destroy", i32, [vp]),
    ("psi_model_params", i32, [vp, vp, u32, vp]),
    ("psi_model_grad", i32, [vp, vp, u32, vp]),
    ("psi_mpnn_workspace_size", i32, [vp, i32, ctypes.POINTER(sz)]),
    ("psi_mpnn_forward", i32, [vp, vp, vp, vp, vp, sz, vp]),
    ("psi_warmstart", i32, [vp, vp, vp, vp, sz, vp]),
    ("psi_mpnn_loss_backward", i32, [vp, vp, vp, ctypes.POINTER(f64), vp, vp, sz, vp]),
    ("psi_mpnn_adam_step", i32, [vp, f64, f64, f64, f64, vp]),
]

_lib = None


def load(path: str | None = None) -> ctypes.CDLL:
    """Load libpsi.so.  Raises if it has not been built: there is no fallback."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"HIP library {p} is missing: run `python -m paper_2206_09960_amd.build`")
    lib = ctypes.CDLL(p)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = lib
    return lib
