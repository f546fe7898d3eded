"""ctypes mirror of include/mipdhg.h and the loader of libmipdhg.so.

Argument marshalling only: every step of the solver runs in the HIP library.
The library must resolve to the HIP runtime that torch has already loaded, so
torch is imported before the library is opened.
"""
from __future__ import annotations

import ctypes as C
import os

import torch  # noqa: F401  (loads the HIP runtime the library must share)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmipdhg.so")

# status / error codes
OPTIMAL, ITER_LIMIT, TIME_LIMIT, NUMERICAL, PRIMAL_INFEASIBLE, DUAL_INFEASIBLE, IN_PROGRESS = 0, 1, 2, 3, 4, 5, 6
ERR_INVALID_ARG, ERR_BAD_CSR, ERR_TRANSPOSE, ERR_HIP = -1, -2, -3, -4
ERR_WORKSPACE, ERR_UNSUPPORTED, ERR_NONFINITE = -5, -6, -7

PRECISION = {"fp64": 0, "fp32": 1, "bf16": 2, "fp32acc32": 3, "fp32a": 4}

_i32, _i64, _f64, _p = C.c_int32, C.c_int64, C.c_double, C.c_void_p


class LPStruct(C.Structure):
    _fields_ = [("m", _i32), ("n", _i32), ("nnz", _i64),
                ("a_rowptr", _p), ("a_col", _p), ("a_val", _p),
                ("at_rowptr", _p), ("at_col", _p), ("at_val", _p),
                ("b", _p), ("c", _p), ("lo", _p), ("hi", _p), ("sense", _p)]


class OptionsStruct(C.Structure):
    _fields_ = [("precision", _i32), ("ruiz_iters", _i32), ("pock_chambolle", _i32),
                ("power_iters", _i32), ("eval_every", _i32),
                ("step_safety", _f64), ("reflect_rho", _f64),
                ("halpern", _i32), ("restarts", _i32),
                ("beta_suff", _f64), ("beta_nec", _f64), ("beta_art", _f64), ("pw_theta", _f64),
                ("max_iter", _i64), ("time_limit_s", _f64),
                ("validate", _i32), ("use_graph", _i32), ("spmv_kind", _i32), ("tile_nnz", _i32), ("tile_rows", _i32),
                ("short_row", _i32), ("lanes_a", _i32), ("lanes_at", _i32),
                ("long_row", _i32), ("kernel_timing", _i32), ("trace_iters", _i32),
                ("trace_x", _p), ("trace_y", _p), ("trace_xhat", _p), ("trace_yhat", _p),
                ("x_init", _p), ("y_init", _p), ("gather_order", _i32), ("resume", _i32),
                ("infeas_tol", _f64), ("pw_ki", _f64), ("pw_kd", _f64),
                ("tile_nnz_at", _i32), ("tile_rows_at", _i32), ("short_row_at", _i32), ("restart_avg", _i32),
                ("panel_width", _i32), ("step_rule", _i32), ("step0", _f64),
                ("batch_split", _i32), ("batch_block_iters", _i32)]


class InfoStruct(C.Structure):
    _fields_ = [("status", _i32), ("restarts", _i32), ("iters", _i64),
                ("rp_norm", _f64), ("rd_norm", _f64), ("gap", _f64), ("pobj", _f64), ("dobj", _f64),
                ("rel_rp", _f64), ("rel_rd", _f64), ("rel_gap", _f64), ("rp_inf", _f64),
                ("rd_inf", _f64), ("xz", _f64), ("max_violation", _f64), ("b_norm", _f64),
                ("c_norm", _f64), ("sigma_hat", _f64), ("eta", _f64), ("omega0", _f64),
                ("omega", _f64), ("ms_setup", _f64), ("ms_iter", _f64), ("ms_total", _f64),
                ("bytes_per_iter", _f64), ("bytes_primal", _f64), ("bytes_dual", _f64),
                ("ms_primal", _f64), ("ms_dual", _f64), ("n_primal", _i64), ("n_dual", _i64),
                ("lanes_a", _i32), ("lanes_at", _i32), ("long_a", _i32), ("long_at", _i32),
                ("ms_graph", _f64), ("rejected", _i64)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class IpmOptionsStruct(C.Structure):
    _fields_ = [("tol", _f64), ("max_iter", _i32), ("max_lifts", _i32), ("step_frac", _f64), ("min_step", _f64),
                ("mu_min", _f64), ("delta_max", _f64), ("alpha_min", _f64)]


class IpmInfoStruct(C.Structure):
    _fields_ = [("status", _i32), ("iters", _i32), ("lifts", _i32), ("pivots_replaced", _i32),
                ("alpha_min", _f64), ("mu_target", _f64), ("first_step_p", _f64), ("first_step_d", _f64),
                ("rel_rp", _f64), ("rel_rd", _f64), ("rel_gap", _f64), ("pobj", _f64), ("dobj", _f64),
                ("mu", _f64), ("ms_total", _f64)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class BatchStruct(C.Structure):
    _fields_ = [("count", _i32), ("row_off", _p), ("col_off", _p), ("nnz_off", _p), ("whole", LPStruct)]


# every symbol include/mipdhg.h declares, with its ctypes signature
SIGNATURES = {
    "mipdhg_default_options": (None, [C.POINTER(OptionsStruct)]),
    "mipdhg_workspace_size": (C.c_int, [C.POINTER(LPStruct), C.POINTER(OptionsStruct), C.POINTER(C.c_size_t)]),
    "mipdhg_solve": (C.c_int, [C.POINTER(LPStruct), C.POINTER(OptionsStruct), _f64, _p, C.c_size_t, _p,
                               _p, _p, _p, _p, _p, _p, _p, C.POINTER(InfoStruct)]),
    "mipdhg_batch_workspace_size": (C.c_int, [C.POINTER(BatchStruct), C.POINTER(OptionsStruct),
                                              C.POINTER(C.c_size_t)]),
    "mipdhg_solve_batched": (C.c_int, [C.POINTER(BatchStruct), C.POINTER(OptionsStruct), _p, _p, C.c_size_t,
                                       _p, _p, _p, _p, _p, _p, _p]),
    "mipdhg_autotune_batched": (C.c_int, [C.POINTER(BatchStruct), C.POINTER(OptionsStruct), _p, _p, C.c_size_t,
                                          _p, _p, _p, _p, _p, _p, C.POINTER(_f64)]),
    "mipdhg_unrolled_tape_size": (C.c_int, [C.POINTER(BatchStruct), C.POINTER(OptionsStruct), _i32, _i32,
                                            C.POINTER(C.c_size_t)]),
    "mipdhg_unrolled_forward": (C.c_int, [C.POINTER(BatchStruct), C.POINTER(OptionsStruct), _i32, _i32, _i32,
                                          _p, C.c_size_t, _p, _p]),
    "mipdhg_unrolled_backward": (C.c_int, [C.POINTER(BatchStruct), C.POINTER(OptionsStruct), _i32, _i32, _p,
                                           C.c_size_t, _p, _p, _p, _p]),
    "mipdhg_unrolled_schedule": (C.c_int, [C.POINTER(BatchStruct), C.POINTER(OptionsStruct), _i32, _i32, _p,
                                           C.c_size_t, _i32, _p, _i32, _p, _p, _p, C.POINTER(_i32)]),
    "mipdhg_center_workspace_size": (C.c_size_t, [_i32]),
    "mipdhg_center_start": (C.c_int, [_i32, _p, _p, _p, _f64, _f64, _f64, _p, C.c_size_t, _p, _p, _p,
                                      C.POINTER(_f64)]),
    "mipdhg_center_reclamp": (C.c_int, [_i32, _f64, _p, _p, _p]),
    "mipdhg_center_noalloc_max_n": (_i32, []),
    "mipdhg_read_probe": (C.c_int, [_p, C.c_size_t, _i32, _p, _p]),
    "mipdhg_ipm_default_options": (None, [C.POINTER(IpmOptionsStruct)]),
    "mipdhg_ipm_workspace_size": (C.c_int, [C.POINTER(LPStruct), C.POINTER(C.c_size_t)]),
    "mipdhg_ipm_solve": (C.c_int, [C.POINTER(LPStruct), _p, _p, _p, _p, _p, C.POINTER(IpmOptionsStruct), _p,
                                   C.c_size_t, _p, _p, _p, _p, C.POINTER(IpmInfoStruct)]),
    "mipdhg_ipm_warm": (C.c_int, [C.POINTER(LPStruct), _p, _p, _p, _p, _p, C.POINTER(IpmOptionsStruct), _p,
                                  C.c_size_t, _p, _p, _p, _p, C.POINTER(IpmInfoStruct)]),
    "mipdhg_center_start_noalloc": (C.c_int, [_i32, _p, _p, _p, _f64, _f64, _f64, _p, _p, _p, C.POINTER(_f64)]),
    "mipdhg_autotune": (C.c_int, [C.POINTER(LPStruct), C.POINTER(OptionsStruct), _i32, _p, C.c_size_t, _p,
                                  _p, _p, _p, _p, _p, C.POINTER(_f64)]),
    "mipdhg_autotune_cached": (C.c_int, [C.POINTER(LPStruct), C.POINTER(OptionsStruct), _i32, C.c_char_p, _p,
                                         C.c_size_t, _p, _p, _p, _p, _p, _p, C.POINTER(_f64), C.POINTER(_i32)]),
    "mipdhg_state_size": (C.c_int, [C.POINTER(LPStruct), C.POINTER(OptionsStruct), C.POINTER(C.c_size_t)]),
    "mipdhg_state_export": (C.c_int, [C.POINTER(LPStruct), C.POINTER(OptionsStruct), _p, C.c_size_t, _p, C.c_size_t,
                                      _p]),
    "mipdhg_state_import": (C.c_int, [C.POINTER(LPStruct), C.POINTER(OptionsStruct), _p, C.c_size_t, _p, C.c_size_t,
                                      _p]),
    "mipdhg_sizeof": (C.c_size_t, [C.c_int]),
    "mipdhg_status_string": (C.c_char_p, [C.c_int]),
    "mipdhg_last_error": (C.c_char_p, []),
}

_LIB = None


def _hip_runtimes() -> set:
    try:
        with open("/proc/self/maps") as f:
            return {l.split()[-1] for l in f if "libamdhip64" in l}
    except OSError:
        return set()


def load() -> C.CDLL:
    """Open libmipdhg.so (built by paper_2603_03150_amd.build).  Raises if it
    is missing: there is no fallback path."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run paper_2603_03150_amd.build.build() first")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    rts = _hip_runtimes()
    if len(rts) > 1:
        raise RuntimeError(f"two HIP runtimes are loaded ({sorted(rts)}); import torch first")
    for which, cls in ((0, LPStruct), (1, OptionsStruct), (2, InfoStruct), (3, BatchStruct)):
        if lib.mipdhg_sizeof(which) != C.sizeof(cls):
            raise RuntimeError(f"ABI mismatch for {cls.__name__}")
    _LIB = lib
    return lib


def check(rc: int) -> int:
    """Raise on a negative return code, return a status otherwise."""
    if rc < 0:
        lib = load()
        msg = lib.mipdhg_last_error().decode(errors="replace")
        name = lib.mipdhg_status_string(rc).decode()
        raise MipdhgError(rc, f"{name}: {msg}")
    return rc


class MipdhgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(msg)
        self.code = code
