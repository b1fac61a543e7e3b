"""ctypes declarations of include/ldopf.h (argument marshalling only).

Loading fails loudly when the compiled library is absent: there is no CPU
fallback for any call.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# LDOPF_LIBRARY selects another build of the same library (the host
# sanitizer build of build.build_sanitized); default: the in-tree build.
LIB_PATH = os.environ.get("LDOPF_LIBRARY") or os.path.join(HERE, "libldopf.so")

LDOPF_OK = 0
LDOPF_NOT_CONVERGED = 1
LDOPF_INVALID_ARGUMENT = -1
LDOPF_INVALID_NETWORK = -2
LDOPF_INFEASIBLE_BOUNDS = -3
LDOPF_INCONSISTENT_SUBSYSTEM = -4
LDOPF_OUT_OF_MEMORY = -5
LDOPF_DEVICE_ERROR = -6
LDOPF_NUMERICAL = -7
LDOPF_BUFFER_TOO_SMALL = -8
LDOPF_UNSUPPORTED = -9

LDOPF_FP64 = 0
LDOPF_FP32_MIXED = 1
LDOPF_RESIDUAL_PAPER = 0
LDOPF_RESIDUAL_AGGREGATED = 1
LDOPF_RHO_FIXED = 0
LDOPF_RHO_BALANCE = 1
LDOPF_PATH_AUTO = 0
LDOPF_PATH_PERSISTENT = 1
LDOPF_PATH_STREAMED = 2

_d = C.POINTER(C.c_double)
_i32 = C.POINTER(C.c_int32)
_i64 = C.POINTER(C.c_int64)
_u8 = C.POINTER(C.c_uint8)


class ldopf_network(C.Structure):
    _fields_ = [
        ("n_bus", C.c_int32), ("n_line", C.c_int32), ("n_load", C.c_int32), ("n_gen", C.c_int32),
        ("root", C.c_int32),
        ("bus_phases", _u8), ("bus_wlo", _d), ("bus_whi", _d), ("bus_gsh", _d), ("bus_bsh", _d),
        ("line_from", _i32), ("line_to", _i32), ("line_phases", _u8), ("line_r", _d), ("line_x", _d),
        ("line_gs_from", _d), ("line_bs_from", _d), ("line_gs_to", _d), ("line_bs_to", _d),
        ("line_tau", _d), ("line_plo", _d), ("line_phi", _d), ("line_qlo", _d), ("line_qhi", _d),
        ("load_bus", _i32), ("load_phases", _u8), ("load_conn", _u8), ("load_a", _d), ("load_b", _d),
        ("load_alpha", _d), ("load_beta", _d),
        ("gen_bus", _i32), ("gen_phases", _u8), ("gen_plo", _d), ("gen_phi", _d), ("gen_qlo", _d),
        ("gen_qhi", _d), ("gen_cost_p", _d), ("gen_cost_q", _d),
    ]


class ldopf_options(C.Structure):
    _fields_ = [
        ("rho", C.c_double), ("eps_rel", C.c_double), ("eps_abs", C.c_double), ("max_iter", C.c_int64),
        ("precision", C.c_int32), ("residual_form", C.c_int32), ("check_termination", C.c_int32),
        ("history", C.c_int32), ("rows_per_part", C.c_int32), ("block_threads", C.c_int32),
        ("profile", C.c_int32), ("rho_update", C.c_int32), ("rho_period", C.c_int32),
        ("rho_max_changes", C.c_int32), ("sweep_path", C.c_int32), ("reserved", C.c_int32), ("rho_mu", C.c_double),
        ("rho_tau", C.c_double),
    ]


class ldopf_sizes(C.Structure):
    _fields_ = [
        ("n", C.c_int64), ("n_sub", C.c_int64), ("n_local", C.c_int64), ("sum_m", C.c_int64),
        ("op_words", C.c_int64), ("rank_words", C.c_int64), ("max_n", C.c_int32), ("max_m", C.c_int32),
        ("n_parts", C.c_int32), ("block_threads", C.c_int32), ("lds_bytes", C.c_int64),
        ("sync_bytes", C.c_int64), ("sweep_path", C.c_int32), ("reserved", C.c_int32),
    ]


class ldopf_status(C.Structure):
    _fields_ = [
        ("iterations", C.c_int64), ("converged", C.c_int32), ("code", C.c_int32),
        ("pres", C.c_double), ("dres", C.c_double), ("eps_prim", C.c_double), ("eps_dual", C.c_double),
        ("sweep_ms", C.c_double), ("precompute_ms", C.c_double), ("sweeps_computed", C.c_int64),
        ("rho", C.c_double), ("rho_changes", C.c_int64),
    ]


class ldopf_batch_status(C.Structure):
    _fields_ = [
        ("sweeps", C.c_int64), ("n_scen", C.c_int32), ("n_converged", C.c_int32), ("n_numerical", C.c_int32),
        ("code", C.c_int32), ("solve_ms", C.c_double), ("precompute_ms", C.c_double),
    ]


class ldopf_batch_sizes(C.Structure):
    _fields_ = [
        ("n", C.c_int64), ("n_sub", C.c_int64), ("n_local", C.c_int64), ("n_scen", C.c_int32),
        ("n_scen_padded", C.c_int32), ("n_mfma_subsystems", C.c_int64), ("n_vector_subsystems", C.c_int64),
        ("scenario_operator_words", C.c_int64), ("shared_operator_words", C.c_int64),
        ("rows_per_chunk", C.c_int32), ("blocks_per_tile", C.c_int32), ("graph_sweeps", C.c_int32),
        ("pad", C.c_int32),
    ]


class ldopf_server_stats(C.Structure):
    _fields_ = [
        ("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64), ("queued", C.c_int64),
        ("running", C.c_int64), ("peak_running", C.c_int64), ("bytes_in_use", C.c_int64),
        ("peak_bytes_in_use", C.c_int64), ("budget_bytes", C.c_int64), ("p50_ms", C.c_double),
        ("p99_ms", C.c_double), ("mean_ms", C.c_double), ("max_ms", C.c_double), ("wall_s", C.c_double),
        ("solves_per_s", C.c_double),
    ]


LDOPF_REQ_QUEUED, LDOPF_REQ_RUNNING, LDOPF_REQ_DONE, LDOPF_REQ_FAILED = 0, 1, 2, 3


# Every exported call: name -> (restype, argtypes)
SIGNATURES = {
    "ldopf_error_string": (C.c_char_p, [C.c_int]),
    "ldopf_last_error_detail": (C.c_char_p, []),
    "ldopf_default_options": (None, [C.POINTER(ldopf_options)]),
    "ldopf_describe_network": (C.c_int, [C.POINTER(ldopf_network), _i64, _d, _d, _d, _d, _i32, _i32, _d, _d, _i64]),
    "ldopf_create": (C.c_int, [C.POINTER(ldopf_network), C.POINTER(ldopf_options), C.c_void_p, C.POINTER(C.c_void_p)]),
    "ldopf_create_lp": (C.c_int, [C.c_int64, _d, _d, _d, _d, C.c_int64, _i32, _i32, _d, _d, _i64,
                                  C.POINTER(ldopf_options), C.c_void_p, C.POINTER(C.c_void_p)]),
    "ldopf_destroy": (C.c_int, [C.c_void_p]),
    "ldopf_get_sizes": (C.c_int, [C.c_void_p, C.POINTER(ldopf_sizes)]),
    "ldopf_set_options": (C.c_int, [C.c_void_p, C.POINTER(ldopf_options)]),
    "ldopf_solve": (C.c_int, [C.c_void_p, C.POINTER(ldopf_status)]),
    "ldopf_solve_noalloc": (C.c_int, [C.c_void_p, C.POINTER(ldopf_status)]),
    "ldopf_solve_many": (C.c_int, [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(ldopf_status)]),
    "ldopf_reset": (C.c_int, [C.c_void_p]),
    "ldopf_warm_start": (C.c_int, [C.c_void_p, _d, _d, C.c_int64]),
    "ldopf_get_global": (C.c_int, [C.c_void_p, _d, C.c_int64]),
    "ldopf_get_local": (C.c_int, [C.c_void_p, _d, _d, C.c_int64]),
    "ldopf_get_structure": (C.c_int, [C.c_void_p, _i64, C.c_int64, _i64, C.c_int64]),
    "ldopf_get_history": (C.c_int, [C.c_void_p, _d, C.c_int64, _i64]),
    "ldopf_get_operators": (C.c_int, [C.c_void_p, _d, C.c_int64, _d, C.c_int64, _i32, C.c_int64]),
    "ldopf_get_rho_log": (C.c_int, [C.c_void_p, _i64, _d, C.c_int64, _i64]),
    "ldopf_get_phase_times": (C.c_int, [C.c_void_p, _d]),
    "ldopf_get_phase_times_part": (C.c_int, [C.c_void_p, C.c_int32, _d]),
    "ldopf_objective": (C.c_int, [C.c_void_p, _d]),
    "ldopf_get_global_device": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64]),
    "ldopf_get_local_device": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64]),
    "ldopf_batch_create": (C.c_int, [C.POINTER(ldopf_network), C.c_int32, _d, C.POINTER(ldopf_options), C.c_void_p,
                                     C.POINTER(C.c_void_p)]),
    "ldopf_batch_destroy": (C.c_int, [C.c_void_p]),
    "ldopf_batch_set_options": (C.c_int, [C.c_void_p, C.POINTER(ldopf_options)]),
    "ldopf_batch_reset": (C.c_int, [C.c_void_p]),
    "ldopf_batch_solve": (C.c_int, [C.c_void_p, C.POINTER(ldopf_batch_status)]),
    "ldopf_batch_get_scenario": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(ldopf_status)]),
    "ldopf_batch_get_global": (C.c_int, [C.c_void_p, C.c_int32, _d, C.c_int64]),
    "ldopf_batch_get_local": (C.c_int, [C.c_void_p, C.c_int32, _d, _d, C.c_int64]),
    "ldopf_batch_get_sizes": (C.c_int, [C.c_void_p, C.POINTER(ldopf_batch_sizes)]),
    "ldopf_batch_tune": (C.c_int, [C.c_void_p, C.c_char_p, _i32, _i32]),
    "ldopf_request_estimate": (C.c_int, [C.POINTER(ldopf_network), C.POINTER(ldopf_options), _i64, _i32]),
    "ldopf_server_create": (C.c_int, [C.c_int64, C.c_int32, C.POINTER(C.c_void_p)]),
    "ldopf_server_submit": (C.c_int, [C.c_void_p, C.POINTER(ldopf_network), C.POINTER(ldopf_options), _i64]),
    "ldopf_server_poll": (C.c_int, [C.c_void_p, C.c_int64, _i32, C.POINTER(ldopf_status)]),
    "ldopf_server_wait": (C.c_int, [C.c_void_p, C.c_int64, C.c_double, _i32, C.POINTER(ldopf_status)]),
    "ldopf_server_cancel": (C.c_int, [C.c_void_p, C.c_int64]),
    "ldopf_server_fetch": (C.c_int, [C.c_void_p, C.c_int64, _d, C.c_int64, _d, _d, C.c_int64, _i64]),
    "ldopf_server_release": (C.c_int, [C.c_void_p, C.c_int64]),
    "ldopf_server_get_stats": (C.c_int, [C.c_void_p, C.POINTER(ldopf_server_stats)]),
    "ldopf_server_destroy": (C.c_int, [C.c_void_p]),
}

_lib = None


def lib():
    """The loaded libldopf; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2310_09410_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib
