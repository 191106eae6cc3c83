"""ctypes binding of libleapfrog.so (include/leapfrog.h): argument
marshalling only.  Every step of the path runs in the library's HIP kernels.
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libleapfrog.so")

LF_OK = 0
LF_INVALID_ARGUMENT = 1
LF_PLAN_INFEASIBLE = 2
LF_OUT_OF_WORKSPACE = 3
LF_HIP_ERROR = 4
LF_OVERFLOW = 5
LF_NOT_BOUND = 6
LF_INTERNAL = 7
STATUS_NAMES = {0: "OK", 1: "INVALID_ARGUMENT", 2: "PLAN_INFEASIBLE", 3: "OUT_OF_WORKSPACE",
                4: "HIP_ERROR", 5: "OVERFLOW", 6: "NOT_BOUND", 7: "INTERNAL"}

LF_C64 = 0
LF_CHALF = 1
LF_COST_FLOPMEM = 0
LF_COST_MLP = 1
LF_LAUNCH_STREAM = 0
LF_LAUNCH_GRAPH = 1
LF_OVERFLOW_RECALIBRATE = 0
LF_OVERFLOW_REPORT = 1
LF_MULT_AUTO = 0
LF_MULT_4M = 1
LF_MULT_3M = 2
LF_N_FEATURES = 14


class lf_gate(ctypes.Structure):
    _fields_ = [("n_q", ctypes.c_int32), ("q", ctypes.c_int32 * 2), ("layer", ctypes.c_int32),
                ("mat", ctypes.c_double * 32)]


class lf_circuit(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_int32), ("n_gates", ctypes.c_int32),
                ("gates", ctypes.POINTER(lf_gate))]


class lf_plan_opts(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("max_log2_intermediate", ctypes.c_int32),
                ("n_sliced_wires", ctypes.c_int32), ("sliced_wires", ctypes.POINTER(ctypes.c_int32)),
                ("n_forced", ctypes.c_int32), ("cost_model", ctypes.c_int32),
                ("greedy_trials", ctypes.c_int32), ("partition_trials", ctypes.c_int32),
                ("sa_iters", ctypes.c_int64),
                ("seed", ctypes.c_uint64), ("chalf_min_log2", ctypes.c_int32),
                ("launch_mode", ctypes.c_int32), ("check_overflow", ctypes.c_int32),
                ("slices_per_graph", ctypes.c_int32), ("search_dtype", ctypes.c_int32),
                ("autotune", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("chalf_headroom_bits", ctypes.c_int32), ("overflow_policy", ctypes.c_int32),
                ("chalf_exec_min_log2", ctypes.c_int32), ("mult", ctypes.c_int32),
                ("autotune_cache", ctypes.c_char_p), ("keep_batch_order", ctypes.c_int32),
                ("group_small_steps", ctypes.c_int32)]


class lf_overflow_info(ctypes.Structure):
    _fields_ = [("saturated", ctypes.c_uint32), ("recalibrations", ctypes.c_int32),
                ("first_bad_slice", ctypes.c_int64), ("headroom_bits", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class lf_batch_item(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("slice_begin", ctypes.c_int64),
                ("slice_end", ctypes.c_int64), ("out_amps", ctypes.c_void_p)]


LF_BATCH_SEQUENTIAL = 0
LF_BATCH_GRAPH = 1


class lf_plan_info(ctypes.Structure):
    _fields_ = [("n_slices", ctypes.c_int64), ("n_sliced_wires", ctypes.c_int32),
                ("n_steps", ctypes.c_int32), ("n_variant_steps", ctypes.c_int32),
                ("n_leaves", ctypes.c_int32), ("max_log2_intermediate", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("n_open", ctypes.c_int32), ("n_batch", ctypes.c_int64),
                ("n_batch_log2", ctypes.c_int32), ("n_half_steps", ctypes.c_int32),
                ("macs_per_slice", ctypes.c_double), ("macs_invariant", ctypes.c_double),
                ("bytes_per_slice", ctypes.c_double), ("bytes_invariant", ctypes.c_double),
                ("log2_total_macs", ctypes.c_double), ("workspace_bytes", ctypes.c_uint64),
                ("leaf_id_base", ctypes.c_int32), ("n_step_groups", ctypes.c_int32),
                ("n_grouped_steps", ctypes.c_int32)]


# name -> (restype, argtypes)
_P = ctypes.c_void_p
SIGNATURES = {
    "lf_plan_opts_default": (None, [ctypes.POINTER(lf_plan_opts)]),
    "lf_build_network": (ctypes.c_int32, [ctypes.POINTER(lf_circuit), ctypes.POINTER(ctypes.c_int32),
                                          ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64),
                                          ctypes.c_int64, ctypes.POINTER(lf_plan_opts),
                                          ctypes.POINTER(_P)]),
    "lf_plan_get_info": (ctypes.c_int32, [_P, ctypes.POINTER(lf_plan_info)]),
    "lf_plan_sliced_wires": (ctypes.c_int32, [_P, ctypes.POINTER(ctypes.c_int32)]),
    "lf_plan_tree": (ctypes.c_int32, [_P, ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "lf_plan_steps": (ctypes.c_int32, [_P, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "lf_plan_step_strides": (ctypes.c_int32, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]),
    "lf_plan_step_gather": (ctypes.c_int32, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                             ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64),
                                             ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)]),
    "lf_plan_bind_workspace": (ctypes.c_int32, [_P, _P, ctypes.c_uint64, _P]),
    "lf_contract_slices": (ctypes.c_int32, [_P, ctypes.c_int64, ctypes.c_int64, _P, _P]),
    "lf_plan_overflow": (ctypes.c_int32, [_P, _P, ctypes.POINTER(lf_overflow_info), ctypes.c_int32]),
    "lf_plan_recalibrate": (ctypes.c_int32, [_P, ctypes.c_int64, ctypes.c_int32, _P]),
    "lf_debug_scale_slice_leaf": (ctypes.c_int32, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P]),
    "lf_contract_batch": (ctypes.c_int32, [ctypes.POINTER(lf_batch_item), ctypes.c_int32, ctypes.c_int32,
                                           ctypes.c_int32, _P]),
    "lf_postselect_topk": (ctypes.c_int32, [_P, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, _P, _P, _P]),
    "lf_probabilities_at": (ctypes.c_int32, [_P, ctypes.c_int64, _P, ctypes.c_int64, _P, _P]),
    "lf_mcmc_sample": (ctypes.c_int32, [_P, ctypes.c_int64, _P, ctypes.c_int64, ctypes.c_int64,
                                        ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                        ctypes.c_int64, ctypes.c_uint64, _P, _P, _P]),
    "lf_postselect_topk_noalloc": (ctypes.c_int32, [_P, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                                    _P, _P, _P]),
    "lf_profile_steps": (ctypes.c_int32, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double), _P]),
    "lf_plan_time_kernel": (ctypes.c_int32, [_P, ctypes.c_int32, ctypes.c_int64]),
    "lf_plan_kernel_times": (ctypes.c_int32, [_P, ctypes.POINTER(ctypes.c_double),
                                              ctypes.POINTER(ctypes.c_int64),
                                              ctypes.POINTER(ctypes.c_double),
                                              ctypes.POINTER(ctypes.c_int64)]),
    "lf_contract_pair": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                          _P, _P, _P,
                                          ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                                          ctypes.c_float, _P]),
    "lf_step_features": (ctypes.c_int32, [ctypes.c_int32] * 5 + [ctypes.POINTER(ctypes.c_float)]),
    "lf_mlp_sizes": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                      ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_uint64)]),
    "lf_mlp_forward": (ctypes.c_int32, [_P, ctypes.c_int32, ctypes.c_int32, _P, ctypes.c_int64, _P, _P,
                                        ctypes.c_uint64, _P]),
    "lf_mlp_gradients": (ctypes.c_int32, [_P, ctypes.c_int32, ctypes.c_int32, _P, _P, ctypes.c_int64, _P,
                                          _P, _P, ctypes.c_uint64, _P]),
    "lf_mlp_adam_step": (ctypes.c_int32, [_P, _P, _P, _P, ctypes.c_int64, ctypes.c_int32, ctypes.c_float,
                                          ctypes.c_float, ctypes.c_float, ctypes.c_float, _P]),
    "lf_costmodel_train": (ctypes.c_int32, [_P, _P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.c_int32, ctypes.c_int32, ctypes.c_float, ctypes.c_uint64,
                                            _P, _P, _P, _P, _P, _P, _P]),
    "lf_costmodel_load": (ctypes.c_int32, [ctypes.POINTER(ctypes.c_float), ctypes.c_int32, ctypes.c_int32,
                                           ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float),
                                           ctypes.c_float, ctypes.c_float]),
    "lf_costmodel_clear": (ctypes.c_int32, []),
    "lf_costmodel_predict": (ctypes.c_int32, [ctypes.c_int32] * 5 + [ctypes.POINTER(ctypes.c_double)]),
    "lf_autotune_save": (ctypes.c_int32, [ctypes.c_char_p]),
    "lf_autotune_load": (ctypes.c_int32, [ctypes.c_char_p]),
    "lf_plan_destroy": (None, [_P]),
    "lf_last_error": (ctypes.c_char_p, []),
}

_lib = None


def load():
    """Loads the in-tree library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2406_18889_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class LeapfrogError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = load().lf_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(status: int, where: str) -> None:
    if status != LF_OK:
        raise LeapfrogError(status, where)
