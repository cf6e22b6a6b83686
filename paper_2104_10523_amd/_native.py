"""ctypes declarations of the C ABI in include/tn.h (marshalling only)."""

from __future__ import annotations

import ctypes as C
import os
from pathlib import Path

LIB_PATH = Path(__file__).resolve().parent / "libtn.so"

TN_OK = 0
ERRORS = {
    -1: "TN_ERR_ARG", -2: "TN_ERR_MODES", -3: "TN_ERR_EXTENT", -4: "TN_ERR_BITS",
    -5: "TN_ERR_BUDGET", -6: "TN_ERR_WORKSPACE", -7: "TN_ERR_DEVICE", -8: "TN_ERR_GATE",
    -9: "TN_ERR_SITE", -10: "TN_ERR_UNSUPPORTED", -11: "TN_ERR_NOMEM", -12: "TN_ERR_STATE",
}

GATE_IDS = {
    "sqrt_x": 1, "sqrt_y": 2, "sqrt_w": 3, "h": 4, "x": 5, "y": 6, "z": 7, "s": 8, "t": 9,
    "rz": 10, "cz": 20, "cx": 21, "fsim": 22, "cphase": 23, "swap": 24,
    "custom1": 40, "custom2": 41, "depol1": 60, "depol2": 61, "amp_damp": 62,
}

PREC = {"fp32": 0, "bf16x3": 1, "bf16x6": 2, "auto": 3, "f16x3": 4, "fp64": 5}
PATH_ALGO = {"greedy": 0, "random_greedy": 1, "learned": 2, "partition": 3}
PAULI = {"I": 0, "X": 1, "Y": 2, "Z": 3}


class TnOp(C.Structure):
    _fields_ = [("gate", C.c_int32), ("q0", C.c_int32), ("q1", C.c_int32),
                ("param", C.c_double * 2), ("matrix", C.POINTER(C.c_double))]


class TnCircuit(C.Structure):
    _fields_ = [("n_qubits", C.c_int32), ("n_ops", C.c_int64), ("ops", C.POINTER(TnOp))]


class TnNetworkInfo(C.Structure):
    _fields_ = [("n_qubits", C.c_int32), ("n_tensors", C.c_int32), ("n_labels", C.c_int32)]


class TnPathOpts(C.Structure):
    _fields_ = [("algo", C.c_int32), ("trials", C.c_int32), ("seed", C.c_uint64),
                ("temperature", C.c_double), ("mem_budget_bytes", C.c_double),
                ("open_mask", C.POINTER(C.c_int8)), ("model", C.c_void_p),
                ("rank", C.c_int32), ("rank_precision", C.c_int32),
                ("rescore_every", C.c_int32)]


class TnPathCost(C.Structure):
    _fields_ = [("flops_per_slice", C.c_double), ("total_flops", C.c_double),
                ("peak_elems", C.c_double), ("n_slices", C.c_double), ("n_steps", C.c_int32),
                ("n_sliced", C.c_int32), ("algo_used", C.c_int32), ("reserved", C.c_int32)]


class TnTensor(C.Structure):
    _fields_ = [("data", C.c_void_p), ("rank", C.c_int32), ("dtype", C.c_int32),
                ("extents", C.POINTER(C.c_int64))]


class TnReport(C.Structure):
    _fields_ = [("seconds", C.c_double), ("flops", C.c_double), ("bytes", C.c_double),
                ("slices_run", C.c_double), ("kernels", C.c_double), ("precision", C.c_int32),
                ("nonfinite", C.c_int32), ("err_bound", C.c_double)]


class TnExecOpts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("use_graph", C.c_int32), ("slice_begin", C.c_int64),
                ("slice_count", C.c_int64), ("accumulate", C.c_int32), ("sync", C.c_int32),
                ("op_seconds", C.POINTER(C.c_double))]


class TnPlanInfo(C.Structure):
    _fields_ = [("n_ops", C.c_int32), ("n_by_kind", C.c_int32 * 4),
                ("flops_by_kind", C.c_double * 4), ("bytes_by_kind", C.c_double * 4),
                ("workspace_bytes", C.c_double), ("err_bound", C.c_double)]


P = C.c_void_p
PP = C.POINTER(C.c_void_p)
I32, I64, U64, D = C.c_int32, C.c_int64, C.c_uint64, C.c_double
PI8, PI32, PD = C.POINTER(C.c_int8), C.POINTER(C.c_int32), C.POINTER(C.c_double)

# name -> (restype, argtypes); every entry point declared in include/tn.h
SIGNATURES = {
    "tn_last_error": (C.c_char_p, []),
    "tn_version": (C.c_char_p, []),
    "tn_build_network": (I32, [C.POINTER(TnCircuit), PP]),
    "tn_network_destroy": (I32, [P]),
    "tn_network_get_info": (I32, [P, C.POINTER(TnNetworkInfo)]),
    "tn_network_get_tensor": (I32, [P, I32, PI32, PI32, PD]),
    "tn_network_output_labels": (I32, [P, PI32]),
    "tn_find_path": (I32, [P, C.POINTER(TnPathOpts), PP, C.POINTER(TnPathCost)]),
    "tn_path_from_pairs": (I32, [P, C.POINTER(TnPathOpts), PI32, I32, PP, C.POINTER(TnPathCost)]),
    "tn_path_get": (I32, [P, PI32, PI32]),
    "tn_path_destroy": (I32, [P]),
    "tn_set_workspace": (I32, [P, C.c_size_t]),
    "tn_contract_pair": (I32, [C.POINTER(TnTensor), PI32, C.POINTER(TnTensor), PI32,
                               C.POINTER(TnTensor), PI32, I32, P]),
    "tn_contract_pair_noalloc": (I32, [C.POINTER(TnTensor), PI32, C.POINTER(TnTensor), PI32,
                                       C.POINTER(TnTensor), PI32, I32, P]),
    "tn_amplitudes": (I32, [P, P, PI8, I64, C.POINTER(TnExecOpts), P, C.POINTER(TnReport), P]),
    "tn_amplitudes_workspace": (I32, [P, P, I64, I32, C.POINTER(C.c_size_t)]),
    "tn_amplitudes_plan_info": (I32, [P, P, I32, C.POINTER(TnPlanInfo)]),
    "tn_amplitudes_autotune": (I32, [P, P, I32, I32, P]),
    "tn_amplitudes_plan_ops": (I32, [P, P, I32, PI32, PD, PD, C.POINTER(C.c_int64)]),  # shape: 8 per op
    "tn_build_expectation_network": (I32, [C.POINTER(TnCircuit), PI8, PP, C.POINTER(C.c_int64)]),
    "tn_build_density_network": (I32, [C.POINTER(TnCircuit), PI8, PP, C.POINTER(C.c_int64)]),
    "tn_pauli_expectation": (I32, [P, PI8, I64, I32, PI8, PD, P]),
    "tn_sample_amplitudes": (I32, [P, I64, PD, I64, C.POINTER(C.c_int64), PD, P]),
    "tn_mps_create": (I32, [I32, I32, P, PP]),
    "tn_mps_destroy": (I32, [P]),
    "tn_mps_apply_gate1": (I32, [P, I32, PD, P]),
    "tn_mps_apply_gate": (I32, [P, I32, PD, I32, D, PD, P]),
    "tn_pmps_create": (I32, [I32, I32, I32, P, C.POINTER(C.c_void_p)]),
    "tn_pmps_destroy": (I32, [P]),
    "tn_pmps_apply_gate1": (I32, [P, I32, PD, P]),
    "tn_pmps_apply_gate": (I32, [P, I32, PD, C.c_double, PD, P]),
    "tn_pmps_apply_channel": (I32, [P, I32, I32, PD, I32, C.c_double, PD, PD, P]),
    "tn_pmps_dims": (I32, [P, PI32, PI32]),
    "tn_pmps_expect_z": (I32, [P, PD, P]),
    "tn_pmps_get_site": (I32, [P, I32, PD, PI32, P]),
    "tn_mps_bond_dims": (I32, [P, PI32]),
    "tn_mps_bond_spectrum": (I32, [P, I32, PD, I32, PI32]),
    "tn_mps_expect_z": (I32, [P, PD, P]),
    "tn_mps_amplitudes": (I32, [P, PI8, I64, PD, P]),
    "tn_run_trajectories": (I32, [C.POINTER(C.POINTER(TnCircuit)), I32, I32, PD, I64, PD,
                                  C.POINTER(TnReport), P]),
    "tn_model_create": (I32, [I32, I32, PP]),
    "tn_model_destroy": (I32, [P]),
    "tn_model_n_params": (I32, [P, C.POINTER(C.c_int64)]),
    "tn_model_set_params": (I32, [P, PD]),
    "tn_model_get_params": (I32, [P, PD]),
    "tn_model_state_features": (I32, [P, PI8, PI32, I32, PI32, PI32, PI32, PD, PI32, PI32]),
    "tn_model_loss_grad": (I32, [P, I32, PD, PI32, PI32, I32, PD, PD, PD, P]),
    "tn_model_add_teacher": (I32, [P, P, PI8, PI32, I32, I32]),
    "tn_model_train": (I32, [P, I32, I32, D, U64, PD, PD, P]),
}

_lib = None


class TnError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def lib():
    """Load libtn.so (raises if it has not been built: there is no fallback)."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise RuntimeError(f"native library missing: {LIB_PATH} (run __graft_entry__.build())")
        L = C.CDLL(str(LIB_PATH))
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(code: int):
    if code != TN_OK:
        raise TnError(code, lib().tn_last_error().decode())
