"""ctypes view of include/cutqc.h.  Loading fails loudly when the built
library is missing: there is no fallback implementation."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcutqc.so")

CQ_OK = 0
STATUS = {0: "CQ_OK", -1: "CQ_ERR_ARG", -2: "CQ_ERR_SHAPE", -3: "CQ_ERR_CUTMAP",
          -4: "CQ_ERR_MASK", -5: "CQ_ERR_WORKSPACE", -6: "CQ_ERR_UNSUPPORTED", -7: "CQ_ERR_HIP"}
PRECISION = {"fp64": 0, "fp32": 1, "bf16": 2, "bf16_split": 3, "fp16": 4, "fp16_split": 5}

MAX_SUBCIRCUITS = 8
MAX_DD_R = 16
FD_NOALLOC_SCRATCH_BYTES = 64 << 20

EXPORTED = ["cq_profile_enable", "cq_profile_read", "cq_plan_json", "cq_autotune_enable",
            "cq_label_balance_enable", "cq_column_scaling_enable", "cq_dd_lanes",
            "cq_autotune_json", "cq_autotune_load", "cq_autotune_save",
            "cq_status_string", "cq_last_error", "cq_validate_cutmap",
            "cq_attribute_workspace_size", "cq_attribute", "cq_fd_workspace_size",
            "cq_reconstruct_fd", "cq_reconstruct_fd_noalloc", "cq_dd_workspace_size", "cq_reconstruct_dd",
            "cq_dd_checkpoint_bytes",
            "cq_dd_bfs_workspace_size", "cq_reconstruct_dd_bfs",
            "cq_sample_shots_workspace_size", "cq_sample_shots", "cq_chi2_workspace_size", "cq_chi2",
            "cq_simulate_workspace_size", "cq_simulate_probabilities", "cq_variants_workspace_size",
            "cq_variant_probabilities", "cq_find_cuts"]

GATE_U, GATE_CZ = 0, 1


class cq_subcircuit(C.Structure):
    _fields_ = [("width", C.c_int32), ("init_cut", C.POINTER(C.c_int32)),
                ("meas_cut", C.POINTER(C.c_int32))]


class cq_dd_instance(C.Structure):
    _fields_ = [("n_sub", C.c_int32), ("subs", C.POINTER(cq_subcircuit)),
                ("entries", C.POINTER(C.c_void_p)),
                ("active", C.POINTER(C.c_uint64)), ("merged", C.POINTER(C.c_uint64)),
                ("fixed", C.POINTER(C.c_uint64)), ("fixed_vals", C.POINTER(C.c_uint64)),
                ("max_active", C.POINTER(C.c_int32))]


class cq_dd_params(C.Structure):
    _fields_ = [("prec", C.c_int), ("R", C.c_int32), ("launch", C.c_int32), ("recursions", C.c_int32),
                ("resume", C.c_void_p), ("checkpoint", C.c_void_p)]


DD_LAUNCH = {"graph": 0, "direct": 1}


class cq_dd_record(C.Structure):
    _fields_ = [("recursion", C.c_int32), ("active", C.c_uint64 * MAX_SUBCIRCUITS), ("merged", C.c_uint64 * MAX_SUBCIRCUITS),
                ("fixed", C.c_uint64 * MAX_SUBCIRCUITS),
                ("fixed_vals", C.c_uint64 * MAX_SUBCIRCUITS),
                ("n_active", C.c_int32), ("total", C.c_double), ("n_list", C.c_int32),
                ("list_val", C.c_double * MAX_DD_R), ("list_rec", C.c_int32 * MAX_DD_R),
                ("list_bin", C.c_uint64 * MAX_DD_R), ("popped", C.c_int32),
                ("tiles", C.c_int64), ("tiles_run", C.c_int64)]


class cq_dd_bfs_params(C.Structure):
    _fields_ = [("prec", C.c_int), ("levels", C.c_int32), ("width", C.c_int32), ("launch", C.c_int32)]


class cq_cut_problem(C.Structure):
    _fields_ = [("n_qubits", C.c_int32), ("n_gates", C.c_int32),
                ("gate_qubits", C.POINTER(C.c_int32)), ("max_width", C.c_int32),
                ("max_subcircuits", C.c_int32)]


class cq_gate(C.Structure):
    _fields_ = [("kind", C.c_int32), ("q0", C.c_int32), ("q1", C.c_int32), ("u", C.c_double * 8)]


class cq_dd_bfs_node(C.Structure):
    _fields_ = [("rec", cq_dd_record), ("level", C.c_int32), ("parent", C.c_int32),
                ("parent_bin", C.c_uint64)]


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2205_05836_amd.build` "
            "(there is no fallback implementation)")
    L = C.CDLL(LIB_PATH)
    st = C.c_int
    p = C.c_void_p
    L.cq_status_string.restype = C.c_char_p
    L.cq_status_string.argtypes = [st]
    L.cq_last_error.restype = C.c_char_p
    L.cq_last_error.argtypes = []
    L.cq_validate_cutmap.restype = st
    L.cq_validate_cutmap.argtypes = [C.c_int32, C.POINTER(cq_subcircuit),
                                     C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    L.cq_attribute_workspace_size.restype = st
    L.cq_attribute_workspace_size.argtypes = [C.POINTER(cq_subcircuit), C.POINTER(C.c_size_t)]
    L.cq_attribute.restype = st
    L.cq_attribute.argtypes = [C.POINTER(cq_subcircuit), p, p, p, C.c_size_t, p]
    L.cq_fd_workspace_size.restype = st
    L.cq_fd_workspace_size.argtypes = [C.c_int32, C.POINTER(cq_subcircuit), C.c_int,
                                       C.POINTER(C.c_int32), C.POINTER(C.c_size_t)]
    L.cq_reconstruct_fd.restype = st
    L.cq_reconstruct_fd.argtypes = [C.c_int32, C.POINTER(cq_subcircuit), C.POINTER(C.c_void_p),
                                    C.c_int, C.POINTER(C.c_int32), p, p, C.c_size_t, p]
    L.cq_reconstruct_fd_noalloc.restype = st
    L.cq_reconstruct_fd_noalloc.argtypes = [C.c_int32, C.POINTER(cq_subcircuit), C.POINTER(C.c_void_p),
                                            C.c_int, C.POINTER(C.c_int32), p, p]
    L.cq_dd_workspace_size.restype = st
    L.cq_dd_workspace_size.argtypes = [C.c_int32, C.POINTER(cq_dd_instance),
                                       C.POINTER(cq_dd_params), C.c_int32, C.POINTER(C.c_size_t)]
    L.cq_dd_bfs_workspace_size.restype = st
    L.cq_dd_bfs_workspace_size.argtypes = [C.POINTER(cq_dd_instance), C.POINTER(cq_dd_bfs_params),
                                           C.POINTER(C.c_size_t)]
    L.cq_reconstruct_dd_bfs.restype = st
    L.cq_reconstruct_dd_bfs.argtypes = [C.POINTER(cq_dd_instance), C.POINTER(cq_dd_bfs_params),
                                        C.POINTER(cq_dd_bfs_node), C.c_int32, C.POINTER(C.c_int32),
                                        C.c_void_p, C.c_size_t, C.c_void_p]
    L.cq_sample_shots_workspace_size.restype = st
    L.cq_sample_shots_workspace_size.argtypes = [C.c_int64, C.c_int64, C.c_int64, C.POINTER(C.c_size_t)]
    L.cq_sample_shots.restype = st
    L.cq_sample_shots.argtypes = [p, C.c_int64, C.c_int64, C.c_int64, C.c_uint64, p, p, C.c_size_t, p]
    L.cq_chi2_workspace_size.restype = st
    L.cq_chi2_workspace_size.argtypes = [C.POINTER(C.c_size_t)]
    L.cq_chi2.restype = st
    L.cq_chi2.argtypes = [p, p, C.c_int64, p, p, C.c_size_t, p]
    L.cq_simulate_workspace_size.restype = st
    L.cq_simulate_workspace_size.argtypes = [C.c_int32, C.POINTER(C.c_size_t)]
    L.cq_simulate_probabilities.restype = st
    L.cq_simulate_probabilities.argtypes = [C.c_int32, C.POINTER(cq_gate), C.c_int32, p, p, C.c_size_t, p]
    L.cq_variants_workspace_size.restype = st
    L.cq_variants_workspace_size.argtypes = [C.POINTER(cq_subcircuit), C.POINTER(C.c_size_t)]
    L.cq_variant_probabilities.restype = st
    L.cq_variant_probabilities.argtypes = [C.POINTER(cq_subcircuit), C.POINTER(cq_gate), C.c_int32, p, p,
                                           C.c_size_t, p]
    L.cq_find_cuts.restype = st
    L.cq_find_cuts.argtypes = [C.POINTER(cq_cut_problem), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                               C.POINTER(C.c_int32), C.POINTER(C.c_double)]
    L.cq_reconstruct_dd.restype = st
    L.cq_reconstruct_dd.argtypes = [C.c_int32, C.POINTER(cq_dd_instance), C.POINTER(cq_dd_params),
                                    C.POINTER(cq_dd_record), C.POINTER(C.c_void_p),
                                    C.POINTER(C.c_int32), p, C.c_size_t, p]
    L.cq_plan_json.restype = st
    L.cq_plan_json.argtypes = [C.c_int32, C.POINTER(cq_subcircuit), C.c_int, C.POINTER(C.c_int32),
                               C.POINTER(C.c_int32), C.c_char_p, C.c_size_t,
                               C.POINTER(C.c_size_t)]
    L.cq_profile_enable.restype = st
    L.cq_profile_enable.argtypes = [C.c_int32]
    L.cq_autotune_enable.restype = st
    L.cq_autotune_enable.argtypes = [C.c_int32]
    L.cq_label_balance_enable.restype = st
    L.cq_label_balance_enable.argtypes = [C.c_int32]
    L.cq_column_scaling_enable.restype = st
    L.cq_column_scaling_enable.argtypes = [C.c_int32]
    L.cq_dd_lanes.restype = st
    L.cq_dd_lanes.argtypes = [C.c_int32]
    L.cq_autotune_load.restype = st
    L.cq_autotune_load.argtypes = [C.c_char_p]
    L.cq_autotune_save.restype = st
    L.cq_autotune_save.argtypes = [C.c_char_p]
    L.cq_dd_checkpoint_bytes.restype = C.c_size_t
    L.cq_dd_checkpoint_bytes.argtypes = []
    L.cq_autotune_json.restype = st
    L.cq_autotune_json.argtypes = [C.c_char_p, C.c_size_t, C.POINTER(C.c_size_t)]
    L.cq_profile_read.restype = st
    L.cq_profile_read.argtypes = [C.c_char_p, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                  C.c_int32, C.POINTER(C.c_int32)]
    _lib = L
    return L


class CQError(RuntimeError):
    def __init__(self, status, detail):
        self.status = status
        super().__init__(f"{STATUS.get(status, status)}: {detail}")


def check(status: int):
    if status != CQ_OK:
        raise CQError(status, lib().cq_last_error().decode())
