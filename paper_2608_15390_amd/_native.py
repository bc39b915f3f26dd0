"""ctypes declarations of the C ABI in ``include/perm_est.h``.

Argument marshalling only: every step of the estimator runs in the HIP
library.  Loading fails loudly when the library has not been built."""
from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
# PERM_EST_LIBRARY selects another build of the same library (same ABI)
LIB_PATH = os.environ.get("PERM_EST_LIBRARY") or os.path.join(_PKG, "libpermest.so")

PE_OK, PE_EINVAL, PE_ENOMEM, PE_EDEVICE, PE_ENOTSUP, PE_EIO = 0, -1, -2, -3, -4, -5


class Options(C.Structure):
    _fields_ = [("device", C.c_int32), ("flags", C.c_uint32)]


class Schedule(C.Structure):
    _fields_ = [
        ("vertex_rule", C.c_int32),
        ("sk_policy", C.c_int32),
        ("dm_policy", C.c_int32),
        ("initial_dm", C.c_int32),
        ("K0", C.c_int32),
        ("K", C.c_int32),
        ("theta_th", C.c_double),
        ("theta_tr", C.c_double),
        ("local_gate", C.c_int32),
        ("local_cap", C.c_int32),
        ("reserved", C.c_int32 * 2),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class Result(C.Structure):
    _fields_ = [
        ("log_estimate", C.c_double),
        ("p_match", C.c_double),
        ("rel_spread", C.c_double),
        ("rse", C.c_double),
        ("ess", C.c_double),
        ("var_logw", C.c_double),
        ("max_logw", C.c_double),
        ("n_traj", C.c_int64),
        ("n_alive", C.c_int64),
        ("n_dm", C.c_int64),
        ("n_full_sk", C.c_int64),
        ("n_local_sk", C.c_int64),
        ("n_steps", C.c_int64),
        ("seconds", C.c_double),
        ("n_entries_scanned", C.c_int64),
        ("n_decrements", C.c_int64),
        ("n_local_entries", C.c_int64),
        ("n_local_values", C.c_int64),
        ("n_mlp_tiles", C.c_int64),
        ("n_entries_scanned_v", C.c_int64),
        ("kernel_seconds", C.c_double),
        ("wave_seconds", C.c_double),
        ("wave_seconds_full_sk", C.c_double),
        ("wave_seconds_dm", C.c_double),
        ("wave_seconds_local", C.c_double),
        ("n_dm_entries", C.c_int64),
        ("launch_blocks", C.c_int32),
        ("launch_waves_per_block", C.c_int32),
        ("launch_trajectories_per_wave", C.c_int32),
        ("launch_blocks_per_cu", C.c_int32),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class ConsensusResult(C.Structure):
    _fields_ = [
        ("log_p_con", C.c_double),
        ("log_e_con", C.c_double),
        ("rel_half_width", C.c_double),
        ("variant_ratio", C.c_double),
        ("min_ess", C.c_double),
        ("d_max", C.c_double),
        ("c_bonf", C.c_double),
        ("t_crit", C.c_double),
        ("checks", C.c_uint32),
        ("provisional", C.c_int32),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


PE_CON_ALL_RUNS, PE_CON_T_INTERVALS, PE_CON_BONFERRONI = 1, 2, 4
PE_CON_ALIVE, PE_CON_ESS, PE_CON_HALF_WIDTH = 8, 16, 32


class RecordBuffers(C.Structure):
    _fields_ = [
        ("x", C.c_void_p),
        ("y", C.c_void_p),
        ("gstart", C.c_void_p),
        ("ginfo", C.c_void_p),
        ("rec_cap", C.c_int64),
        ("group_cap", C.c_int64),
        ("stride", C.c_int32),
        ("reserved", C.c_int32),
    ]


EXPORTS = [
    "perm_est_create",
    "perm_est_create_batch",
    "perm_est_schedule_preset",
    "perm_est_run",
    "perm_est_run_range",
    "perm_est_run_range_noalloc",
    "perm_est_run_batch",
    "perm_est_set_model",
    "perm_est_model_save",
    "perm_est_model_load",
    "perm_est_record",
    "perm_est_mlp_create",
    "perm_est_mlp_get_params",
    "perm_est_mlp_forward",
    "perm_est_mlp_loss_grad",
    "perm_est_mlp_train",
    "perm_est_mlp_destroy",
    "perm_est_consensus",
    "perm_est_destroy",
    "perm_est_last_error",
]

PE_FLAG_FORCE_HBM = 1
PE_FLAG_WAVE_PER_TRAJECTORY = 2
PE_RUN_AUTOTUNE = 1
PE_RUN_GRAPH = 2
PE_SK_LEARNED = 4
PE_MLP_NPARAM = 4801

_lib = None


def load():
    """Load libpermest.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"HIP library {LIB_PATH} is not built; run `python -m paper_2608_15390_amd.build`")
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    L.perm_est_create.argtypes = [C.c_int32, C.c_int64, P, P, P, P, P, C.POINTER(Options), C.POINTER(P)]
    L.perm_est_create.restype = C.c_int
    L.perm_est_schedule_preset.argtypes = [C.c_char_p, C.POINTER(Schedule)]
    L.perm_est_schedule_preset.restype = C.c_int
    L.perm_est_run.argtypes = [P, C.c_int64, C.c_uint64, C.POINTER(Schedule), C.POINTER(Result), P, P, P, P]
    L.perm_est_run.restype = C.c_int
    L.perm_est_run_range.argtypes = [P, C.c_int64, C.c_int64, C.c_uint64, C.POINTER(Schedule),
                                     C.POINTER(Result), P, P, P, P, P, P]
    L.perm_est_run_range.restype = C.c_int
    L.perm_est_run_range_noalloc.argtypes = L.perm_est_run_range.argtypes
    L.perm_est_run_range_noalloc.restype = C.c_int
    PP = C.POINTER(C.c_void_p)
    L.perm_est_create_batch.argtypes = [C.c_int32, P, P, PP, PP, PP, PP, PP, C.POINTER(Options), C.POINTER(P)]
    L.perm_est_create_batch.restype = C.c_int
    L.perm_est_run_batch.argtypes = [P, P, C.c_uint64, C.POINTER(Schedule), P, P, P, P, C.c_int32, P]
    L.perm_est_run_batch.restype = C.c_int
    L.perm_est_set_model.argtypes = [P, P, C.c_double, P]
    L.perm_est_set_model.restype = C.c_int
    L.perm_est_model_save.argtypes = [C.c_char_p, P, C.c_double]
    L.perm_est_model_save.restype = C.c_int
    L.perm_est_model_load.argtypes = [C.c_char_p, P, C.POINTER(C.c_double)]
    L.perm_est_model_load.restype = C.c_int
    L.perm_est_record.argtypes = [P, P, C.c_uint64, C.POINTER(Schedule), C.POINTER(RecordBuffers), P,
                                  C.POINTER(C.c_int64), C.POINTER(C.c_int64), P]
    L.perm_est_record.restype = C.c_int
    L.perm_est_mlp_create.argtypes = [C.c_int32, P, C.POINTER(P)]
    L.perm_est_mlp_create.restype = C.c_int
    L.perm_est_mlp_get_params.argtypes = [P, P, P]
    L.perm_est_mlp_get_params.restype = C.c_int
    L.perm_est_mlp_forward.argtypes = [P, P, C.c_int64, P, P]
    L.perm_est_mlp_forward.restype = C.c_int
    L.perm_est_mlp_loss_grad.argtypes = [P, P, P, P, P, C.c_int64, C.c_int64, C.POINTER(C.c_double), P, P]
    L.perm_est_mlp_loss_grad.restype = C.c_int
    L.perm_est_mlp_train.argtypes = [P, P, P, P, P, C.c_int64, C.c_int32, C.c_int64, C.c_double, C.c_uint64,
                                     P, P]
    L.perm_est_mlp_train.restype = C.c_int
    L.perm_est_mlp_destroy.argtypes = [P]
    L.perm_est_mlp_destroy.restype = None
    L.perm_est_consensus.argtypes = [C.c_int32, C.c_int32, C.POINTER(Result), C.c_double,
                                     C.POINTER(ConsensusResult), P, P]
    L.perm_est_consensus.restype = C.c_int
    L.perm_est_destroy.argtypes = [P]
    L.perm_est_destroy.restype = None
    L.perm_est_last_error.argtypes = []
    L.perm_est_last_error.restype = C.c_char_p
    _lib = L
    return L


class PermEstError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"perm_est error {code}: {msg}")
        self.code = code


def check(rc: int):
    if rc != PE_OK:
        raise PermEstError(rc, load().perm_est_last_error().decode(errors="replace"))
