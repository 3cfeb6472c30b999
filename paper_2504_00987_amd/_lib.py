"""ctypes binding of liblabs.so: argument marshalling only.

Every computation happens in the HIP library; this module converts Python
arguments into the C ABI of ``include/liblabs.h``.  It raises if the library
has not been built -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblabs.so")

LABS_OK, LABS_E_INVAL, LABS_E_NOMEM, LABS_E_HIP, LABS_E_CANCELLED, LABS_E_NOTFOUND, LABS_E_AGAIN = range(7)
MIN_N, MAX_N, MAX_K = 3, 256, 128
NOALLOC_MAX_WALKS = 65536

EXPORTED = [
    "labs_create", "labs_destroy", "labs_last_error", "labs_status_name", "labs_version",
    "labs_energy_batch", "labs_skew_deviation_batch", "labs_bruteforce_min",
    "labs_skew_bruteforce_min", "labs_tabu_batch",
    "labs_tabu_batch_noalloc",
    "labs_set_launch", "labs_get_launch", "labs_device_peaks",
    "labs_autotune", "labs_memetic_run", "labs_cancel",
    "labs_memetic_checkpoint_bytes", "labs_memetic_save", "labs_memetic_load",
    "labs_server_create", "labs_server_submit",
    "labs_server_poll", "labs_server_cancel", "labs_server_stats", "labs_server_destroy",
]


class TabuParams(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in (
        "steps_rule", "steps_a", "tenure_rule", "lo_num", "lo_den", "lo_add",
        "hi_num", "hi_den", "hi_add", "aspiration", "slo_num", "slo_den", "shi_num",
        "shi_den")]


class Launch(ctypes.Structure):
    _fields_ = [("group_lanes", ctypes.c_int32), ("walks_per_group", ctypes.c_int32),
                ("persistent", ctypes.c_int32), ("groups_per_cu", ctypes.c_int32),
                ("layout", ctypes.c_int32)]


class MemeticParams(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int32), ("p_comb", ctypes.c_uint32), ("mut_rule", ctypes.c_int32),
                ("p_mut", ctypes.c_uint32), ("tabu", TabuParams), ("generations", ctypes.c_int64),
                ("target_e", ctypes.c_int32), ("mode", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("stop_all", ctypes.c_int32), ("waves_per_replica", ctypes.c_int32),
                ("children", ctypes.c_int32), ("resume", ctypes.c_int32)]


class LabsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


_STATUS = {0: "LABS_OK", 1: "LABS_E_INVAL", 2: "LABS_E_NOMEM", 3: "LABS_E_HIP",
           4: "LABS_E_CANCELLED", 5: "LABS_E_NOTFOUND", 6: "LABS_E_AGAIN"}

_lib = None


def load():
    """Load liblabs.so (built by ``python -m paper_2504_00987_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"liblabs.so is not built ({LIB_PATH}); run "
                           "`python -m paper_2504_00987_amd.build` first")
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    PP = ctypes.POINTER(ctypes.c_void_p)
    L.labs_create.argtypes = [PP, ctypes.c_int]
    L.labs_destroy.argtypes = [P]
    L.labs_last_error.argtypes = [P]
    L.labs_last_error.restype = ctypes.c_char_p
    L.labs_status_name.argtypes = [ctypes.c_int]
    L.labs_status_name.restype = ctypes.c_char_p
    L.labs_version.restype = ctypes.c_char_p
    L.labs_energy_batch.argtypes = [P, P, P, i32, i32, i64, P, P]
    L.labs_skew_deviation_batch.argtypes = [P, P, P, i32, i32, i64, P, P]
    L.labs_bruteforce_min.argtypes = [P, i32, ctypes.POINTER(i32), ctypes.POINTER(i64), P]
    L.labs_skew_bruteforce_min.argtypes = L.labs_bruteforce_min.argtypes
    L.labs_tabu_batch.argtypes = [P, ctypes.POINTER(TabuParams), P, i32, P, i32, i64, u64,
                                  P, i32, P, P, P, i32, P]
    L.labs_tabu_batch_noalloc.argtypes = L.labs_tabu_batch.argtypes
    L.labs_device_peaks.argtypes = [P] + [ctypes.POINTER(ctypes.c_double)] * 4
    L.labs_set_launch.argtypes = [P, ctypes.POINTER(Launch)]
    L.labs_get_launch.argtypes = [P, i32, i32, ctypes.POINTER(Launch)]
    L.labs_autotune.argtypes = [P, ctypes.POINTER(TabuParams), i32, i32, i64, u64,
                                ctypes.POINTER(i32)]
    L.labs_memetic_run.argtypes = [P, ctypes.POINTER(MemeticParams), P, i32, i32, u64, P, i32,
                                   P, P, P, P]
    L.labs_cancel.argtypes = [P]
    L.labs_memetic_checkpoint_bytes.argtypes = [P, ctypes.POINTER(i64)]
    L.labs_memetic_save.argtypes = [P, P, i64, P]
    L.labs_memetic_load.argtypes = [P, P, i64, P]
    L.labs_server_create.argtypes = [P, ctypes.POINTER(MemeticParams), i32, PP]
    L.labs_server_submit.argtypes = [P, i32, u64, i32, i64, ctypes.POINTER(i64)]
    L.labs_server_poll.argtypes = [P, i64, P, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)]
    L.labs_server_cancel.argtypes = [P, i64]
    L.labs_server_stats.argtypes = [P] + [ctypes.POINTER(i64)] * 4
    L.labs_server_destroy.argtypes = [P]
    _lib = L
    return L


def check(rc: int, handle=None):
    if rc != LABS_OK:
        msg = ""
        if handle is not None:
            msg = (load().labs_last_error(handle) or b"").decode()
        raise LabsError(rc, msg)
