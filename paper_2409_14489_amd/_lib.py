"""ctypes binding of libcbessfm.so: argument marshalling only.

Every function here forwards to the C ABI declared in ``include/cbessfm.h``;
all arithmetic of the backpropagation runs in the HIP kernels.  Importing this
module fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcbessfm.so")

OK, EINVAL, EUNSUPPORTED, ENOMEM, EHIP, ESYNC, EWORKSPACE = 0, -1, -2, -3, -4, -5, -6

EXPORTED = (
    "cbessfm_plan_check", "cbessfm_plan", "cbessfm_set_coeffs", "cbessfm_set_split_ratio",
    "cbessfm_run", "cbessfm_backward_workspace", "cbessfm_backward", "cbessfm_analytic_coeffs",
    "cbessfm_plan_info", "cbessfm_status", "cbessfm_destroy", "cbessfm_strerror",
    "cbessfm_batch_create", "cbessfm_batch_run", "cbessfm_batch_describe", "cbessfm_batch_status",
    "cbessfm_batch_destroy", "cbessfm_schedule", "cbessfm_autotune",
    "cbessfm_tie_expand", "cbessfm_tie_reduce", "cbessfm_step_weights", "cbessfm_tied_half_taps",
    "cbessfm_complexity", "cbessfm_set_nlpr", "cbessfm_set_gvd_lengths", "cbessfm_backward_gvd",
    "cbessfm_backward_static", "cbessfm_set_wait_limit",
)

STATIC_SCRATCH_BYTES = 64 << 20   # CBESSFM_STATIC_SCRATCH_BYTES

TUNE_MEASURE = 1


class Link(ctypes.Structure):
    _fields_ = [("alpha_db_km", ctypes.c_double), ("beta2_ps2_km", ctypes.c_double),
                ("gamma_w_km", ctypes.c_double), ("span_km", ctypes.c_double),
                ("n_spans", ctypes.c_int32), ("sample_rate_hz", ctypes.c_double),
                ("manakov_8_9", ctypes.c_int32)]


class Subbands(ctypes.Structure):
    _fields_ = [("n_sb", ctypes.c_int32), ("block_sb", ctypes.c_int32),
                ("overlap", ctypes.c_int32), ("fir_mode", ctypes.c_int32), ("boundary", ctypes.c_int32)]


FIR_MODES = {"auto": 0, "time": 1, "freq": 2}


class Coeffs(ctypes.Structure):
    _fields_ = [("n_taps", ctypes.c_int32), ("c", ctypes.POINTER(ctypes.c_float)),
                ("grid_m", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("n_sb", ctypes.c_int32), ("block_sb", ctypes.c_int32), ("block", ctypes.c_int32),
                ("overlap", ctypes.c_int32), ("hop", ctypes.c_int32), ("steps", ctypes.c_int32),
                ("n_taps", ctypes.c_int32), ("threads_per_group", ctypes.c_int32),
                ("team_capacity", ctypes.c_int32), ("step_km", ctypes.c_double),
                ("split_ratio", ctypes.c_double)]


class Instance(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("field_in", ctypes.c_void_p), ("field_out", ctypes.c_void_p),
                ("T", ctypes.c_int64), ("batch", ctypes.c_int32)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int32), ("teams", ctypes.c_int32), ("workgroups", ctypes.c_int32),
                ("items", ctypes.c_int64), ("makespan_s", ctypes.c_double), ("lower_bound_s", ctypes.c_double),
                ("streamed", ctypes.c_int32), ("streamed_items", ctypes.c_int64),
                ("stream_classes", ctypes.c_int32), ("stream_lone", ctypes.c_int32),
                ("kernel_launches", ctypes.c_int32)]


class SchedJob(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("n_items", ctypes.c_int64), ("cost", ctypes.c_double)]


class SchedStats(ctypes.Structure):
    _fields_ = [("grid", ctypes.c_int32), ("n_teams", ctypes.c_int32), ("makespan", ctypes.c_double),
                ("lower_bound", ctypes.c_double)]


class Tuning(ctypes.Structure):
    _fields_ = [("block_sb", ctypes.c_int32), ("overlap", ctypes.c_int32), ("memory", ctypes.c_int32),
                ("covered", ctypes.c_int32), ("measured", ctypes.c_int32), ("predicted_s", ctypes.c_double)]


class CbessfmError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {strerror(code)} ({code})")
        self.code = code


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2409_14489_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i32, i64, dbl, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    LP, SP, CP = ctypes.POINTER(Link), ctypes.POINTER(Subbands), ctypes.POINTER(Coeffs)
    sig = {
        "cbessfm_plan_check": ([LP, SP, i32, dbl, CP], ctypes.c_int),
        "cbessfm_plan": ([ctypes.POINTER(P), LP, SP, i32, dbl, CP], ctypes.c_int),
        "cbessfm_set_coeffs": ([P, P, P, P], ctypes.c_int),
        "cbessfm_set_split_ratio": ([P, dbl, P], ctypes.c_int),
        "cbessfm_run": ([P, P, P, i64, i32, P], ctypes.c_int),
        "cbessfm_backward_workspace": ([P, i64, i32, i32, ctypes.POINTER(sz)], ctypes.c_int),
        "cbessfm_backward": ([P, P, P, P, P, P, i64, i32, i32, P, sz, P], ctypes.c_int),
        "cbessfm_analytic_coeffs": ([LP, SP, i32, dbl, i32, i32, ctypes.POINTER(dbl)], ctypes.c_int),
        "cbessfm_plan_info": ([P, ctypes.POINTER(Info)], ctypes.c_int),
        "cbessfm_status": ([P], ctypes.c_int),
        "cbessfm_destroy": ([P], None),
        "cbessfm_strerror": ([ctypes.c_int], ctypes.c_char_p),
        "cbessfm_batch_create": ([ctypes.POINTER(P), ctypes.POINTER(Instance), i32], ctypes.c_int),
        "cbessfm_batch_run": ([P, P], ctypes.c_int),
        "cbessfm_batch_describe": ([P, ctypes.POINTER(BatchInfo)], ctypes.c_int),
        "cbessfm_batch_status": ([P], ctypes.c_int),
        "cbessfm_batch_destroy": ([P], None),
        "cbessfm_schedule": ([ctypes.POINTER(SchedJob), i32, i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i32),
                              ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(SchedStats)], ctypes.c_int),
        "cbessfm_autotune": ([LP, i32, i32, i32, i64, i32, i32, ctypes.POINTER(Tuning)], ctypes.c_int),
        "cbessfm_tie_expand": ([P, P, i32, i32, i32, ctypes.POINTER(i32), P, P], ctypes.c_int),
        "cbessfm_tie_reduce": ([P, P, i32, i32, i32, ctypes.POINTER(i32), P, P], ctypes.c_int),
        "cbessfm_step_weights": ([LP, i32, ctypes.POINTER(dbl), ctypes.POINTER(dbl)], ctypes.c_int),
        "cbessfm_tied_half_taps": ([LP, i32, i32, i32, ctypes.POINTER(i32)], ctypes.c_int),
        "cbessfm_complexity": ([i32, dbl, i64, i64, i32, i32, i32, ctypes.POINTER(dbl), ctypes.POINTER(dbl)],
                               ctypes.c_int),
        "cbessfm_set_nlpr": ([P, i32], ctypes.c_int),
        "cbessfm_set_gvd_lengths": ([P, P, P], ctypes.c_int),
        "cbessfm_backward_gvd": ([P, P, P, P, P, P, P, i64, i32, i32, P, sz, P], ctypes.c_int),
        "cbessfm_backward_static": ([P, P, P, P, P, P, i64, i32, i32, P], ctypes.c_int),
        "cbessfm_set_wait_limit": ([P, ctypes.c_uint32], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


lib = _load()


def strerror(code: int) -> str:
    return lib.cbessfm_strerror(code).decode()


def check(code: int, what: str) -> None:
    if code != OK:
        raise CbessfmError(code, what)
