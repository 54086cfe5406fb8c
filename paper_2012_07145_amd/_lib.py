"""ctypes declarations of the C ABI in include/cm.h (libcm.so).

Names and argument order follow the header; this module only marshals
arguments.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libcm.so")

CM_OK, CM_EINVAL, CM_ENOMEM, CM_EDEVICE, CM_EAGAIN, CM_E2BIG = 0, -1, -2, -3, -4, -5
CM_ENOTFOUND, CM_ECANCELED, CM_EUNSUPPORTED = -6, -7, -8
STATUS_NAMES = {0: "CM_OK", -1: "CM_EINVAL", -2: "CM_ENOMEM", -3: "CM_EDEVICE",
                -4: "CM_EAGAIN", -5: "CM_E2BIG", -6: "CM_ENOTFOUND", -7: "CM_ECANCELED",
                -8: "CM_EUNSUPPORTED"}
CM_FP32, CM_BF16, CM_FP8 = 0, 1, 2
CM_MAX_K = 256
CM_N_PARAMS = 4184
CM_STAGE_CHUNK = 32
CM_STEP_MAX_QUERIES = 256
CM_STATIC_MAX_STAGES = 32768

# Every function the header declares, for the export check.
EXPORTS = (
    "cm_model_create", "cm_model_destroy", "cm_workspace_create", "cm_workspace_destroy",
    "cm_eval_batch", "cm_hoist_stages", "cm_eval_hoisted", "cm_topk_per_query",
    "cm_step_create", "cm_step_destroy", "cm_step_run", "cm_step_set_config",
    "cm_step_get_config", "cm_step_autotune", "cm_step_kernel_time", "cm_step_tuned_config",
    "cm_server_create", "cm_server_destroy", "cm_session_open", "cm_session_close",
    "cm_session_beam", "cm_serve_submit", "cm_serve_poll", "cm_serve_wait",
    "cm_serve_submit_batch", "cm_serve_wait_all",
    "cm_server_get_stats", "cm_server_reset_stats", "cm_server_fail_next_launch",
    "cm_model_prepare_fp8", "cm_fp8_calibrate", "cm_fp8_encode",
    "cm_eval_stages", "cm_freeze_stages", "cm_penalize_known_bad", "cm_eval_indexed",
    "cm_sampler_create", "cm_sampler_destroy", "cm_sample_buckets",
    "cm_server_set_step_config", "cm_server_get_step_config", "cm_eval_batch_static",
    "cm_last_error", "cm_version",
)


class cm_model_desc(ctypes.Structure):
    _fields_ = [("n_pipe_features", ctypes.c_int32), ("n_sched_features", ctypes.c_int32),
                ("embed", ctypes.c_int32), ("hidden", ctypes.c_int32),
                ("n_coefs", ctypes.c_int32)]


class cm_workspace_desc(ctypes.Structure):
    _fields_ = [("max_queries", ctypes.c_int32), ("max_stages", ctypes.c_int64),
                ("max_cands", ctypes.c_int64), ("max_rows", ctypes.c_int64),
                ("max_k", ctypes.c_int32)]


class cm_query(ctypes.Structure):
    _fields_ = [("n_stages", ctypes.c_int32), ("n_cands", ctypes.c_int32),
                ("pipe_off", ctypes.c_int64), ("sched_off", ctypes.c_int64),
                ("terms_off", ctypes.c_int64), ("cost_off", ctypes.c_int64)]


class cm_batch(ctypes.Structure):
    _fields_ = [("n_queries", ctypes.c_int32), ("queries", ctypes.POINTER(cm_query)),
                ("pipe", ctypes.c_void_p), ("sched", ctypes.c_void_p),
                ("terms", ctypes.c_void_p)]


class cm_step_desc(ctypes.Structure):
    _fields_ = [("max_queries", ctypes.c_int32), ("max_stages", ctypes.c_int64),
                ("max_cands", ctypes.c_int64), ("max_k", ctypes.c_int32),
                ("slots", ctypes.c_int32)]


class cm_step_config(ctypes.Structure):
    _fields_ = [("grid", ctypes.c_int32), ("group_tiles", ctypes.c_int32),
                ("use_graph", ctypes.c_int32)]


class cm_server_cfg(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("k", ctypes.c_int32),
                ("arena_bytes", ctypes.c_int64), ("max_slots", ctypes.c_int32),
                ("max_pending", ctypes.c_int32), ("max_sessions", ctypes.c_int32),
                ("max_stages", ctypes.c_int32), ("max_batch_queries", ctypes.c_int32),
                ("max_batch_cands", ctypes.c_int64)]


class cm_request(ctypes.Structure):
    _fields_ = [("n_cands", ctypes.c_int32), ("k", ctypes.c_int32),
                ("sched", ctypes.c_void_p), ("terms", ctypes.c_void_p)]


# The same layout as a numpy record, for filling request arrays column by
# column.
REQUEST_DTYPE = np.dtype({"names": ["n_cands", "k", "sched", "terms"],
                          "formats": [np.int32, np.int32, np.uint64, np.uint64],
                          "offsets": [cm_request.n_cands.offset, cm_request.k.offset,
                                      cm_request.sched.offset, cm_request.terms.offset],
                          "itemsize": ctypes.sizeof(cm_request)})
assert ctypes.sizeof(ctypes.c_void_p) == 8 and REQUEST_DTYPE.itemsize == 24


class cm_result(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("n", ctypes.c_int32),
                ("idx", ctypes.POINTER(ctypes.c_int32)), ("val", ctypes.POINTER(ctypes.c_float)),
                ("t_submit_us", ctypes.c_double), ("t_admit_us", ctypes.c_double),
                ("t_done_us", ctypes.c_double)]


class cm_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("canceled", ctypes.c_int64), ("candidates", ctypes.c_int64),
                ("rows", ctypes.c_int64), ("micro_batches", ctypes.c_int64),
                ("wall_us", ctypes.c_double), ("cands_per_s", ctypes.c_double),
                ("p50_us", ctypes.c_double), ("p99_us", ctypes.c_double),
                ("max_us", ctypes.c_double), ("queue_depth", ctypes.c_int32),
                ("in_flight", ctypes.c_int32), ("arena_in_use", ctypes.c_int64),
                ("arena_high_water", ctypes.c_int64), ("kernel_us", ctypes.c_double),
                ("kernel_bytes", ctypes.c_int64), ("kernel_span_us", ctypes.c_double),
                ("kernel_busy_us", ctypes.c_double), ("kernel_busy_launches", ctypes.c_int64)]


class CmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_L = None


def lib():
    global _L
    if _L is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.cm_model_create.argtypes = [ctypes.POINTER(cm_model_desc), vp, ctypes.POINTER(vp)]
        L.cm_model_destroy.argtypes = [vp]
        L.cm_workspace_create.argtypes = [ctypes.POINTER(cm_workspace_desc), ctypes.POINTER(vp)]
        L.cm_workspace_destroy.argtypes = [vp]
        L.cm_eval_batch.argtypes = [vp, i32, ctypes.POINTER(cm_batch), vp, vp, vp]
        L.cm_eval_batch_static.argtypes = [vp, i32, ctypes.POINTER(cm_batch), vp, vp]
        L.cm_hoist_stages.argtypes = [vp, i32, ctypes.POINTER(cm_batch), vp, vp]
        L.cm_eval_hoisted.argtypes = [vp, i32, ctypes.POINTER(cm_batch), vp, vp, vp, vp]
        L.cm_topk_per_query.argtypes = [vp, ctypes.POINTER(cm_batch), i32, vp, vp, vp, vp]
        L.cm_step_create.argtypes = [vp, i32, ctypes.POINTER(cm_step_desc), ctypes.POINTER(vp)]
        L.cm_step_destroy.argtypes = [vp]
        L.cm_step_run.argtypes = [vp, ctypes.POINTER(cm_batch), vp, i32, vp, vp, vp, vp]
        L.cm_step_set_config.argtypes = [vp, ctypes.POINTER(cm_step_config)]
        L.cm_step_get_config.argtypes = [vp, ctypes.POINTER(cm_step_config)]
        L.cm_step_autotune.argtypes = [vp, ctypes.POINTER(cm_batch), vp, i32, vp, vp, vp, vp,
                                       i32, ctypes.POINTER(cm_step_config),
                                       ctypes.POINTER(ctypes.c_float)]
        L.cm_step_tuned_config.argtypes = [vp, i32, i64, ctypes.POINTER(cm_step_config)]
        L.cm_step_kernel_time.argtypes = [vp, ctypes.POINTER(ctypes.c_float)]
        L.cm_server_create.argtypes = [vp, ctypes.POINTER(cm_server_cfg), ctypes.POINTER(vp)]
        L.cm_server_destroy.argtypes = [vp]
        L.cm_session_open.argtypes = [vp, vp, i32, ctypes.POINTER(i32)]
        L.cm_session_close.argtypes = [vp, i32]
        L.cm_session_beam.argtypes = [vp, i32, i32, vp, vp]
        L.cm_serve_submit.argtypes = [vp, i32, ctypes.POINTER(cm_request),
                                      ctypes.POINTER(ctypes.c_uint64)]
        L.cm_serve_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(cm_result)]
        L.cm_serve_wait.argtypes = [vp, ctypes.c_uint64, i32, ctypes.POINTER(cm_result)]
        L.cm_serve_submit_batch.argtypes = [vp, i32, vp, ctypes.POINTER(cm_request), vp]
        L.cm_serve_wait_all.argtypes = [vp, i32, vp, i32, ctypes.POINTER(cm_result)]
        L.cm_server_get_stats.argtypes = [vp, ctypes.POINTER(cm_server_stats)]
        L.cm_server_reset_stats.argtypes = [vp]
        L.cm_server_fail_next_launch.argtypes = [vp]
        fl = ctypes.c_float
        L.cm_model_prepare_fp8.argtypes = [vp, fl, fl]
        L.cm_fp8_calibrate.argtypes = [vp, i64, vp, vp, ctypes.POINTER(fl), ctypes.POINTER(fl)]
        L.cm_fp8_encode.argtypes = [vp, i64, fl, vp, vp]
        L.cm_eval_stages.argtypes = [vp, i32, ctypes.POINTER(cm_batch), vp, vp, vp, vp]
        L.cm_freeze_stages.argtypes = [vp, ctypes.POINTER(cm_batch), vp, i64, vp, vp]
        L.cm_penalize_known_bad.argtypes = [ctypes.POINTER(cm_batch), vp, vp, i64, fl, vp, vp]
        L.cm_eval_indexed.argtypes = [vp, i32, ctypes.POINTER(cm_batch), vp, i64, vp, vp, vp]
        L.cm_sampler_create.argtypes = [i32, i64, ctypes.POINTER(vp)]
        L.cm_sampler_destroy.argtypes = [vp]
        L.cm_sample_buckets.argtypes = [vp, ctypes.POINTER(cm_batch), vp, vp, vp, vp, vp]
        L.cm_server_set_step_config.argtypes = [vp, ctypes.POINTER(cm_step_config)]
        L.cm_server_get_step_config.argtypes = [vp, ctypes.POINTER(cm_step_config)]
        for f in ("cm_model_create", "cm_model_destroy", "cm_workspace_create",
                  "cm_workspace_destroy", "cm_eval_batch", "cm_hoist_stages",
                  "cm_eval_hoisted", "cm_topk_per_query", "cm_step_create",
                  "cm_step_destroy", "cm_step_run", "cm_step_set_config",
                  "cm_step_get_config", "cm_step_autotune", "cm_step_kernel_time", "cm_step_tuned_config",
                  "cm_server_create", "cm_server_destroy", "cm_session_open",
                  "cm_session_close", "cm_session_beam", "cm_serve_submit", "cm_serve_poll",
                  "cm_serve_wait", "cm_server_get_stats", "cm_server_reset_stats",
                  "cm_serve_submit_batch", "cm_serve_wait_all", "cm_model_prepare_fp8",
                  "cm_fp8_calibrate", "cm_fp8_encode", "cm_eval_stages", "cm_freeze_stages",
                  "cm_penalize_known_bad", "cm_eval_indexed", "cm_sampler_create",
                  "cm_sampler_destroy", "cm_sample_buckets", "cm_server_set_step_config",
                  "cm_server_get_step_config", "cm_eval_batch_static"):
            getattr(L, f).restype = i32
        L.cm_last_error.restype = ctypes.c_char_p
        L.cm_last_error.argtypes = []
        L.cm_version.restype = i32
        L.cm_version.argtypes = []
        _L = L
    return _L


def check(status: int):
    if status != CM_OK:
        raise CmError(status, lib().cm_last_error().decode())
    return status
