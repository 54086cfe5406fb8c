"""CPU-side checks of the C ABI: the library loads, exports every function
include/cm.h declares, and rejects bad arguments before any device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = []
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not h.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(cm_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def cm():
    import paper_2012_07145_amd as cm
    return cm


def test_header_declares_the_boundary():
    names = _declared_functions()
    for f in ("cm_eval_batch", "cm_topk_per_query", "cm_model_create", "cm_workspace_create"):
        assert f in names


def test_library_exports_every_declared_symbol(cm):
    from paper_2012_07145_amd import _lib
    L = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in _declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    assert set(_lib.EXPORTS) <= set(_declared_functions())


def test_version(cm):
    assert cm.cm_version() == (0 << 16) | 1


def test_invalid_arguments_are_rejected_before_device_work(cm):
    from paper_2012_07145_amd import _lib
    L = _lib.lib()
    h = ctypes.c_void_p()
    assert L.cm_model_create(None, None, ctypes.byref(h)) == _lib.CM_EINVAL
    bad = _lib.cm_model_desc(56, 40, 24, 31, 8)
    blob = (ctypes.c_float * 4184)()
    assert L.cm_model_create(ctypes.byref(bad), blob, ctypes.byref(h)) == _lib.CM_EINVAL
    assert b"56/40/24/32/8" in L.cm_last_error()
    good = _lib.cm_model_desc(56, 40, 24, 32, 8)
    blob[7] = float("nan")
    assert L.cm_model_create(ctypes.byref(good), blob, ctypes.byref(h)) == _lib.CM_EINVAL
    wd = _lib.cm_workspace_desc(0, 1, 1, 1, 8)
    assert L.cm_workspace_create(ctypes.byref(wd), ctypes.byref(h)) == _lib.CM_EINVAL
    wd = _lib.cm_workspace_desc(1, 1, 1, 1, 257)
    assert L.cm_workspace_create(ctypes.byref(wd), ctypes.byref(h)) == _lib.CM_EINVAL
    assert L.cm_eval_batch(None, 0, None, None, None, None) == _lib.CM_EINVAL
    assert L.cm_topk_per_query(None, None, 8, None, None, None, None) == _lib.CM_EINVAL
    assert L.cm_model_destroy(None) == _lib.CM_EINVAL
    assert L.cm_workspace_destroy(None) == _lib.CM_EINVAL


def test_binding_refuses_wrong_parameter_count(cm):
    import numpy as np
    with pytest.raises(ValueError):
        cm.cm_model_create(np.zeros(10, np.float32))


def test_step_arguments_are_rejected_before_device_work(cm):
    from paper_2012_07145_amd import _lib
    L = _lib.lib()
    h = ctypes.c_void_p()
    good = _lib.cm_step_desc(4, 64, 1024, 32, 2)
    assert L.cm_step_create(None, _lib.CM_BF16, ctypes.byref(good), ctypes.byref(h)) == _lib.CM_EINVAL
    # a model handle is only read after the arguments have been checked
    fake = ctypes.c_void_p(16)
    assert L.cm_step_create(fake, _lib.CM_FP32, ctypes.byref(good), ctypes.byref(h)) == _lib.CM_EUNSUPPORTED
    for bad in (_lib.cm_step_desc(0, 64, 1024, 32, 2),       # no queries
                _lib.cm_step_desc(257, 64, 1024, 32, 2),     # above CM_STEP_MAX_QUERIES
                _lib.cm_step_desc(4, 64, 1024, 257, 2),      # k above CM_MAX_K
                _lib.cm_step_desc(4, 64, 1024, 32, 0),       # no slot
                _lib.cm_step_desc(4, 64, 1024, 32, 9)):      # too many slots
        assert L.cm_step_create(fake, _lib.CM_BF16, ctypes.byref(bad), ctypes.byref(h)) == _lib.CM_EINVAL
    assert L.cm_step_run(None, None, None, 8, None, None, None, None) == _lib.CM_EINVAL
    assert L.cm_step_destroy(None) == _lib.CM_EINVAL
    cfg = _lib.cm_step_config(0, 1, 1)
    assert L.cm_step_set_config(None, ctypes.byref(cfg)) == _lib.CM_EINVAL
    assert L.cm_step_get_config(None, ctypes.byref(cfg)) == _lib.CM_EINVAL
    assert L.cm_step_autotune(None, None, None, 8, None, None, None, None, 5, None, None) == _lib.CM_EINVAL


def test_server_arguments_are_rejected_before_device_work(cm):
    from paper_2012_07145_amd import _lib
    L = _lib.lib()
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(16)
    good = dict(precision=_lib.CM_BF16, k=32, arena_bytes=1 << 30, max_slots=2, max_pending=64,
                max_sessions=8, max_stages=128, max_batch_queries=16, max_batch_cands=1 << 16)
    assert L.cm_server_create(None, ctypes.byref(_lib.cm_server_cfg(**good)), ctypes.byref(h)) == _lib.CM_EINVAL
    assert L.cm_server_create(fake, None, ctypes.byref(h)) == _lib.CM_EINVAL
    assert L.cm_server_create(fake, ctypes.byref(_lib.cm_server_cfg(**{**good, "precision": _lib.CM_FP32})),
                              ctypes.byref(h)) == _lib.CM_EUNSUPPORTED
    for bad in ({"k": 0}, {"k": 257}, {"max_slots": 0}, {"max_slots": 9}, {"max_pending": 0},
                {"max_batch_queries": 257}, {"max_batch_cands": 0}, {"arena_bytes": 0}):
        cfg = _lib.cm_server_cfg(**{**good, **bad})
        assert L.cm_server_create(fake, ctypes.byref(cfg), ctypes.byref(h)) == _lib.CM_EINVAL, bad
    assert L.cm_server_destroy(None) == _lib.CM_EINVAL
    sid = ctypes.c_int32()
    assert L.cm_session_open(None, None, 4, ctypes.byref(sid)) == _lib.CM_EINVAL
    assert L.cm_session_close(None, 0) == _lib.CM_EINVAL
    t = ctypes.c_uint64()
    assert L.cm_serve_submit(None, 0, None, ctypes.byref(t)) == _lib.CM_EINVAL
    assert L.cm_serve_poll(None, 1, None) == _lib.CM_EINVAL
    assert L.cm_serve_wait(None, 1, 10, None) == _lib.CM_EINVAL
    assert L.cm_server_get_stats(None, None) == _lib.CM_EINVAL
    assert L.cm_server_reset_stats(None) == _lib.CM_EINVAL


def test_fp8_arguments_are_rejected_before_device_work(cm):
    from paper_2012_07145_amd import _lib
    L = _lib.lib()
    f = ctypes.c_float()
    x = (ctypes.c_float * 64)()
    assert L.cm_model_prepare_fp8(None, 1.0, 1.0) == _lib.CM_EINVAL
    assert L.cm_fp8_calibrate(None, 1, x, x, ctypes.byref(f), ctypes.byref(f)) == _lib.CM_EINVAL
    assert L.cm_fp8_encode(None, 0, 1.0, None, None) == _lib.CM_OK          # nothing to do
    assert L.cm_fp8_encode(None, -1, 1.0, None, None) == _lib.CM_EINVAL
    assert L.cm_fp8_encode(None, 4, 1.0, None, None) == _lib.CM_EINVAL
    for s in (3.0, 0.0, -2.0, float("nan"), float("inf")):
        assert L.cm_fp8_encode(x, 4, s, x, None) == _lib.CM_EINVAL, s
    base = (ctypes.addressof(x) + 15) // 16 * 16
    assert L.cm_fp8_encode(base, 8, 1.0, base + 16, None) == _lib.CM_EINVAL  # overlap
    assert b"overlap" in L.cm_last_error()
    assert L.cm_fp8_encode(base + 4, 4, 1.0, base + 64, None) == _lib.CM_EINVAL  # misaligned


def test_stage_and_freeze_arguments_are_rejected_before_device_work(cm):
    from paper_2012_07145_amd import _lib
    L = _lib.lib()
    assert L.cm_eval_stages(None, 1, None, None, None, None, None) == _lib.CM_EINVAL
    assert L.cm_freeze_stages(None, None, None, 1, None, None) == _lib.CM_EINVAL
    q = (_lib.cm_query * 1)(_lib.cm_query(3, 2, 0, 0, 12, 0))
    b = _lib.cm_batch(1, q, None, None, None)
    buf = (ctypes.c_int32 * 8)()
    assert L.cm_freeze_stages(buf, ctypes.byref(b), buf, 1, buf, None) == _lib.CM_EINVAL
    assert b"multiple of 8" in L.cm_last_error()
    q[0] = _lib.cm_query(3, 2, 0, 0, 16, 0)
    assert L.cm_freeze_stages(buf, ctypes.byref(b), buf, 0, buf, None) == _lib.CM_EINVAL
    assert L.cm_freeze_stages(buf, ctypes.byref(b), None, 1, buf, None) == _lib.CM_EINVAL
    assert L.cm_freeze_stages(None, ctypes.byref(b), buf, 1, buf, None) == _lib.CM_EINVAL
    q[0] = _lib.cm_query(0, 2, 0, 0, 16, 0)
    assert L.cm_freeze_stages(buf, ctypes.byref(b), buf, 1, buf, None) == _lib.CM_EINVAL


def test_penalty_arguments_are_rejected_before_device_work(cm):
    from paper_2012_07145_amd import _lib
    L = _lib.lib()
    q = (_lib.cm_query * 1)(_lib.cm_query(1, 4, 0, 0, 0, 0))
    b = _lib.cm_batch(1, q, None, None, None)
    buf = (ctypes.c_int64 * 8)()
    assert L.cm_penalize_known_bad(None, buf, buf, 1, 1.0, buf, None) == _lib.CM_EINVAL
    assert L.cm_penalize_known_bad(ctypes.byref(b), buf, buf, -1, 1.0, buf, None) == _lib.CM_EINVAL
    assert L.cm_penalize_known_bad(ctypes.byref(b), buf, None, 2, 1.0, buf, None) == _lib.CM_EINVAL
    assert L.cm_penalize_known_bad(ctypes.byref(b), buf, buf, 2, float("nan"), buf, None) == _lib.CM_EINVAL
    assert L.cm_penalize_known_bad(ctypes.byref(b), None, buf, 2, 1.0, buf, None) == _lib.CM_EINVAL
    assert L.cm_penalize_known_bad(ctypes.byref(b), None, None, 0, 1.0, None, None) == _lib.CM_OK


def test_sampler_arguments_are_rejected_before_device_work(cm):
    from paper_2012_07145_amd import _lib
    L = _lib.lib()
    h = ctypes.c_void_p()
    assert L.cm_sampler_create(0, 10, ctypes.byref(h)) == _lib.CM_EINVAL
    assert L.cm_sampler_create(1, 0, ctypes.byref(h)) == _lib.CM_EINVAL
    assert L.cm_sampler_create(1, 2 ** 31, ctypes.byref(h)) == _lib.CM_EINVAL
    assert L.cm_sampler_destroy(None) == _lib.CM_EINVAL
    assert L.cm_sample_buckets(None, None, None, None, None, None, None) == _lib.CM_EINVAL


def test_log_table_range_reading():
    # The bf16 evaluator's log table holds the codes 0x3380 .. 0x3380 + 8191
    # (csrc/cm_internal.h: LOG_BASE, LOG_N).  Every smaller non-negative code
    # maps to entry 0, which is right only if 1 + x rounds to 1 in float32
    # for all of them (round to nearest even), and the first code of the
    # table must be the last one that does.  The table ends just below 2^40.
    import numpy as np
    from synth import bf16_bits_to_f32
    base, n = 0x3380, 8192
    one = np.float32(1.0)
    below = bf16_bits_to_f32(np.arange(0, base + 1, dtype=np.uint16))
    assert np.all(one + below == one)
    assert one + bf16_bits_to_f32(np.array([base + 1], np.uint16))[0] > one
    last = bf16_bits_to_f32(np.array([base + n - 1, base + n], np.uint16))
    assert last[0] < 2.0 ** 40 <= last[1]


def test_query_above_the_32_bit_offsets_is_rejected_before_device_work(cm):
    # The bf16 and FP8 evaluators address one query's features and terms
    # with 32-bit byte offsets; a query that would reach 2^32 - 2^16 bytes is
    # rejected with CM_E2BIG before the model or workspace is read (fake
    # handles: reading them would crash this process).
    from paper_2012_07145_amd import _lib
    L = _lib.lib()
    fake = ctypes.c_void_p(16)
    limit = 2 ** 32 - 2 ** 16
    buf = (ctypes.c_float * 64)()
    base = (ctypes.addressof(buf) + 15) // 16 * 16

    def batch(S, N):
        q = (_lib.cm_query * 2)(_lib.cm_query(4, 100, 0, 0, 0, 0), _lib.cm_query(S, N, 0, 0, 0, 0))
        return q, _lib.cm_batch(2, q, base, base, base)

    # bf16: 64 x 840,000 rows of 80 feature bytes = 4.3e9
    q, b = batch(64, 840_000)
    assert 64 * 840_000 * 80 > limit
    assert L.cm_eval_batch(fake, _lib.CM_BF16, ctypes.byref(b), fake, base, None) == _lib.CM_E2BIG
    msg = L.cm_last_error()
    assert b"query 1" in msg and b"schedule features" in msg
    assert L.cm_eval_stages(fake, _lib.CM_BF16, ctypes.byref(b), fake, base, base, None) == _lib.CM_E2BIG
    assert L.cm_eval_hoisted(fake, _lib.CM_BF16, ctypes.byref(b), base, fake, base, None) == _lib.CM_E2BIG
    # the largest bf16 query below the limit is only a little smaller
    S, N = 64, limit // (64 * 80)
    assert S * N * 80 <= limit < S * (N + 1) * 80
    # FP8: 40 feature bytes per row, so twice the rows before the limit
    q, b = batch(128, 840_000)
    assert L.cm_eval_batch(fake, _lib.CM_FP8, ctypes.byref(b), fake, base, None) == _lib.CM_E2BIG
    assert b"schedule features" in L.cm_last_error()
    # memoized rows: the features come from the table, the terms still count
    # (1024 x 140,000 rows of 32 term bytes = 4.6e9)
    q, b = batch(1024, 140_000)
    rc = L.cm_eval_indexed(fake, _lib.CM_BF16, ctypes.byref(b), base, 16, fake, base, None)
    assert rc == _lib.CM_E2BIG
    assert b"cost terms" in L.cm_last_error()


def test_static_scratch_limits_are_checked_before_device_work(cm):
    # cm_eval_batch_static keeps the hoisted rows in a fixed device array of
    # CM_STATIC_MAX_STAGES stages: a batch with more stages, or a query above
    # the 32-bit offsets, is rejected with CM_E2BIG before the model is read
    # (fake handle: reading it would crash this process).
    from paper_2012_07145_amd import _lib
    L = _lib.lib()
    fake = ctypes.c_void_p(16)
    buf = (ctypes.c_float * 64)()
    base = (ctypes.addressof(buf) + 15) // 16 * 16
    n = _lib.CM_STATIC_MAX_STAGES // 100 + 1
    q = (_lib.cm_query * n)(*[_lib.cm_query(100, 16, 0, 0, 0, 0) for _ in range(n)])
    b = _lib.cm_batch(n, q, base, base, base)
    assert n * 100 > _lib.CM_STATIC_MAX_STAGES
    for prec in (_lib.CM_FP32, _lib.CM_BF16, _lib.CM_FP8):
        assert L.cm_eval_batch_static(fake, prec, ctypes.byref(b), base, None) == _lib.CM_E2BIG
        assert b"static scratch" in L.cm_last_error()
    q1 = (_lib.cm_query * 1)(_lib.cm_query(64, 840_000, 0, 0, 0, 0))
    b1 = _lib.cm_batch(1, q1, base, base, base)
    assert L.cm_eval_batch_static(fake, _lib.CM_BF16, ctypes.byref(b1), base, None) == _lib.CM_E2BIG
    assert b"schedule features" in L.cm_last_error()
    assert L.cm_eval_batch_static(None, _lib.CM_BF16, ctypes.byref(b1), base, None) == _lib.CM_EINVAL
