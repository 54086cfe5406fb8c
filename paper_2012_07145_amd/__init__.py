"""MI355X (gfx950) batched evaluator of the learned cost model of Anderson et
al. (OOPSLA 2021, Sec. 5.2 and App. B) with on-device beam top-k (Sec. 4).

Thin Python binding of ``libcm.so`` (include/cm.h).  Functions carry the C
names and only marshal arguments: torch tensors supply device pointers and
the HIP stream, every step of the computation runs in the library's kernels.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import REQUEST_DTYPE as _REQUEST_DTYPE
from ._lib import (CM_BF16, CM_FP8, CM_FP32, CM_MAX_K, CM_N_PARAMS, CM_STAGE_CHUNK,  # noqa: F401
                   CmError, check, lib)

__all__ = [
    "CM_FP32", "CM_BF16", "CM_FP8", "CM_MAX_K", "CmError", "Model", "Workspace", "Batch",
    "cm_model_create", "cm_model_destroy", "cm_workspace_create", "cm_workspace_destroy",
    "cm_eval_batch", "cm_eval_batch_static", "cm_hoist_stages", "cm_eval_hoisted", "cm_topk_per_query",
    "cm_version", "pack_queries", "Step", "cm_step_create", "cm_step_destroy", "cm_step_run",
    "cm_step_set_config", "cm_step_get_config", "cm_step_autotune", "cm_step_kernel_time",
    "cm_step_tuned_config",
    "Server", "cm_server_create", "cm_model_prepare_fp8", "cm_fp8_calibrate", "cm_fp8_encode",
    "cm_eval_stages", "cm_freeze_stages", "cm_penalize_known_bad", "cm_eval_indexed",
    "Sampler", "cm_sampler_create", "cm_sample_buckets",
]

PRECISIONS = {"fp32": CM_FP32, "bf16": CM_BF16, "fp8": CM_FP8}

lib()  # fail at import when the HIP library is missing


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream))


def _ptr(t):
    return None if t is None else ctypes.c_void_p(int(t.data_ptr()))


class Model:
    """Handle of a cm_model (weights resident on the current device)."""

    def __init__(self, handle):
        self.handle = handle

    def close(self):
        if self.handle is not None:
            check(lib().cm_model_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Workspace:
    """Handle of a cm_workspace (device scratch of fixed capacity)."""

    def __init__(self, handle, caps):
        self.handle = handle
        self.caps = caps

    def close(self):
        if self.handle is not None:
            check(lib().cm_workspace_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """A cm_batch: host descriptors plus the device tensors they point into.

    ``queries`` is a sequence of (n_stages, n_cands, pipe_off, sched_off,
    terms_off, cost_off) tuples.  The tensors are kept referenced so that
    they outlive every call made with this batch.
    """

    def __init__(self, queries, pipe, sched, terms):
        n = len(queries)
        self._q = (_lib.cm_query * max(n, 1))()
        for j, q in enumerate(queries):
            self._q[j] = _lib.cm_query(*[int(v) for v in q])
        self.queries = [tuple(int(v) for v in q) for q in queries]
        self.pipe, self.sched, self.terms = pipe, sched, terms
        self.c = _lib.cm_batch(n, self._q, _ptr(pipe), _ptr(sched), _ptr(terms))

    @property
    def n_queries(self):
        return len(self.queries)

    @property
    def n_cands(self):
        return sum(q[1] for q in self.queries)


def cm_version() -> int:
    return int(lib().cm_version())


def cm_model_create(params) -> Model:
    blob = np.ascontiguousarray(params, dtype=np.float32).ravel()
    if blob.size != CM_N_PARAMS:
        raise ValueError(f"expected {CM_N_PARAMS} parameters, got {blob.size}")
    desc = _lib.cm_model_desc(56, 40, 24, 32, 8)
    h = ctypes.c_void_p()
    check(lib().cm_model_create(ctypes.byref(desc), blob.ctypes.data_as(ctypes.c_void_p),
                                ctypes.byref(h)))
    return Model(h)


def cm_model_destroy(model: Model):
    model.close()


def cm_model_prepare_fp8(model: Model, in_scale: float, act_scale: float):
    """Derive the model's FP8 (e4m3) form for input scale in_scale and hidden
    scale act_scale (powers of two)."""
    check(lib().cm_model_prepare_fp8(model.handle, float(in_scale), float(act_scale)))


def cm_fp8_calibrate(model: Model, pipe_rows, sched_rows):
    """(in_scale, act_scale) suggested for the FP8 form from host rows
    pipe_rows[n][56], sched_rows[n][40] (raw float32 features)."""
    p = np.ascontiguousarray(pipe_rows, np.float32).reshape(-1, 56)
    x = np.ascontiguousarray(sched_rows, np.float32).reshape(-1, 40)
    if p.shape[0] != x.shape[0]:
        raise ValueError("pipe_rows and sched_rows differ in row count")
    a, b = ctypes.c_float(), ctypes.c_float()
    check(lib().cm_fp8_calibrate(model.handle, int(p.shape[0]), p.ctypes.data_as(ctypes.c_void_p),
                                 x.ctypes.data_as(ctypes.c_void_p), ctypes.byref(a),
                                 ctypes.byref(b)))
    return a.value, b.value


def cm_fp8_encode(x, in_scale: float, codes_out=None, stream=None):
    """e4m3 codes of log1p(x) * in_scale (x: float32 device tensor) into
    codes_out (uint8 device tensor of x.numel() values, allocated if None)."""
    import torch
    if x.dtype != torch.float32 or not x.is_contiguous():
        raise ValueError("x must be a contiguous float32 tensor")
    if codes_out is None:
        codes_out = torch.empty(x.numel(), dtype=torch.uint8, device=x.device)
    check(lib().cm_fp8_encode(_ptr(x), int(x.numel()), float(in_scale), _ptr(codes_out),
                              _stream_handle(stream)))
    return codes_out


def cm_workspace_create(max_queries, max_stages, max_cands, max_rows, max_k=32) -> Workspace:
    desc = _lib.cm_workspace_desc(int(max_queries), int(max_stages), int(max_cands),
                                  int(max_rows), int(max_k))
    h = ctypes.c_void_p()
    check(lib().cm_workspace_create(ctypes.byref(desc), ctypes.byref(h)))
    return Workspace(h, dict(max_queries=max_queries, max_stages=max_stages,
                             max_cands=max_cands, max_rows=max_rows, max_k=max_k))


def cm_workspace_destroy(ws: Workspace):
    ws.close()


def cm_eval_batch(model: Model, precision, batch: Batch, ws: Workspace, cost_out,
                  stream=None):
    """Predicted runtime of every candidate of every query into cost_out
    (float32 device tensor, indexed by each query's cost_off)."""
    prec = PRECISIONS.get(precision, precision)
    check(lib().cm_eval_batch(model.handle, int(prec), ctypes.byref(batch.c), ws.handle,
                              _ptr(cost_out), _stream_handle(stream)))


def cm_eval_batch_static(model: Model, precision, batch: Batch, cost_out, stream=None):
    """cm_eval_batch without a workspace: the hoisted rows go to the library's
    static device scratch (at most CM_STATIC_MAX_STAGES stages per call; calls
    that overlap on one device race)."""
    prec = PRECISIONS.get(precision, precision)
    check(lib().cm_eval_batch_static(model.handle, int(prec), ctypes.byref(batch.c),
                                     _ptr(cost_out), _stream_handle(stream)))


def cm_eval_stages(model: Model, precision, batch: Batch, ws: Workspace, cost_out, stage_out,
                   stream=None):
    """cm_eval_batch that also writes each query's per-stage costs [S][N] into
    stage_out (float32 device tensor) at terms_off / 8."""
    prec = PRECISIONS.get(precision, precision)
    check(lib().cm_eval_stages(model.handle, int(prec), ctypes.byref(batch.c), ws.handle,
                               _ptr(cost_out), _ptr(stage_out), _stream_handle(stream)))


def cm_freeze_stages(stage_cost, batch: Batch, cand, cand_stride, frozen_out, stream=None):
    """Freeze flags (uint8 device tensor, one per stage in batch order) of the
    kept candidate cand[q * cand_stride] of every query."""
    check(lib().cm_freeze_stages(_ptr(stage_cost), ctypes.byref(batch.c), _ptr(cand),
                                 int(cand_stride), _ptr(frozen_out), _stream_handle(stream)))


def cm_penalize_known_bad(batch: Batch, hashes, bad_sorted, penalty, cost, stream=None):
    """cost[cost_off + i] += penalty where hashes[cost_off + i] is in
    bad_sorted (uint64 device tensors viewed as int64; bad_sorted ascending as
    unsigned 64-bit values)."""
    n_bad = 0 if bad_sorted is None else int(bad_sorted.numel())
    check(lib().cm_penalize_known_bad(ctypes.byref(batch.c), _ptr(hashes), _ptr(bad_sorted),
                                      n_bad, float(penalty), _ptr(cost), _stream_handle(stream)))


def cm_eval_indexed(model: Model, precision, batch: Batch, row_idx, table_rows, ws: Workspace,
                    cost_out, stream=None):
    """cm_eval_batch over memoized rows: batch.sched is the row table,
    row_idx (int32 device tensor) holds each query's row numbers at its
    sched_off."""
    prec = PRECISIONS.get(precision, precision)
    check(lib().cm_eval_indexed(model.handle, int(prec), ctypes.byref(batch.c), _ptr(row_idx),
                                int(table_rows), ws.handle, _ptr(cost_out),
                                _stream_handle(stream)))


class Sampler:
    """Handle of a cm_sampler (device scratch of the hierarchical sampling)."""

    def __init__(self, handle):
        self.handle = handle

    def close(self):
        if self.handle is not None:
            check(lib().cm_sampler_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cm_sampler_create(max_queries, max_options) -> Sampler:
    h = ctypes.c_void_p()
    check(lib().cm_sampler_create(int(max_queries), int(max_options), ctypes.byref(h)))
    return Sampler(h)


def cm_sample_buckets(sampler: Sampler, batch: Batch, hashes, seeds, sel_idx, sel_count,
                      stream=None):
    """Representatives of every query's hash buckets into sel_idx (at
    cost_off, ascending) and their counts into sel_count; seeds: one
    unsigned 64-bit seed per query (host)."""
    sd = np.ascontiguousarray(np.asarray(seeds, dtype=np.uint64).ravel())
    if sd.size < batch.n_queries:
        raise ValueError("one seed per query")
    check(lib().cm_sample_buckets(sampler.handle, ctypes.byref(batch.c), _ptr(hashes),
                                  sd.ctypes.data_as(ctypes.c_void_p), _ptr(sel_idx),
                                  _ptr(sel_count), _stream_handle(stream)))


def cm_hoist_stages(model: Model, precision, batch: Batch, U_out, stream=None):
    """Per-stage hoisted first-layer rows of the batch into U_out (float32
    device tensor of at least sum(n_stages) * 32 values)."""
    prec = PRECISIONS.get(precision, precision)
    check(lib().cm_hoist_stages(model.handle, int(prec), ctypes.byref(batch.c), _ptr(U_out),
                                _stream_handle(stream)))


def cm_eval_hoisted(model: Model, precision, batch: Batch, U, ws: Workspace, cost_out,
                    stream=None):
    """cm_eval_batch reading hoisted rows U written by cm_hoist_stages."""
    prec = PRECISIONS.get(precision, precision)
    check(lib().cm_eval_hoisted(model.handle, int(prec), ctypes.byref(batch.c), _ptr(U),
                                ws.handle, _ptr(cost_out), _stream_handle(stream)))


def cm_topk_per_query(cost, batch: Batch, k: int, ws: Workspace, idx_out, val_out,
                      stream=None):
    """The k best candidates per query into idx_out/val_out [n_queries*k]."""
    check(lib().cm_topk_per_query(_ptr(cost), ctypes.byref(batch.c), int(k), ws.handle,
                                  _ptr(idx_out), _ptr(val_out), _stream_handle(stream)))


class Step:
    """Handle of a cm_step (persistent, graph-replayed beam step)."""

    def __init__(self, handle, model):
        self.handle = handle
        self.model = model  # the step reads the model's device buffers

    def close(self):
        if self.handle is not None:
            check(lib().cm_step_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cm_step_create(model: Model, precision="bf16", max_queries=32, max_stages=4096,
                   max_cands=1 << 16, max_k=32, slots=2) -> Step:
    prec = PRECISIONS.get(precision, precision)
    desc = _lib.cm_step_desc(int(max_queries), int(max_stages), int(max_cands), int(max_k),
                             int(slots))
    h = ctypes.c_void_p()
    check(lib().cm_step_create(model.handle, int(prec), ctypes.byref(desc), ctypes.byref(h)))
    return Step(h, model)


def cm_step_destroy(step: Step):
    step.close()


def cm_step_run(step: Step, batch: Batch, U, k: int, cost_out, idx_out, val_out, stream=None):
    """Hoist (when U is None) + evaluate + select for every query of the
    batch, as one persistent launch (replayed as a graph by default)."""
    check(lib().cm_step_run(step.handle, ctypes.byref(batch.c), _ptr(U), int(k), _ptr(cost_out),
                            _ptr(idx_out), _ptr(val_out), _stream_handle(stream)))


def cm_step_set_config(step: Step, grid=0, group_tiles=1, use_graph=1):
    cfg = _lib.cm_step_config(int(grid), int(group_tiles), int(use_graph))
    check(lib().cm_step_set_config(step.handle, ctypes.byref(cfg)))


def cm_step_get_config(step: Step) -> dict:
    cfg = _lib.cm_step_config()
    check(lib().cm_step_get_config(step.handle, ctypes.byref(cfg)))
    return dict(grid=cfg.grid, group_tiles=cfg.group_tiles, use_graph=cfg.use_graph)


def cm_step_autotune(step: Step, batch: Batch, U, k: int, cost_out, idx_out, val_out,
                     stream=None, reps=10):
    """Time the built-in configurations on this batch and keep the fastest.
    Returns (config dict, median microseconds)."""
    cfg = _lib.cm_step_config()
    us = ctypes.c_float()
    check(lib().cm_step_autotune(step.handle, ctypes.byref(batch.c), _ptr(U), int(k),
                                 _ptr(cost_out), _ptr(idx_out), _ptr(val_out),
                                 _stream_handle(stream), int(reps), ctypes.byref(cfg),
                                 ctypes.byref(us)))
    return dict(grid=cfg.grid, group_tiles=cfg.group_tiles, use_graph=cfg.use_graph), us.value


def cm_step_tuned_config(step: Step, n_queries: int, rows: int = 0):
    """The tuning cache's configuration (dict) for batches of this size on
    the step's device and precision, or None when it holds none."""
    cfg = _lib.cm_step_config()
    st = lib().cm_step_tuned_config(step.handle, int(n_queries), int(rows), ctypes.byref(cfg))
    if st == _lib.CM_ENOTFOUND:
        return None
    check(st)
    return dict(grid=cfg.grid, group_tiles=cfg.group_tiles, use_graph=cfg.use_graph)


def cm_step_kernel_time(step: Step) -> float:
    """Microseconds of the step kernel alone in the step's latest run."""
    us = ctypes.c_float()
    check(lib().cm_step_kernel_time(step.handle, ctypes.byref(us)))
    return us.value


class Server:
    """Handle of a cm_server (continuous batching of beam-step queries)."""

    def __init__(self, handle, model, k):
        self.handle = handle
        self.model = model  # the server reads the model's device buffers
        self.k = k

    def close(self):
        if self.handle is not None:
            check(lib().cm_server_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def session_open(self, pipe) -> int:
        """Open a session for host algorithm features pipe[S][56] (float32)."""
        p = np.ascontiguousarray(pipe, dtype=np.float32)
        sid = ctypes.c_int32()
        check(lib().cm_session_open(self.handle, p.ctypes.data_as(ctypes.c_void_p),
                                    int(p.shape[0]), ctypes.byref(sid)))
        return sid.value

    def session_close(self, sid: int):
        check(lib().cm_session_close(self.handle, int(sid)))

    def session_beam(self, sid: int, k: int):
        idx = np.empty(k, np.int32)
        val = np.empty(k, np.float32)
        check(lib().cm_session_beam(self.handle, int(sid), int(k),
                                    idx.ctypes.data_as(ctypes.c_void_p),
                                    val.ctypes.data_as(ctypes.c_void_p)))
        return idx, val

    def submit(self, sid: int, n_cands: int, sched, terms, k: int) -> int:
        """Queue a request over device tensors sched (bf16 [S][N][40]) and
        terms (float32 [S][N][8]); the tensors must outlive the request."""
        r = _lib.cm_request(int(n_cands), int(k), _ptr(sched), _ptr(terms))
        t = ctypes.c_uint64()
        check(lib().cm_serve_submit(self.handle, int(sid), ctypes.byref(r), ctypes.byref(t)))
        return t.value

    def _result(self, k):
        idx = np.empty(k, np.int32)
        val = np.empty(k, np.float32)
        res = _lib.cm_result(k, 0, idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                             val.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), 0.0, 0.0, 0.0)
        return res, idx, val

    def poll(self, ticket: int):
        """None while the request is not finished, else (idx, val, times)."""
        res, idx, val = self._result(self.k)
        st = lib().cm_serve_poll(self.handle, ctypes.c_uint64(ticket), ctypes.byref(res))
        if st == _lib.CM_EAGAIN:
            return None
        check(st)
        return idx[:res.n], val[:res.n], (res.t_submit_us, res.t_admit_us, res.t_done_us)

    def wait(self, ticket: int, timeout_ms: int = 10000):
        res, idx, val = self._result(self.k)
        check(lib().cm_serve_wait(self.handle, ctypes.c_uint64(ticket), int(timeout_ms),
                                  ctypes.byref(res)))
        return idx[:res.n], val[:res.n], (res.t_submit_us, res.t_admit_us, res.t_done_us)

    def submit_batch(self, sessions, n_cands, sched_ptrs, terms_ptrs, k):
        """Queue len(sessions) requests in one call.  sched_ptrs/terms_ptrs
        are device addresses (ints) of each request's inputs.  Returns the
        tickets as a uint64 array."""
        n = len(sessions)
        sess = np.ascontiguousarray(sessions, dtype=np.int32)
        # the cm_request array filled column by column (one numpy pass per
        # field instead of a ctypes object per request)
        reqs = np.zeros(max(n, 1), _REQUEST_DTYPE)
        reqs["n_cands"][:n] = n_cands
        reqs["k"][:n] = k
        reqs["sched"][:n] = np.asarray(sched_ptrs, dtype=np.uint64)
        reqs["terms"][:n] = np.asarray(terms_ptrs, dtype=np.uint64)
        tickets = np.zeros(max(n, 1), np.uint64)
        check(lib().cm_serve_submit_batch(self.handle, n, sess.ctypes.data_as(ctypes.c_void_p),
                                          reqs.ctypes.data_as(ctypes.POINTER(_lib.cm_request)),
                                          tickets.ctypes.data_as(ctypes.c_void_p)))
        return tickets[:n]

    def wait_all(self, tickets, timeout_ms: int = 60000):
        """Wait for every ticket and release them (results discarded)."""
        t = np.ascontiguousarray(tickets, dtype=np.uint64)
        check(lib().cm_serve_wait_all(self.handle, len(t), t.ctypes.data_as(ctypes.c_void_p),
                                      int(timeout_ms), None))

    def wait_all_results(self, tickets, timeout_ms: int = 60000):
        """Wait for every ticket and release them; returns [(idx, val), ...]
        in ticket order (each the request's beam)."""
        t = np.ascontiguousarray(tickets, dtype=np.uint64)
        n = len(t)
        outs = (_lib.cm_result * max(n, 1))()
        bufs = []
        for j in range(n):
            res, idx, val = self._result(self.k)
            outs[j] = res
            bufs.append((idx, val))
        check(lib().cm_serve_wait_all(self.handle, n, t.ctypes.data_as(ctypes.c_void_p),
                                      int(timeout_ms), outs))
        return [(idx[:outs[j].n], val[:outs[j].n]) for j, (idx, val) in enumerate(bufs)]

    def stats(self) -> dict:
        s = _lib.cm_server_stats()
        check(lib().cm_server_get_stats(self.handle, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in _lib.cm_server_stats._fields_}

    def reset_stats(self):
        check(lib().cm_server_reset_stats(self.handle))

    def fail_next_launch(self):
        """The next micro-batch launch fails (forced from the host)."""
        check(lib().cm_server_fail_next_launch(self.handle))

    def set_step_config(self, grid=0, group_tiles=1, use_graph=1):
        c = _lib.cm_step_config(int(grid), int(group_tiles), int(use_graph))
        check(lib().cm_server_set_step_config(self.handle, ctypes.byref(c)))

    def get_step_config(self):
        c = _lib.cm_step_config()
        check(lib().cm_server_get_step_config(self.handle, ctypes.byref(c)))
        return {"grid": c.grid, "group_tiles": c.group_tiles, "use_graph": c.use_graph}


def cm_server_create(model: Model, k=32, arena_bytes=8 << 30, max_slots=2, max_pending=4096,
                     max_sessions=256, max_stages=128, max_batch_queries=64,
                     max_batch_cands=1 << 17, precision="bf16") -> Server:
    prec = PRECISIONS.get(precision, precision)
    cfg = _lib.cm_server_cfg(int(prec), int(k), int(arena_bytes), int(max_slots),
                             int(max_pending), int(max_sessions), int(max_stages),
                             int(max_batch_queries), int(max_batch_cands))
    h = ctypes.c_void_p()
    check(lib().cm_server_create(model.handle, ctypes.byref(cfg), ctypes.byref(h)))
    return Server(h, model, int(k))


def pack_queries(queries, precision, device="cuda", in_scale=None):
    """Lay a list of queries (objects with pipe[S][56], sched[S][N][40],
    terms[S][N][8] float32 arrays) out in the ABI's flat device arrays.

    The schedule features are stored as float32 (fp32), as bfloat16 (bf16,
    round to nearest even) or as e4m3 codes written by cm_fp8_encode with
    in_scale (fp8).  Returns (Batch, cost tensor).
    """
    import torch
    prec = PRECISIONS.get(precision, precision)
    descs, pipes, scheds, terms = [], [], [], []
    po = so = to = co = 0
    for q in queries:
        S, N = q.sched.shape[0], q.sched.shape[1]
        descs.append((S, N, po, so, to, co))
        pipes.append(np.ascontiguousarray(q.pipe, np.float32).ravel())
        scheds.append(np.ascontiguousarray(q.sched, np.float32).ravel())
        terms.append(np.ascontiguousarray(q.terms, np.float32).ravel())
        po += S * 56
        so += S * N * 40
        to += S * N * 8
        co += N
    pipe_t = torch.from_numpy(np.concatenate(pipes) if pipes else np.zeros(1, np.float32)).to(device)
    sched_f = torch.from_numpy(np.concatenate(scheds) if scheds else np.zeros(8, np.float32)).to(device)
    if prec == CM_FP8:
        if in_scale is None:
            raise ValueError("fp8 needs in_scale")
        sched_t = cm_fp8_encode(sched_f, in_scale)
    else:
        sched_t = sched_f if prec == CM_FP32 else sched_f.to(torch.bfloat16)
    terms_t = torch.from_numpy(np.concatenate(terms) if terms else np.zeros(4, np.float32)).to(device)
    cost_t = torch.zeros(max(co, 1), dtype=torch.float32, device=device)
    return Batch(descs, pipe_t, sched_t, terms_t), cost_t
