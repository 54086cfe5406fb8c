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
from ._lib import (CM_BF16, CM_FP32, CM_MAX_K, CM_N_PARAMS, CM_STAGE_CHUNK,  # noqa: F401
                   CmError, check, lib)

__all__ = [
    "CM_FP32", "CM_BF16", "CM_MAX_K", "CmError", "Model", "Workspace", "Batch",
    "cm_model_create", "cm_model_destroy", "cm_workspace_create", "cm_workspace_destroy",
    "cm_eval_batch", "cm_hoist_stages", "cm_eval_hoisted", "cm_topk_per_query",
    "cm_version", "pack_queries",
]

PRECISIONS = {"fp32": CM_FP32, "bf16": CM_BF16}

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


def pack_queries(queries, precision, device="cuda"):
    """Lay a list of queries (objects with pipe[S][56], sched[S][N][40],
    terms[S][N][8] float32 arrays) out in the ABI's flat device arrays.

    The schedule features are stored as float32 (fp32) or as bfloat16
    (bf16, round to nearest even).  Returns (Batch, cost tensor).
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
    sched_t = sched_f if prec == CM_FP32 else sched_f.to(torch.bfloat16)
    terms_t = torch.from_numpy(np.concatenate(terms) if terms else np.zeros(4, np.float32)).to(device)
    cost_t = torch.zeros(max(co, 1), dtype=torch.float32, device=device)
    return Batch(descs, pipe_t, sched_t, terms_t), cost_t
