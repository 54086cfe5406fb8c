"""FP64 CPU oracle of the learned cost model and beam selection.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline use it to check and time the GPU library.  The product path never
imports it; the two share no code.

Python side: ctypes marshalling of numpy arrays into ``libcm_oracle.so``
(built from ``cm_oracle.c``).  The arithmetic lives in the C file.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


class Oracle:
    """ctypes handle on one build of the oracle library."""

    def __init__(self, path: str):
        L = ctypes.CDLL(path)
        L.cmo_n_params.restype = ctypes.c_int32
        L.cmo_max_threads.restype = ctypes.c_int32
        L.cmo_eval.restype = None
        L.cmo_eval.argtypes = [_f32p, ctypes.c_int32, ctypes.c_int32, _f32p, _f32p,
                               _f32p, _f64p, ctypes.c_void_p, ctypes.c_void_p,
                               ctypes.c_int32]
        L.cmo_e4m3_decode.restype = ctypes.c_double
        L.cmo_e4m3_decode.argtypes = [ctypes.c_uint8]
        L.cmo_e4m3_encode.restype = ctypes.c_uint8
        L.cmo_e4m3_encode.argtypes = [ctypes.c_double]
        L.cmo_fp8_scale.restype = ctypes.c_double
        L.cmo_fp8_scale.argtypes = [ctypes.c_double]
        L.cmo_eval_fp8.restype = None
        L.cmo_eval_fp8.argtypes = [_f32p, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                   ctypes.c_int32, _f32p,
                                   np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS"),
                                   _f32p, _f64p, ctypes.c_double, ctypes.c_void_p,
                                   ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
        L.cmo_fp8_codes.restype = None
        L.cmo_fp8_codes.argtypes = [_f32p, ctypes.c_int64, ctypes.c_double,
                                    np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")]
        L.cmo_freeze.restype = ctypes.c_int32
        L.cmo_freeze.argtypes = [_f64p, ctypes.c_int32,
                                 np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")]
        _u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
        L.cmo_penalize_f32.restype = None
        L.cmo_penalize_f32.argtypes = [_f32p, _u64p, ctypes.c_int64, _u64p, ctypes.c_int64,
                                       ctypes.c_float]
        L.cmo_splitmix64.restype = ctypes.c_uint64
        L.cmo_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.cmo_sample.restype = ctypes.c_int64
        L.cmo_sample.argtypes = [_u64p, ctypes.c_int64, ctypes.c_uint64, _i32p]
        L.cmo_select.restype = ctypes.c_int32
        L.cmo_select.argtypes = [_f64p, ctypes.c_int32, ctypes.c_int32, _i32p, _f64p]
        self.L = L
        self.path = path

    def max_threads(self) -> int:
        return int(self.L.cmo_max_threads())

    def n_params(self) -> int:
        return int(self.L.cmo_n_params())

    def eval_query(self, params, pipe, sched, terms, *, nthreads: int = 0,
                   stage_costs: bool = False, coefs: bool = False):
        """FP64 predicted runtime per candidate of one query.

        pipe[S][56], sched[S][N][40], terms[S][N][8] (float32 values).  Returns
        cost[N] (float64), plus stage_cost[S][N] and coef[S][N][8] when asked.
        """
        params, pipe, sched, terms = _f32(params), _f32(pipe), _f32(sched), _f32(terms)
        S, N = sched.shape[0], sched.shape[1]
        assert params.size == self.n_params()
        assert pipe.shape == (S, 56) and sched.shape == (S, N, 40)
        assert terms.shape == (S, N, 8)
        cost = np.empty(N, np.float64)
        sc = np.empty((S, N), np.float64) if stage_costs else None
        co = np.empty((S, N, 8), np.float64) if coefs else None
        self.L.cmo_eval(params, S, N, pipe, sched, terms, cost,
                        None if sc is None else sc.ctypes.data,
                        None if co is None else co.ctypes.data, int(nthreads))
        out = [cost]
        if stage_costs:
            out.append(sc)
        if coefs:
            out.append(co)
        return out[0] if len(out) == 1 else tuple(out)

    def e4m3_decode(self, code: int) -> float:
        return float(self.L.cmo_e4m3_decode(int(code)))

    def e4m3_encode(self, v: float) -> int:
        return int(self.L.cmo_e4m3_encode(float(v)))

    def fp8_scale(self, amax: float) -> float:
        return float(self.L.cmo_fp8_scale(float(amax)))

    def fp8_codes(self, x, in_scale):
        """e4m3 codes of log1p(x) * in_scale (FP64), same shape as x."""
        x = _f32(x)
        out = np.empty(x.shape, np.uint8)
        self.L.cmo_fp8_codes(x.ravel(), x.size, float(in_scale), out.reshape(-1))
        return out

    def eval_query_fp8(self, params, in_scale, act_scale, pipe, codes, terms, *,
                       nthreads: int = 0, acc_tol=None, stage_costs: bool = False):
        """FP64 predicted runtime of the FP8 form: codes[S][N][40] uint8 are e4m3
        codes of log1p(x) * in_scale.  With acc_tol also returns each
        candidate's error bound for product sums off by acc_tol of their
        largest term.  With stage_costs also returns the per-stage costs
        [S][N] (and, with acc_tol, each stage's share of the bound [S][N]).
        Returns cost, or a tuple (cost, [bound,] [stage, [stage_bound]])."""
        params, pipe, terms = _f32(params), _f32(pipe), _f32(terms)
        codes = np.ascontiguousarray(codes, dtype=np.uint8)
        S, N = codes.shape[0], codes.shape[1]
        assert codes.shape == (S, N, 40) and pipe.shape == (S, 56) and terms.shape == (S, N, 8)
        cost = np.empty(N, np.float64)
        bound = np.empty(N, np.float64) if acc_tol is not None else None
        stage = np.empty((S, N), np.float64) if stage_costs else None
        sbound = np.empty((S, N), np.float64) if stage_costs and acc_tol is not None else None

        def vp(a):
            return None if a is None else a.ctypes.data_as(ctypes.c_void_p)
        self.L.cmo_eval_fp8(params, float(in_scale), float(act_scale), S, N, pipe, codes,
                            terms, cost, float(acc_tol or 0.0), vp(bound), int(nthreads),
                            vp(stage), vp(sbound))
        out = [cost] + [a for a in (bound, stage, sbound) if a is not None]
        return tuple(out) if len(out) > 1 else cost

    def freeze(self, stage_cost):
        """Freeze flags (uint8[S]) of one candidate's per-stage costs."""
        c = np.ascontiguousarray(stage_cost, dtype=np.float64).ravel()
        out = np.empty(c.size, np.uint8)
        rc = self.L.cmo_freeze(c, c.size, out)
        if rc != 0:
            raise ValueError(f"cmo_freeze failed ({rc})")
        return out

    def penalize(self, cost, hashes, bad, penalty):
        """float32 costs with penalty added where the hash is in bad."""
        c = np.array(cost, dtype=np.float32).ravel()
        h = np.ascontiguousarray(hashes, dtype=np.uint64).ravel()
        b = np.ascontiguousarray(bad, dtype=np.uint64).ravel()
        assert h.size == c.size
        self.L.cmo_penalize_f32(c, h, c.size, b if b.size else np.zeros(1, np.uint64), b.size,
                                float(penalty))
        return c

    def splitmix64(self, seed: int, i: int) -> int:
        return int(self.L.cmo_splitmix64(seed & (2 ** 64 - 1), i))

    def sample(self, hashes, seed: int):
        """Representatives (ascending option indices) of the hash buckets."""
        h = np.ascontiguousarray(hashes, dtype=np.uint64).ravel()
        out = np.empty(max(1, h.size), np.int32)
        n = self.L.cmo_sample(h if h.size else np.zeros(1, np.uint64), h.size,
                              seed & (2 ** 64 - 1), out)
        if n < 0:
            raise ValueError(f"cmo_sample failed ({n})")
        return out[:n].copy()

    def select(self, cost, k: int):
        """The k best (lowest cost) candidates: (idx int32[k], val float64[k])."""
        cost = np.ascontiguousarray(cost, dtype=np.float64)
        idx = np.empty(k, np.int32)
        val = np.empty(k, np.float64)
        rc = self.L.cmo_select(cost, cost.size, int(k), idx, val)
        if rc != 0:
            raise ValueError(f"cmo_select failed ({rc})")
        return idx, val


_DEFAULT = None


def lib() -> Oracle:
    """The default oracle build, compiled first only if it is missing."""
    global _DEFAULT
    if _DEFAULT is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        _DEFAULT = Oracle(_build.LIB)
    return _DEFAULT


def n_params() -> int:
    return lib().n_params()


def eval_query(*a, **kw):
    return lib().eval_query(*a, **kw)


def select(cost, k: int):
    return lib().select(cost, k)


def eval_query_fp8(*a, **kw):
    return lib().eval_query_fp8(*a, **kw)


def fp8_codes(x, in_scale):
    return lib().fp8_codes(x, in_scale)


def e4m3_encode(v: float) -> int:
    return lib().e4m3_encode(v)


def e4m3_decode(code: int) -> float:
    return lib().e4m3_decode(code)


def fp8_scale(amax: float) -> float:
    return lib().fp8_scale(amax)


def freeze(stage_cost):
    return lib().freeze(stage_cost)


def penalize(cost, hashes, bad, penalty):
    return lib().penalize(cost, hashes, bad, penalty)


def splitmix64(seed: int, i: int) -> int:
    return lib().splitmix64(seed, i)


def sample(hashes, seed: int):
    return lib().sample(hashes, seed)
