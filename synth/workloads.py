"""Seeded synthetic workloads for the learned cost model of Anderson et al.,
"Efficient Automatic Scheduling of Imaging and Vision Pipelines for the GPU"
(OOPSLA 2021).

The paper's inputs (featurized schedules of its Halide apps, trained weights)
are not available, so every input is drawn here from fixed seeds:

* weights: N(0, 1/fan_in) (variance 1/fan_in), drawn in float64 and rounded
  to float32 with round-to-nearest-even; biases are zero unless asked for;
* pipeline (algorithm-specific) features, one vector of 56 per stage, shared by
  every candidate of a query: Poisson(3) operation counts (Sec. 5 inherits
  per-stage operation histograms);
* schedule features, 40 per (stage, candidate): exp(N(4, 2^2));
* cost terms, 8 per (stage, candidate): exp(N(6, 1.5^2)) (App. B's terms are
  non-negative products of counts and ratios);
* stage counts log-uniform in [3, 120] ("from a few to around one hundred
  stages", Sec. 6) and candidates per query uniform in [16, 4096].

Array layouts are the ones the C ABI takes: ``pipe[S][56]``,
``sched[S][N][40]`` and ``terms[S][N][8]``, all C-contiguous float32.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

DIMS = dict(FP=56, FS=40, E=24, H=32, C=8)

# Flat parameter blob, in this order (row-major matrices [out][in]).
PARAM_LAYOUT = (
    ("W_p", (24, 56)), ("b_p", (24,)),
    ("W_s", (24, 40)), ("b_s", (24,)),
    ("W_1", (32, 48)), ("b_1", (32,)),
    ("W_2", (8, 32)), ("b_2", (8,)),
)
N_PARAMS = sum(int(np.prod(s)) for _, s in PARAM_LAYOUT)  # 4184
WEIGHT_SEED = 2012


def f32_to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (round to nearest, ties to even) and
    return the 16-bit patterns.  NaN stays NaN (quiet)."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    rounded = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    nan = np.isnan(x)
    out = rounded.astype(np.uint16)
    if nan.any():
        out[nan] = ((u[nan] >> 16) | 0x40).astype(np.uint16)
    return out


def bf16_bits_to_f32(b: np.ndarray) -> np.ndarray:
    """Widen bfloat16 bit patterns to float32 (exact)."""
    b = np.ascontiguousarray(b, dtype=np.uint16)
    return (b.astype(np.uint32) << 16).view(np.float32)


def model_params(seed: int = WEIGHT_SEED, bias: bool = False) -> np.ndarray:
    """Draw the flat float32 parameter blob (length ``N_PARAMS``).

    Weights ~ N(0, 1/fan_in).  Biases are zero unless ``bias`` is set, in
    which case they are drawn the same way right after their weight matrix.
    """
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape in PARAM_LAYOUT:
        if name.startswith("W"):
            fan_in = shape[1]
            w = rng.standard_normal(shape) / math.sqrt(fan_in)
            last_fan_in = fan_in
            parts.append(w.astype(np.float32).ravel())
        elif bias:
            b = rng.standard_normal(shape) / math.sqrt(last_fan_in)
            parts.append(b.astype(np.float32).ravel())
        else:
            parts.append(np.zeros(shape, np.float32).ravel())
    blob = np.concatenate(parts)
    assert blob.size == N_PARAMS
    return blob


def unpack_params(blob: np.ndarray) -> dict:
    """Split a flat blob into named arrays (views, float32)."""
    blob = np.asarray(blob, dtype=np.float32)
    assert blob.size == N_PARAMS, blob.size
    out, o = {}, 0
    for name, shape in PARAM_LAYOUT:
        n = int(np.prod(shape))
        out[name] = blob[o:o + n].reshape(shape)
        o += n
    return out


@dataclass
class Query:
    """One beam step of one search session: N candidates over S stages."""
    pipe: np.ndarray   # [S][56] float32
    sched: np.ndarray  # [S][N][40] float32
    terms: np.ndarray  # [S][N][8] float32

    @property
    def n_stages(self) -> int:
        return self.pipe.shape[0]

    @property
    def n_cands(self) -> int:
        return self.sched.shape[1]


def draw_query(rng: np.random.Generator, S: int, N: int) -> Query:
    """Draw one query: pipeline features, then schedule features stage by
    stage, then cost terms stage by stage."""
    pipe = rng.poisson(3.0, size=(S, 56)).astype(np.float32)
    sched = np.empty((S, N, 40), np.float32)
    for s in range(S):
        sched[s] = np.exp(rng.normal(4.0, 2.0, size=(N, 40))).astype(np.float32)
    terms = np.empty((S, N, 8), np.float32)
    for s in range(S):
        terms[s] = np.exp(rng.normal(6.0, 1.5, size=(N, 8))).astype(np.float32)
    return Query(pipe, sched, terms)


def ragged_sizes(rng: np.random.Generator, n_queries: int,
                 s_lo: int = 3, s_hi: int = 120,
                 n_lo: int = 16, n_hi: int = 4096):
    """Stage counts S = floor(exp(U(ln s_lo, ln(s_hi + 1)))) (log-uniform
    integers in [s_lo, s_hi]) and candidate counts N ~ U{n_lo..n_hi}."""
    u = rng.uniform(math.log(s_lo), math.log(s_hi + 1), size=n_queries)
    S = np.minimum(np.floor(np.exp(u)).astype(np.int64), s_hi)
    N = rng.integers(n_lo, n_hi + 1, size=n_queries)
    return [int(s) for s in S], [int(n) for n in N]


@dataclass
class Workload:
    name: str
    k: int
    precision: str
    queries: list = field(default_factory=list)

    @property
    def n_cands(self) -> int:
        return sum(q.n_cands for q in self.queries)

    @property
    def n_rows(self) -> int:
        return sum(q.n_cands * q.n_stages for q in self.queries)


WORKLOADS = {
    # name: (data seed, builder)
    "plain_64x4": 1,
    "beam_6400x30": 2,
    "precision_65536x64": 3,
    "ragged_17q": 4,
}


def workload(name: str, seed: int | None = None) -> Workload:
    """Build one of the named workloads.

    plain_64x4          1 query, 64 candidates x 4 stages, top-8, fp32
    beam_6400x30        1 query, beam 32 x 200 children x 30 stages, top-32, fp32
    precision_65536x64  1 query, 65,536 candidates x 64 stages, top-32, bf16
    ragged_17q          17 queries, S log-uniform [3,120], N U[16,4096], top-32, bf16
    """
    data_seed = WORKLOADS[name] if seed is None else seed
    rng = np.random.default_rng(data_seed)
    if name == "plain_64x4":
        return Workload(name, 8, "fp32", [draw_query(rng, 4, 64)])
    if name == "beam_6400x30":
        return Workload(name, 32, "fp32", [draw_query(rng, 30, 6400)])
    if name == "precision_65536x64":
        return Workload(name, 32, "bf16", [draw_query(rng, 64, 65536)])
    if name == "ragged_17q":
        S, N = ragged_sizes(rng, 17)
        return Workload(name, 32, "bf16",
                        [draw_query(rng, s, n) for s, n in zip(S, N)])
    raise KeyError(name)


def serving_stream(n_requests: int, n_sessions: int = 256, rate_hz: float = 2000.0,
                   seed: int = 5):
    """Open-loop request stream of the serving workload.

    Returns (session_stages[n_sessions], arrivals) where arrivals is a list
    of (t_seconds, session, n_cands); gaps are Exp(1/rate), sessions are
    uniform per arrival, N ~ U{16..4096}.
    """
    rng = np.random.default_rng(seed)
    sess_S, _ = ragged_sizes(rng, n_sessions)
    gaps = rng.exponential(1.0 / rate_hz, size=n_requests)
    t = np.cumsum(gaps)
    sess = rng.integers(0, n_sessions, size=n_requests)
    n = rng.integers(16, 4097, size=n_requests)
    return sess_S, [(float(a), int(b), int(c)) for a, b, c in zip(t, sess, n)]
