"""Shared test cases: hand-worked examples and small special-case inputs.

Builds parameter blobs and queries for the pins of the cost model; holds no
cost-model arithmetic of its own.
"""
from __future__ import annotations

import json
import os

import numpy as np

from synth import N_PARAMS, PARAM_LAYOUT, unpack_params

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_golden(name: str) -> dict:
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def zero_params() -> np.ndarray:
    return np.zeros(N_PARAMS, np.float32)


def set_params(blob: np.ndarray, entries: dict) -> np.ndarray:
    """entries: {name: [[i, (j,) value], ...]} written into the flat blob."""
    P = unpack_params(blob)
    for name, items in entries.items():
        for it in items:
            *ix, val = it
            P[name][tuple(int(i) for i in ix)] = val
    return blob


def hand_query(terms_rows, n_cands: int = 1, sched0: float = 0.0, pipe0: float = 0.0):
    """A query whose raw features are zero except feature 0 of every stage;
    every candidate gets the same cost terms per stage."""
    terms_rows = np.asarray(terms_rows, np.float32)
    S = terms_rows.shape[0]
    pipe = np.zeros((S, 56), np.float32)
    pipe[:, 0] = pipe0
    sched = np.zeros((S, n_cands, 40), np.float32)
    sched[:, :, 0] = sched0
    terms = np.broadcast_to(terms_rows[:, None, :], (S, n_cands, 8)).copy()
    return pipe, sched, terms


def hand_params() -> np.ndarray:
    g = load_golden("hand_examples.json")
    return set_params(zero_params(), g["params_nonzero"])


def log_params(route: str) -> np.ndarray:
    """Route one feature straight to coefficient 0 with unit weights."""
    blob = zero_params()
    if route == "sched":
        ent = {"W_s": [[0, 0, 1.0]], "W_1": [[0, 24, 1.0]], "W_2": [[0, 0, 1.0]]}
    else:
        ent = {"W_p": [[0, 0, 1.0]], "W_1": [[0, 0, 1.0]], "W_2": [[0, 0, 1.0]]}
    return set_params(blob, ent)


def positive_params(rng: np.random.Generator) -> np.ndarray:
    """All weights and biases strictly positive: every ReLU stays inactive
    when the features are non-negative."""
    parts = []
    for name, shape in PARAM_LAYOUT:
        parts.append(rng.uniform(0.01, 0.2, size=shape).astype(np.float32).ravel())
    return np.concatenate(parts)


def key_tuple(c: float, i: int):
    """Ranking key used by the brute-force selection check: NaN after all
    numbers, -0 == +0, then the candidate index."""
    if np.isnan(c):
        return (1, 0.0, i)
    return (0, float(c) + 0.0, i)
