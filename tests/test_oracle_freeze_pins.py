"""Pins of the oracle's freezing rule (Sec. 3.2: all but log2 of the stage
count are frozen, the lowest-cost ones) against hand-worked cases and a
brute-force ranking with Python's sort."""
import math

import numpy as np


def test_freeze_counts(oracle_mod):
    # ceil(log2 S) stages stay free: S=1 -> 0, 2 -> 1, 3 -> 2, 4 -> 2, 5 -> 3,
    # 8 -> 3, 9 -> 4, 120 -> 7, 128 -> 7, 129 -> 8
    for S, free in ((1, 0), (2, 1), (3, 2), (4, 2), (5, 3), (8, 3), (9, 4), (120, 7),
                    (128, 7), (129, 8)):
        f = oracle_mod.freeze(np.arange(S, dtype=np.float64))
        assert int(f.sum()) == S - free, (S, f.sum())
        assert f[:S - free].all() and not f[S - free:].any()  # ascending costs: a prefix


def test_freeze_hand_cases(oracle_mod):
    fz = oracle_mod.freeze
    # 5 stages: 2 frozen, the cheapest two (costs 1 and 2 at stages 1 and 3)
    assert fz([5, 1, 4, 2, 3]).tolist() == [0, 1, 0, 1, 0]
    # equal costs: the lower stage index first
    assert fz([2, 1, 1, 1]).tolist() == [0, 1, 1, 0]
    # NaN ranks after every number
    assert fz([np.nan, 3, 2, 1]).tolist() == [0, 0, 1, 1]
    assert fz([np.nan, np.inf, 2, 1, 0]).tolist() == [0, 0, 0, 1, 1]
    # -0 equals +0 (then index order)
    assert fz([0.0, -0.0, 5, 6]).tolist() == [1, 1, 0, 0]
    assert fz([-0.0, 0.0, -1.0, 6]).tolist() == [1, 0, 1, 0]
    # one stage: frozen
    assert fz([7.0]).tolist() == [1]


def test_freeze_brute_force(oracle_mod):
    rng = np.random.default_rng(11)
    for trial in range(300):
        S = int(rng.integers(1, 40))
        c = rng.choice([0.0, -0.0, 1.0, 2.0, 3.0, np.nan, np.inf, -1.5], size=S)
        c = np.where(rng.random(S) < 0.5, rng.normal(size=S), c)
        order = sorted(range(S), key=lambda s: (math.isnan(c[s]), 0.0 if math.isnan(c[s]) else c[s] + 0.0, s))
        free = math.ceil(math.log2(S)) if S > 1 else 0
        want = np.zeros(S, np.uint8)
        want[order[:S - free]] = 1
        assert np.array_equal(oracle_mod.freeze(c), want), (trial, c)
