"""Pins of the oracle's known-bad-state penalty (Sec. 4.5): hand cases, the
float32 addition, and a penalty that moves a candidate out of the beam."""
import numpy as np


def test_penalty_hand_cases(oracle_mod):
    pen = oracle_mod.penalize
    h = np.array([5, 6, 7, 6, 2 ** 63 + 1], np.uint64)
    c = np.array([1.0, 2.0, 3.0, np.nan, -0.0], np.float32)
    got = pen(c, h, np.array([6, 2 ** 63 + 1], np.uint64), 10.0)
    assert got[0] == 1.0 and got[1] == 12.0 and got[2] == 3.0 and np.isnan(got[3])
    assert got[4] == 10.0
    # no bad hashes, zero penalty: unchanged, bit for bit (signed zero kept)
    assert np.array_equal(pen(c, h, np.zeros(0, np.uint64), 10.0).view(np.uint32)[[0, 1, 2, 4]],
                          c.view(np.uint32)[[0, 1, 2, 4]])
    assert pen(c, h, np.array([7], np.uint64), 0.0)[2] == 3.0
    # +inf pushes behind every finite cost
    assert pen(c, h, np.array([5], np.uint64), np.inf)[0] == np.inf


def test_penalty_is_float32_addition(oracle_mod):
    # 1 + 2^-30 is not a float32: the penalized cost is 1.0 exactly
    got = oracle_mod.penalize(np.array([1.0], np.float32), np.array([3], np.uint64),
                              np.array([3], np.uint64), 2.0 ** -30)
    assert got[0] == np.float32(1.0)
    got = oracle_mod.penalize(np.array([1.0], np.float32), np.array([3], np.uint64),
                              np.array([3], np.uint64), 2.0 ** -23)
    assert got[0] == np.float32(1.0 + 2.0 ** -23)


def test_penalty_moves_candidates_back(oracle_mod):
    c = np.arange(10, dtype=np.float32)
    h = np.arange(10, dtype=np.uint64) % 3
    got = oracle_mod.penalize(c, h, np.array([0], np.uint64), 100.0)
    idx, _ = oracle_mod.select(got.astype(np.float64), 4)
    assert idx.tolist() == [1, 2, 4, 5]   # 0, 3, 6, 9 carry the bad hash 0
