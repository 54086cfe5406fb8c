"""Pins of the oracle's hierarchical sampling (Sec. 3.1: log2(B) random
representatives per bucket of structurally equal options) against the
published outputs of its generator, hand-counted bucket sizes, a brute-force
selection with Python's sort, and the uniformity of the draws."""
import math

import numpy as np


def test_splitmix64_reference_outputs(oracle_mod):
    # the first five outputs of SplitMix64 seeded with 1234567, as printed by
    # the public-domain reference implementation
    want = [6457827717110365317, 3203168211198807973, 9817491932198370423,
            4593380528125082431, 16408922859458223821]
    assert [oracle_mod.splitmix64(1234567, i) for i in range(5)] == want


def test_representatives_per_bucket(oracle_mod):
    # one bucket of B options keeps max(1, ceil(log2 B)) of them
    for B, r in ((1, 1), (2, 1), (3, 2), (4, 2), (5, 3), (8, 3), (9, 4), (16, 4), (17, 5),
                 (1000, 10), (1024, 10), (1025, 11)):
        got = oracle_mod.sample(np.full(B, 77, np.uint64), 9)
        assert got.size == r, (B, got.size)
        assert np.all(np.diff(got) > 0) and got.min() >= 0 and got.max() < B
    # all hashes distinct: every option is its own bucket's representative
    h = np.arange(50, dtype=np.uint64) * np.uint64(2 ** 40 + 3)
    assert np.array_equal(oracle_mod.sample(h, 5), np.arange(50))
    assert oracle_mod.sample(np.zeros(0, np.uint64), 5).size == 0


def test_sample_brute_force(oracle_mod):
    rng = np.random.default_rng(3)
    for trial in range(60):
        n = int(rng.integers(1, 300))
        pool = rng.integers(0, 2 ** 64, size=int(rng.integers(1, 40)), dtype=np.uint64)
        h = rng.choice(pool, size=n)
        seed = int(rng.integers(0, 2 ** 63))
        keys = [oracle_mod.splitmix64(seed, i) >> 32 for i in range(n)]
        order = sorted(range(n), key=lambda i: (int(h[i]), keys[i], i))
        keep = set()
        j = 0
        while j < n:
            e = j
            while e < n and h[order[e]] == h[order[j]]:
                e += 1
            r = max(1, math.ceil(math.log2(e - j))) if e - j > 1 else 1
            keep.update(order[j:j + r])
            j = e
        assert oracle_mod.sample(h, seed).tolist() == sorted(keep), trial


def test_draws_are_uniform(oracle_mod):
    """Bucket of 16 keeps 4: over 4,000 seeds each option is kept about 1,000
    times (binomial sd about 27); a draw biased to the first options or to one
    seed bit would be far outside 6 sd."""
    h = np.full(16, 5, np.uint64)
    counts = np.zeros(16)
    for seed in range(4000):
        counts[oracle_mod.sample(h, seed * 7919 + 1)] += 1
    assert np.all(np.abs(counts - 1000) < 6 * 27.4), counts
