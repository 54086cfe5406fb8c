"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test ties the oracle to something other than itself: hand-worked
examples (Sec. 5.2, App. B), closed forms of the log transform, invariants of
the stage sum and of the coefficients, reductions to library routines
(math.fsum, numpy matmul chains) and brute-force ranking on tiny inputs
(Sec. 4's priority queue of the k best states).
"""
import itertools
import math

import numpy as np
import pytest

from synth import model_params, draw_query, unpack_params
from tests import cmcases as cc


def _rand_query(seed, S=5, N=37):
    return draw_query(np.random.default_rng(seed), S, N)


# ---------------------------------------------------------------- hand examples
def test_hand_examples(oracle_mod):
    g = cc.load_golden("hand_examples.json")
    params = cc.hand_params()
    for case in g["cases"]:
        pipe, sched, terms = cc.hand_query(case["terms"], n_cands=3)
        cost = oracle_mod.eval_query(params, pipe, sched, terms)
        assert np.all(cost == case["cost"]), (case["name"], cost)


def test_hand_example_coefficients(oracle_mod):
    params = cc.hand_params()
    pipe, sched, terms = cc.hand_query([[10, 100, 1000, 1, 1, 1, 1, 1]])
    _, coef = oracle_mod.eval_query(params, pipe, sched, terms, coefs=True)
    np.testing.assert_array_equal(coef[0, 0], [3, 6, 0, 0, 0, 0, 0, 0])


@pytest.mark.parametrize("which", [0, 1])
def test_log_transform_closed_form(oracle_mod, which):
    case = cc.load_golden("hand_examples.json")["log_cases"][which]
    route = "sched" if case["sched0"] else "pipe"
    params = cc.log_params(route)
    pipe, sched, terms = cc.hand_query([[1, 0, 0, 0, 0, 0, 0, 0]],
                                       sched0=case["sched0"], pipe0=case["pipe0"])
    cost = oracle_mod.eval_query(params, pipe, sched, terms)[0]
    assert abs(cost - case["cost"]) <= 1e-15 * case["cost"], (case["name"], cost)


def test_log1p_matches_math_over_range(oracle_mod):
    # R4: the transform is log(1 + x) for every feature value, including 0 and
    # values below machine epsilon, checked against math.log1p.
    params = cc.log_params("sched")
    xs = np.array([0.0, 1e-30, 1e-8, 0.5, 1.0, 7.0, 1e3, 3e8, 1e30], np.float32)
    pipe = np.zeros((1, 56), np.float32)
    sched = np.zeros((1, xs.size, 40), np.float32)
    sched[0, :, 0] = xs
    terms = np.zeros((1, xs.size, 8), np.float32)
    terms[0, :, 0] = 1.0
    cost = oracle_mod.eval_query(params, pipe, sched, terms)
    ref = np.array([math.log1p(float(x)) for x in xs])
    np.testing.assert_allclose(cost, ref, rtol=1e-15, atol=0)


# ------------------------------------------------------------------ invariants
def test_stage_permutation_invariance(oracle_mod):
    # I1: the stage sum does not depend on stage order.
    params = model_params(bias=True)
    q = _rand_query(101, S=9, N=50)
    perm = np.random.default_rng(7).permutation(9)
    a = oracle_mod.eval_query(params, q.pipe, q.sched, q.terms)
    b = oracle_mod.eval_query(params, q.pipe[perm], q.sched[perm], q.terms[perm])
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=0)


def test_coefficients_nonnegative(oracle_mod):
    # I2: "positive weights" -- the coefficients are ReLU outputs, so >= 0, and
    # costs of positive terms are >= 0.  Both signs of the pre-activation occur.
    params = model_params(bias=True)
    q = _rand_query(102, S=6, N=200)
    cost, coef = oracle_mod.eval_query(params, q.pipe, q.sched, q.terms, coefs=True)
    assert np.all(coef >= 0.0)
    assert np.any(coef == 0.0) and np.any(coef > 0.0)
    assert np.all(cost >= 0.0)


def test_terms_scale_exactly(oracle_mod):
    # I3: the cost is linear in the terms; a power-of-two scale is exact.
    params = model_params()
    q = _rand_query(103)
    a = oracle_mod.eval_query(params, q.pipe, q.sched, q.terms)
    for m in (-3, 5):
        b = oracle_mod.eval_query(params, q.pipe, q.sched, q.terms * np.float32(2.0 ** m))
        assert np.array_equal(b, a * 2.0 ** m)


def test_zero_terms_stage_adds_nothing(oracle_mod):
    # I4: a stage whose cost terms are all zero contributes exactly 0.
    params = model_params(bias=True)
    q = _rand_query(104, S=4, N=40)
    extra = _rand_query(105, S=1, N=40)
    pipe = np.concatenate([q.pipe, extra.pipe])
    sched = np.concatenate([q.sched, extra.sched])
    terms = np.concatenate([q.terms, np.zeros_like(extra.terms)])
    a = oracle_mod.eval_query(params, q.pipe, q.sched, q.terms)
    b = oracle_mod.eval_query(params, pipe, sched, terms)
    assert np.array_equal(a, b)


def test_split_stages_sum(oracle_mod):
    # I5: stage predictions are summed over stages, so splitting the stages
    # into two queries splits the cost.
    params = model_params(bias=True)
    q = _rand_query(106, S=8, N=30)
    a = oracle_mod.eval_query(params, q.pipe, q.sched, q.terms)
    b1 = oracle_mod.eval_query(params, q.pipe[:3], q.sched[:3], q.terms[:3])
    b2 = oracle_mod.eval_query(params, q.pipe[3:], q.sched[3:], q.terms[3:])
    np.testing.assert_allclose(a, b1 + b2, rtol=1e-13, atol=0)


def test_stage_costs_sum_to_cost(oracle_mod):
    params = model_params()
    q = _rand_query(107, S=7, N=25)
    cost, sc = oracle_mod.eval_query(params, q.pipe, q.sched, q.terms, stage_costs=True)
    np.testing.assert_allclose(sc.sum(0), cost, rtol=1e-13, atol=0)


def test_candidate_permutation(oracle_mod):
    # I6: candidates are independent: permuting them permutes the costs.
    params = model_params(bias=True)
    q = _rand_query(108, S=3, N=64)
    perm = np.random.default_rng(3).permutation(64)
    a = oracle_mod.eval_query(params, q.pipe, q.sched, q.terms)
    b = oracle_mod.eval_query(params, q.pipe, q.sched[:, perm], q.terms[:, perm])
    assert np.array_equal(a[perm], b)
    ia, _ = oracle_mod.select(a, 8)
    ib, _ = oracle_mod.select(b, 8)
    assert np.array_equal(perm[ib], ia)


def test_thread_count_does_not_change_result(oracle_mod):
    params = model_params()
    q = _rand_query(109, S=4, N=300)
    a = oracle_mod.eval_query(params, q.pipe, q.sched, q.terms, nthreads=1)
    b = oracle_mod.eval_query(params, q.pipe, q.sched, q.terms, nthreads=0)
    assert np.array_equal(a, b)


# ------------------------------------------------- reductions to library routines
def test_unit_coefficients_reduce_to_fsum(oracle_mod):
    # R1: W_2 = 0, b_2 = 1 gives every coefficient 1, so the cost is the plain
    # sum of all cost terms of the candidate (math.fsum is correctly rounded).
    params = model_params()
    P = unpack_params(params)
    P["W_2"][:] = 0.0
    P["b_2"][:] = 1.0
    q = _rand_query(110, S=11, N=20)
    cost = oracle_mod.eval_query(params, q.pipe, q.sched, q.terms)
    for i in range(20):
        ref = math.fsum(float(t) for t in q.terms[:, i, :].ravel())
        assert abs(cost[i] - ref) <= 4e-16 * 88 * ref


def test_constant_embeddings(oracle_mod):
    # R2: zero embedding weights and biases make the coefficients the same for
    # every row; the cost is that vector times the summed terms.
    params = model_params(bias=True)
    P = unpack_params(params)
    for n in ("W_p", "b_p", "W_s", "b_s"):
        P[n][:] = 0.0
    P["b_1"][:] = np.abs(P["b_1"]) + 0.1
    P["b_2"][:] = np.linspace(-0.5, 0.5, 8, dtype=np.float32)
    q = _rand_query(111, S=4, N=16)
    cost, coef = oracle_mod.eval_query(params, q.pipe, q.sched, q.terms, coefs=True)
    c0 = coef[0, 0]
    assert np.all(coef == c0)
    assert np.any(c0 == 0) and np.any(c0 > 0)
    h = np.maximum(0.0, P["b_1"].astype(np.float64))
    c_ref = np.maximum(0.0, P["W_2"].astype(np.float64) @ h + P["b_2"])
    np.testing.assert_allclose(c0, c_ref, rtol=1e-14, atol=1e-15)
    ref = q.terms.astype(np.float64).sum(0) @ c_ref
    np.testing.assert_allclose(cost, ref, rtol=1e-13, atol=0)


def test_positive_model_is_a_matmul_chain(oracle_mod):
    # R3: with positive weights, biases and features no ReLU clips, so the
    # model is an affine chain; compared against numpy matmuls.  This pins the
    # orientation of every weight matrix, every bias and the stacking order.
    rng = np.random.default_rng(112)
    params = cc.positive_params(rng)
    P = {k: v.astype(np.float64) for k, v in unpack_params(params).items()}
    q = _rand_query(113, S=3, N=33)
    cost = oracle_mod.eval_query(params, q.pipe, q.sched, q.terms)
    total = np.zeros(33)
    for s in range(3):
        p = np.log1p(q.pipe[s].astype(np.float64))
        x = np.log1p(q.sched[s].astype(np.float64))
        ep = np.tile(P["W_p"] @ p + P["b_p"], (33, 1))
        es = x @ P["W_s"].T + P["b_s"]
        h = np.hstack([ep, es]) @ P["W_1"].T + P["b_1"]
        c = h @ P["W_2"].T + P["b_2"]
        total += np.einsum("ij,ij->i", c, q.terms[s].astype(np.float64))
    np.testing.assert_allclose(cost, total, rtol=1e-12, atol=0)


# ------------------------------------------------------------------- selection
def test_select_all_equal(oracle_mod):
    # I7: equal costs select indices 0..k-1.
    idx, val = oracle_mod.select(np.full(50, 3.5), 8)
    assert idx.tolist() == list(range(8)) and np.all(val == 3.5)


def test_select_signed_zero_tie(oracle_mod):
    # I8: -0 and +0 tie; the lower index wins.
    cost = np.array([1.0, 0.0, -0.0, 2.0, -0.0])
    idx, _ = oracle_mod.select(cost, 4)
    assert idx.tolist() == [1, 2, 4, 0]


def test_select_nan_last_and_padding(oracle_mod):
    cost = np.array([np.nan, np.inf, 5.0, np.nan, -1.0])
    idx, val = oracle_mod.select(cost, 8)
    assert idx.tolist() == [4, 2, 1, 0, 3, -1, -1, -1]
    assert val[5:].tolist() == [np.inf] * 3


def test_select_brute_force_tiny(oracle_mod):
    # Brute force over every ordered k-subset for N <= 7: the selection is the
    # lexicographically smallest sequence of (cost, index) keys.
    rng = np.random.default_rng(114)
    pool = np.array([0.0, -0.0, 1.0, 1.0, 2.5, np.inf, np.nan, -3.0])
    for trial in range(40):
        N = int(rng.integers(1, 8))
        k = int(rng.integers(1, N + 2))
        cost = rng.choice(pool, size=N)
        idx, _ = oracle_mod.select(cost, k)
        kk = min(k, N)
        best = min(itertools.permutations(range(N), kk),
                   key=lambda seq: [cc.key_tuple(cost[i], i) for i in seq])
        assert idx[:kk].tolist() == list(best), (cost, k, idx)
        assert np.all(idx[kk:] == -1)


def test_relu_clips_negative_and_passes_nan(oracle_mod):
    # feature x routed straight to coefficient 0: cost = ReLU(log1p(x)).
    # x = -0.5 gives log1p = -ln 2 < 0, clipped to 0; x = 1 gives ln 2; a NaN
    # feature (or x < -1) gives a NaN cost rather than a silently finite one.
    params = cc.log_params("sched")
    xs = np.array([-0.5, 1.0, np.nan, -3.0], np.float32)
    pipe = np.zeros((1, 56), np.float32)
    sched = np.zeros((1, 4, 40), np.float32)
    sched[0, :, 0] = xs
    terms = np.zeros((1, 4, 8), np.float32)
    terms[0, :, 0] = 1.0
    cost = oracle_mod.eval_query(params, pipe, sched, terms)
    assert cost[0] == 0.0
    assert abs(cost[1] - math.log(2.0)) <= 1e-15
    assert np.isnan(cost[2]) and np.isnan(cost[3])
