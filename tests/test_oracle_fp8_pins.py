"""Pins of the oracle's FP8 (e4m3) form against facts outside the oracle:
the OCP E4M3 format's definition (code table, rounding, saturation, NaN),
hand-worked examples whose quantization points are all exact, invariants of
the model, and closeness to the FP64 model."""
import math

import numpy as np
import pytest

from synth import Query, draw_query, model_params
from tests import cmcases as cc


# OCP E4M3: (code, value) from the format's definition: exponent bias 7,
# 3 mantissa bits, subnormals m * 2^-9, largest finite 448, no infinities.
E4M3_TABLE = [
    (0x00, 0.0), (0x01, 2.0 ** -9), (0x07, 7 * 2.0 ** -9), (0x08, 2.0 ** -6),
    (0x30, 0.5), (0x38, 1.0), (0x39, 1.125), (0x3F, 1.875), (0x40, 2.0),
    (0x48, 4.0), (0x77, 240.0), (0x78, 256.0), (0x7E, 448.0),
    (0x80, -0.0), (0xB8, -1.0), (0xFE, -448.0),
]


def test_e4m3_decode_table(oracle_mod):
    for code, val in E4M3_TABLE:
        got = oracle_mod.e4m3_decode(code)
        assert got == val and math.copysign(1, got) == math.copysign(1, val), (hex(code), got)
    assert math.isnan(oracle_mod.e4m3_decode(0x7F))
    assert math.isnan(oracle_mod.e4m3_decode(0xFF))


def test_e4m3_codes_are_ordered_and_round_trip(oracle_mod):
    vals = [oracle_mod.e4m3_decode(c) for c in range(0x7F)]
    assert all(a < b for a, b in zip(vals, vals[1:]))  # 127 increasing magnitudes
    for c in list(range(0x7F)) + list(range(0x80, 0xFF)):
        assert oracle_mod.e4m3_encode(oracle_mod.e4m3_decode(c)) == c, hex(c)


def test_e4m3_encode_rounding_and_saturation(oracle_mod):
    enc = oracle_mod.e4m3_encode
    # halfway cases go to the even code (last mantissa bit 0)
    assert enc(1.0625) == 0x38            # between 1.0 and 1.125
    assert enc(1.1875) == 0x3A            # between 1.125 and 1.25
    assert enc(0.5 * 2.0 ** -9) == 0x00   # between 0 and the smallest subnormal
    assert enc(1.5 * 2.0 ** -9) == 0x02   # between two subnormals
    assert enc(0.96875) == 0x38           # between 0.9375 and 1.0, across a binade
    # nearest, off the midpoints
    assert enc(1.06) == 0x38 and enc(1.07) == 0x39
    # saturation instead of overflow; no infinities
    assert enc(448.0) == 0x7E and enc(464.0) == 0x7E and enc(1e30) == 0x7E
    assert enc(-1e30) == 0xFE and enc(float("inf")) == 0x7E
    assert enc(float("nan")) == 0x7F
    assert enc(-0.0) == 0x80 and enc(0.0) == 0x00


def test_fp8_scale_is_largest_power_of_two(oracle_mod):
    for amax, want in ((1.0, 256.0), (4.0, 64.0), (448.0, 1.0), (500.0, 0.5), (0.0, 1.0),
                       (3.5, 128.0), (1e-3, 2.0 ** 18)):
        assert oracle_mod.fp8_scale(amax) == want, amax


def _codes(oracle_mod, sched, in_scale):
    flat = [oracle_mod.e4m3_encode(math.log1p(float(x)) * in_scale) for x in sched.ravel()]
    return np.array(flat, np.uint8).reshape(sched.shape)


def test_fp8_form_hand_examples_exact(oracle_mod):
    """Every quantization point of H1/H2 is exact (zero features, integer
    hidden activations, power-of-two weight scales), so the FP8 form gives the
    hand-worked costs exactly."""
    g = cc.load_golden("hand_examples.json")
    params = cc.hand_params()
    for case in g["cases"]:
        pipe, sched, terms = cc.hand_query(case["terms"], n_cands=3)
        codes = _codes(oracle_mod, sched, 1.0)
        for act_scale in (1.0, 4.0, 0.25):
            c = oracle_mod.eval_query_fp8(params, 1.0, act_scale, pipe, codes, terms)
            assert np.all(c == case["cost"]), (case["name"], act_scale, c)
            # the per-stage costs (Sec. 5.2: the predictions that are summed)
            c2, st = oracle_mod.eval_query_fp8(params, 1.0, act_scale, pipe, codes, terms,
                                               stage_costs=True)
            assert np.array_equal(c2, c)
            want = np.repeat(np.array(case["stage_costs"])[:, None], st.shape[1], axis=1)
            assert np.array_equal(st, want), (case["name"], act_scale, st)


def test_fp8_form_quantizes_hidden_and_inputs(oracle_mod):
    """Hand examples whose quantization points are inexact.
    Hidden: H1 with b_1[0] = 0.1, so hidden unit 0 is 3.1, which e4m3 rounds
    to 3 (3.1 * 2^m lies between 3 * 2^m and 3.25 * 2^m, nearer the first):
    coefficient 0 is 3 and the cost 630 (the FP64 model gives 631).
    Inputs: one schedule feature with log1p(x) = 1.1, routed straight to
    coefficient 0 with unit weights; 1.1 rounds to 1.125, so the cost with
    term 8 is 9 (the FP64 model gives 8.8)."""
    g = cc.load_golden("hand_examples.json")
    params = cc.set_params(cc.hand_params(), {"b_1": [[0, 0.1]]})
    case = g["cases"][0]
    pipe, sched, terms = cc.hand_query(case["terms"], n_cands=2)
    ref = oracle_mod.eval_query(params, pipe, sched, terms)
    assert np.allclose(ref, 631.0, rtol=1e-6)
    for act_scale in (1.0, 4.0, 0.125):
        c = oracle_mod.eval_query_fp8(params, 1.0, act_scale, pipe, _codes(oracle_mod, sched, 1.0),
                                      terms)
        assert np.all(c == 630.0), (act_scale, c)
    params = cc.log_params("sched")
    pipe, sched, terms = cc.hand_query([[8, 0, 0, 0, 0, 0, 0, 0]], n_cands=2,
                                       sched0=math.expm1(1.1))
    assert np.allclose(oracle_mod.eval_query(params, pipe, sched, terms), 8.8, rtol=1e-6)  # x is float32
    for in_scale in (1.0, 2.0, 0.5):
        codes = _codes(oracle_mod, sched, in_scale)
        c = oracle_mod.eval_query_fp8(params, in_scale, 1.0, pipe, codes, terms)
        assert np.all(c == 9.0), (in_scale, c)


def test_fp8_form_invariants(oracle_mod):
    params = model_params(bias=True)
    q = draw_query(np.random.default_rng(81), 9, 40)
    codes = _codes(oracle_mod, q.sched, 4.0)
    a = oracle_mod.eval_query_fp8(params, 4.0, 2.0, q.pipe, codes, q.terms)
    # cost terms scaled by 2^m scale every cost exactly
    b = oracle_mod.eval_query_fp8(params, 4.0, 2.0, q.pipe, codes, q.terms * 8)
    assert np.array_equal(b, a * 8)
    # stage permutation
    perm = np.random.default_rng(3).permutation(9)
    c = oracle_mod.eval_query_fp8(params, 4.0, 2.0, q.pipe[perm], codes[perm], q.terms[perm])
    assert np.allclose(c, a, rtol=1e-12)
    # candidate permutation
    cp = np.random.default_rng(4).permutation(40)
    d = oracle_mod.eval_query_fp8(params, 4.0, 2.0, q.pipe, codes[:, cp], q.terms[:, cp])
    assert np.array_equal(d, a[cp])
    # per-stage costs: non-negative, summed over stages they give the cost,
    # and they follow a stage permutation exactly (a stage's cost depends on
    # that stage's data only)
    _, st = oracle_mod.eval_query_fp8(params, 4.0, 2.0, q.pipe, codes, q.terms, stage_costs=True)
    assert np.all(st >= 0)
    assert np.allclose(st.sum(axis=0), a, rtol=1e-12)
    _, stp = oracle_mod.eval_query_fp8(params, 4.0, 2.0, q.pipe[perm], codes[perm], q.terms[perm],
                                       stage_costs=True)
    assert np.array_equal(stp, st[perm])
    assert np.all(a >= 0)


def test_fp8_form_close_to_fp64_model(oracle_mod):
    """The quantization error of e4m3 (3 mantissa bits) bounds how far the FP8
    form can stray from the FP64 model; a wrong scale or a dropped term would
    be off by orders of magnitude."""
    params = model_params()
    rng = np.random.default_rng(82)
    q = draw_query(rng, 12, 300)
    in_scale = 16.0  # log1p of the features stays below 28 = 448 / 16
    codes = _codes(oracle_mod, q.sched, in_scale)
    ref = oracle_mod.eval_query(params, q.pipe, q.sched, q.terms)
    for act_scale in (1.0, 8.0):
        got = oracle_mod.eval_query_fp8(params, in_scale, act_scale, q.pipe, codes, q.terms)
        rel = np.abs(got - ref) / ref
        assert np.median(rel) < 0.05 and rel.max() < 0.5, (act_scale, np.median(rel), rel.max())


def test_fp8_input_codes(oracle_mod):
    """Input codes are e4m3(log1p(x) * s_in): log1p(0) = 0, log1p(-1) = -inf
    saturates to -448, x < -1 has no logarithm (NaN code), log1p(x) = 1.1 lies
    between the codes 1.0 and 1.125, nearer the second, and log1p(1e30) = 69.08
    between 64 and 72 (step 8 in [64, 128)), nearer 72; times 8 it saturates."""
    x = np.array([0.0, -1.0, -2.0, math.expm1(1.1), math.expm1(1.1), np.inf, 1e30, np.nan],
                 np.float32)
    got = oracle_mod.fp8_codes(x, 1.0)
    assert got.tolist() == [0x00, 0xFE, 0x7F, 0x39, 0x39, 0x7E, 0x69, 0x7F]
    assert oracle_mod.fp8_codes(x[3:4], 4.0).tolist() == [0x49]   # 4.4 -> 4.5
    assert oracle_mod.fp8_codes(x[6:7], 8.0).tolist() == [0x7E]
    rng = np.random.default_rng(5)
    y = np.exp(rng.uniform(-12, 12, 300)).astype(np.float32)
    want = [oracle_mod.e4m3_encode(math.log1p(float(v)) * 8.0) for v in y]
    assert oracle_mod.fp8_codes(y.reshape(3, 100), 8.0).ravel().tolist() == want


def test_fp8_error_bound(oracle_mod):
    """Error bound of the hand examples (hidden units h = 3 + b_1[0], 3 and
    ReLU(-4) = 0; W_2 rows (1, 0, 0), (0, 2, 1), (-1, 0, 0); terms H1: 10, 100,
    1000 for coefficients 0..2; H2 adds a stage with 1, 2, 0).
    Coefficient sums off by tau of their largest product: tau * (3*10 + 6*100 +
    3*1000) = 3630 tau for H1, + tau * (3*1 + 6*2) for H2's second stage.
    Hidden rounding: the hoisted rows are off by at most 1e-5 of their terms'
    magnitudes (3 + b_1[0], 7, 4), far from any e4m3 midpoint when b_1[0] = 0;
    with b_1[0] = 0.125 - 2^-20 unit 0 sits just below the midpoint 3.125 of 3
    and 3.25, may round either way, and adds 0.25 * |W_2[:, 0]| . terms =
    0.25 * (10 + 1000) = 252.5 per H1 stage (0.25 * 1 for H2's second)."""
    g = cc.load_golden("hand_examples.json")
    want = {("H1", 0.0): (0.0, 3630.0), ("H2", 0.0): (0.0, 3645.0),
            ("H1", 0.125 - 2.0 ** -20): (252.5, 3630.0), ("H2", 0.125 - 2.0 ** -20): (252.75, 3645.0)}
    for case in g["cases"]:
        pipe, sched, terms = cc.hand_query(case["terms"], n_cands=2)
        codes = _codes(oracle_mod, sched, 1.0)
        for b10 in (0.0, 0.125 - 2.0 ** -20):
            params = cc.set_params(cc.hand_params(), {"b_1": [[0, b10]]})
            flips, per_tau = want[(case["name"], b10)]
            for act_scale in (1.0, 4.0):
                for tau in (0.0, 2e-3):
                    _, bd = oracle_mod.eval_query_fp8(params, 1.0, act_scale, pipe, codes, terms,
                                                      acc_tol=tau)
                    assert np.allclose(bd, flips + per_tau * tau, rtol=1e-9, atol=1e-12), \
                        (case["name"], b10, act_scale, tau, bd)
                    # each stage's share: H1's stage as above; H2's second
                    # stage 15 tau (3*1 + 6*2) plus 0.25 * |W_2[:, 0]| . (1, 2, 0)
                    _, bd2, _, sb = oracle_mod.eval_query_fp8(
                        params, 1.0, act_scale, pipe, codes, terms, acc_tol=tau, stage_costs=True)
                    assert np.array_equal(bd2, bd)
                    f1 = 252.5 if b10 else 0.0
                    assert np.allclose(sb[0], f1 + 3630.0 * tau, rtol=1e-9, atol=1e-12)
                    if case["name"] == "H2":
                        assert np.allclose(sb[1], (0.25 if b10 else 0.0) + 15.0 * tau,
                                           rtol=1e-9, atol=1e-12), (b10, tau, sb)
