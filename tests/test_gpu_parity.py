"""Parity of the gfx950 library with the FP64 oracle, through the C ABI.

Float32 costs: within 1e-5 relative of FP64 for every candidate.
bf16 costs: compared with FP64 evaluated on the same bf16-rounded schedule
features (the arithmetic error alone) within 5e-4 relative; the split
hi/lo products keep it near float32 (about 2^-16 per product).
Selection: bit-exact against the oracle's selection applied to the GPU's own
float32 scores.
"""
import numpy as np
import pytest

from synth import Query, draw_query, model_params, workload
from tests import cmcases as cc
from tests import gpucase as gc

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5
BF16_TOL = 5e-4
BF16_MEDIAN_TOL = 2e-5


@pytest.fixture(scope="module")
def cm():
    import torch
    assert torch.cuda.is_available()
    import paper_2012_07145_amd as cm
    return cm


@pytest.fixture(scope="module")
def params():
    return model_params(bias=True)


@pytest.fixture(scope="module")
def model(cm, params):
    m = cm.cm_model_create(params)
    yield m
    m.close()


# ------------------------------------------------------------ hand examples
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_hand_examples_exact(cm, prec):
    g = cc.load_golden("hand_examples.json")
    m = cm.cm_model_create(cc.hand_params())
    for case in g["cases"]:
        pipe, sched, terms = cc.hand_query(case["terms"], n_cands=70)
        (c,), _, _ = gc.gpu_costs(cm, m, [Query(pipe, sched, terms)], prec)
        assert np.all(c == np.float32(case["cost"])), (prec, case["name"], c[:4])
    m.close()


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-6), ("bf16", 2e-5)])
def test_log_transform_closed_form(cm, prec, tol):
    for case in cc.load_golden("hand_examples.json")["log_cases"]:
        route = "sched" if case["sched0"] else "pipe"
        m = cm.cm_model_create(cc.log_params(route))
        pipe, sched, terms = cc.hand_query([[1, 0, 0, 0, 0, 0, 0, 0]], n_cands=3,
                                           sched0=case["sched0"], pipe0=case["pipe0"])
        (c,), _, _ = gc.gpu_costs(cm, m, [Query(pipe, sched, terms)], prec)
        assert np.all(np.abs(c - case["cost"]) <= tol * case["cost"]), (prec, case["name"], c)
        m.close()


# ------------------------------------------------------------ float32 path
@pytest.mark.parametrize("name", ["plain_64x4", "beam_6400x30"])
def test_fp32_workloads(cm, oracle_mod, name):
    W = workload(name)
    params = model_params()
    m = cm.cm_model_create(params)
    costs, batch, cost_t = gc.gpu_costs(cm, m, W.queries, "fp32")
    for q, c in zip(W.queries, costs):
        ref = oracle_mod.eval_query(params, q.pipe, q.sched, q.terms)
        err = gc.rel_err(c, ref)
        assert err.max() <= FP32_TOL, (name, err.max())
    idx, val = gc.gpu_topk(cm, cost_t, batch, W.k)
    for j, c in enumerate(costs):
        gc.assert_select_bit_exact(oracle_mod, c, idx[j], val[j], W.k)
    agree, _, _ = gc.topk_agreement(costs, [oracle_mod.eval_query(params, q.pipe, q.sched, q.terms)
                                            for q in W.queries], W.k)
    assert agree == 1.0
    m.close()


def test_fp32_with_biases_and_ragged_tail(cm, oracle_mod, model, params):
    q = draw_query(np.random.default_rng(21), 7, 130)  # 3 blocks of 64, tail of 2
    (c,), _, _ = gc.gpu_costs(cm, model, [q], "fp32")
    ref = oracle_mod.eval_query(params, q.pipe, q.sched, q.terms)
    assert gc.rel_err(c, ref).max() <= FP32_TOL


# ------------------------------------------------------------ bf16 path
# the bf16 stage split changes above CHUNK / 2, CHUNK and 2 CHUNK stages
# (CM_STAGE_CHUNK); the sizes straddle each change
CHUNK = 32


@pytest.mark.parametrize("S,N", [(1, 1), (5, 31), (16, 64), (17, 65), (32, 40), (33, 70), (37, 1000),
                                 (64, 33), (65, 50), (120, 97)])
def test_bf16_against_fp64_on_rounded_inputs(cm, oracle_mod, model, params, S, N):
    assert cm.CM_STAGE_CHUNK == CHUNK
    q = draw_query(np.random.default_rng(1000 + S * 7 + N), S, N)
    (c,), batch, cost_t = gc.gpu_costs(cm, model, [q], "bf16")
    qq = gc.quantized(q)
    ref = oracle_mod.eval_query(params, qq.pipe, qq.sched, qq.terms)
    err = gc.rel_err(c, ref)
    assert err.max() <= BF16_TOL, (S, N, err.max())
    # the split products keep the typical error near float32: a lost low
    # part would leave about 1e-3 everywhere
    assert np.median(err) <= BF16_MEDIAN_TOL, (S, N, np.median(err))
    k = min(32, max(1, N))
    idx, val = gc.gpu_topk(cm, cost_t, batch, k)
    gc.assert_select_bit_exact(oracle_mod, c, idx[0], val[0], k)


def test_bf16_full_size_sampled(cm, oracle_mod):
    """65,536 candidates x 64 stages in one call; 512 sampled candidates plus
    the GPU's top-32 recomputed by the oracle on the bf16-rounded inputs; the
    selection bit-exact on the GPU's own scores."""
    W = gc.full_size_query()
    q = W.queries[0]
    params = model_params()
    m = cm.cm_model_create(params)
    (c,), batch, cost_t = gc.gpu_costs(cm, m, [q], "bf16")
    idx, val = gc.gpu_topk(cm, cost_t, batch, W.k)
    gc.assert_select_bit_exact(oracle_mod, c, idx[0], val[0], W.k)
    pick = gc.sample_columns(q.n_cands, idx[0])
    sub = gc.quantized(Query(q.pipe, q.sched[:, pick], q.terms[:, pick]))
    ref = oracle_mod.eval_query(params, sub.pipe, sub.sched, sub.terms)
    err = gc.rel_err(c[pick], ref)
    assert err.max() <= BF16_TOL and np.median(err) <= BF16_MEDIAN_TOL, (err.max(), np.median(err))
    m.close()


def test_ragged_batch_alone_equals_in_mix(cm, oracle_mod):
    """17 ragged queries in one launch: each query's costs are bit-identical to
    the same query evaluated alone; selection bit-exact; agreement reported."""
    W = workload("ragged_17q")
    params = model_params()
    m = cm.cm_model_create(params)
    ws = gc.workspace_for(cm, W.queries)
    mix, batch, cost_t = gc.gpu_costs(cm, m, W.queries, "bf16", ws)
    for j, q in enumerate(W.queries):
        (alone,), _, _ = gc.gpu_costs(cm, m, [q], "bf16", ws)
        assert np.array_equal(alone.view(np.uint32), mix[j].view(np.uint32)), j
    idx, val = gc.gpu_topk(cm, cost_t, batch, W.k, ws)
    refs_q, refs = [], []
    for j, q in enumerate(W.queries):
        gc.assert_select_bit_exact(oracle_mod, mix[j], idx[j], val[j], W.k)
        qq = gc.quantized(q)
        rq = oracle_mod.eval_query(params, qq.pipe, qq.sched, qq.terms)
        assert gc.rel_err(mix[j], rq).max() <= BF16_TOL
        refs_q.append(rq)
        refs.append(oracle_mod.eval_query(params, q.pipe, q.sched, q.terms))
    a_q, _, _ = gc.topk_agreement(mix, refs_q, W.k)
    a, hit, tot = gc.topk_agreement(mix, refs, W.k)
    print(f"\nragged_17q bf16 top-32 agreement: {a_q:.4f} vs FP64 on bf16 inputs, "
          f"{a:.4f} ({hit}/{tot}) vs FP64 on float32 inputs")
    assert a_q >= 0.999
    # Against FP64 on the float32 originals the agreement is set by the bf16
    # rounding of the inputs (the precision form's own quantization), not by
    # the arithmetic (a_q above).  This batch has 544 selections, where one
    # miss is 0.18%, so it cannot resolve the metric's 0.1%; the benchmark
    # measures this reading on every served request (about 32,000
    # selections) and reports it.  Here it is a regression guard only.
    assert a >= 0.995
    ws.close()
    m.close()


def test_bf16_many_queries_split_into_launches(cm, oracle_mod, model, params):
    rng = np.random.default_rng(77)
    qs = [draw_query(rng, int(rng.integers(1, 40)), int(rng.integers(0, 90))) for _ in range(45)]
    for prec, tol in (("fp32", FP32_TOL), ("bf16", BF16_TOL)):
        costs, batch, cost_t = gc.gpu_costs(cm, model, qs, prec)
        for q, c in zip(qs, costs):
            if q.n_cands == 0:
                continue
            qq = q if prec == "fp32" else gc.quantized(q)
            ref = oracle_mod.eval_query(params, qq.pipe, qq.sched, qq.terms)
            assert gc.rel_err(c, ref).max() <= tol, prec
        idx, val = gc.gpu_topk(cm, cost_t, batch, 16)
        for j, c in enumerate(costs):
            gc.assert_select_bit_exact(oracle_mod, c, idx[j], val[j], 16)


# ------------------------------------------------------------ invariants on GPU
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_terms_power_of_two_scale_is_bit_exact(cm, model, prec):
    q = draw_query(np.random.default_rng(31), 20, 77)
    (a,), _, _ = gc.gpu_costs(cm, model, [q], prec)
    q2 = Query(q.pipe, q.sched, q.terms * np.float32(4.0))
    (b,), _, _ = gc.gpu_costs(cm, model, [q2], prec)
    assert np.array_equal(b, a * np.float32(4.0))


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_candidate_permutation(cm, model, prec):
    q = draw_query(np.random.default_rng(32), 18, 100)
    perm = np.random.default_rng(5).permutation(100)
    (a,), _, _ = gc.gpu_costs(cm, model, [q], prec)
    (b,), _, _ = gc.gpu_costs(cm, model, [Query(q.pipe, q.sched[:, perm].copy(),
                                                q.terms[:, perm].copy())], prec)
    assert np.array_equal(a[perm], b)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_stage_permutation_within_tolerance(cm, model, prec):
    q = draw_query(np.random.default_rng(33), 30, 50)
    perm = np.random.default_rng(6).permutation(30)
    (a,), _, _ = gc.gpu_costs(cm, model, [q], prec)
    (b,), _, _ = gc.gpu_costs(cm, model, [Query(q.pipe[perm].copy(), q.sched[perm].copy(),
                                                q.terms[perm].copy())], prec)
    assert np.max(np.abs(a.astype(np.float64) - b) / a) <= 1e-6


def test_coefficients_nonnegative_costs(cm, model):
    q = draw_query(np.random.default_rng(34), 9, 300)
    for prec in ("fp32", "bf16"):
        (c,), _, _ = gc.gpu_costs(cm, model, [q], prec)
        assert np.all(c >= 0)


# ------------------------------------------------------------ selection edges
@pytest.mark.parametrize("k", [1, 8, 32, 64, 65, 128, 200, 256])
def test_topk_edges(cm, oracle_mod, k):
    import torch
    rng = np.random.default_rng(k)
    sizes = [0, 1, 5, 63, 64, 65, 2047, 2048, 2049, 10000]
    arrays = []
    for n in sizes:
        kind = rng.integers(0, 3)
        if kind == 0:
            a = rng.standard_normal(n).astype(np.float32)
        elif kind == 1:
            a = rng.integers(0, 4, n).astype(np.float32)  # heavy ties
        else:
            a = rng.choice(np.array([0.0, -0.0, 1.0, np.inf, np.nan, -2.0], np.float32), n)
        arrays.append(a)
    flat = np.concatenate(arrays + [np.zeros(1, np.float32)])
    off, descs = 0, []
    for a in arrays:
        descs.append((1, len(a), 0, 0, 0, off))
        off += len(a)
    cost_t = torch.from_numpy(flat).cuda()
    batch = cm.Batch(descs, None, None, None)
    idx, val = gc.gpu_topk(cm, cost_t, batch, k)
    for j, a in enumerate(arrays):
        gc.assert_select_bit_exact(oracle_mod, a, idx[j], val[j], k)


def test_all_equal_and_signed_zero(cm, oracle_mod):
    import torch
    a = np.full(5000, 2.5, np.float32)
    b = np.zeros(300, np.float32)
    b[::2] = -0.0
    cost_t = torch.from_numpy(np.concatenate([a, b])).cuda()
    batch = cm.Batch([(1, 5000, 0, 0, 0, 0), (1, 300, 0, 0, 0, 5000)], None, None, None)
    idx, val = gc.gpu_topk(cm, cost_t, batch, 32)
    assert idx[0].tolist() == list(range(32))
    assert idx[1].tolist() == list(range(32))
    gc.assert_select_bit_exact(oracle_mod, b, idx[1], val[1], 32)


# ------------------------------------------------------------ errors
def test_capacity_and_alignment_errors(cm, model):
    import torch
    q = draw_query(np.random.default_rng(40), 4, 100)
    batch, cost = cm.pack_queries([q], "bf16")
    small = cm.cm_workspace_create(1, 4, 50, 400, 8)
    with pytest.raises(cm.CmError) as e:
        cm.cm_eval_batch(model, "bf16", batch, small, cost)
    assert e.value.status == -5
    ws = cm.cm_workspace_create(1, 4, 100, 400, 8)
    bad = cm.Batch([(4, 100, 0, 4, 0, 0)], batch.pipe, batch.sched, batch.terms)
    with pytest.raises(cm.CmError) as e:
        cm.cm_eval_batch(model, "bf16", bad, ws, cost)
    assert e.value.status == -1
    with pytest.raises(cm.CmError) as e:
        cm.cm_eval_batch(model, 7, batch, ws, cost)
    assert e.value.status == -8
    idx = torch.empty(8, dtype=torch.int32, device="cuda")
    val = torch.empty(8, dtype=torch.float32, device="cuda")
    with pytest.raises(cm.CmError):
        cm.cm_topk_per_query(cost, batch, 9, ws, idx, val)
    small.close()
    ws.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_hoist_then_eval_equals_eval_batch(cm, model, prec):
    import torch
    rng = np.random.default_rng(50)
    qs = [draw_query(rng, int(rng.integers(1, 40)), int(rng.integers(1, 200))) for _ in range(40)]
    ws = gc.workspace_for(cm, qs)
    batch, cost_a = cm.pack_queries(qs, prec)
    cm.cm_eval_batch(model, prec, batch, ws, cost_a)
    U = torch.empty(sum(q.n_stages for q in qs) * 32, device="cuda")
    cost_b = torch.zeros_like(cost_a)
    cm.cm_hoist_stages(model, prec, batch, U)
    cm.cm_eval_hoisted(model, prec, batch, U, ws, cost_b)
    torch.cuda.synchronize()
    assert torch.equal(cost_a, cost_b)
    ws.close()


def test_negative_and_signed_zero_features(cm, oracle_mod, model, params):
    # log1p is defined above -1: a feature in (-1, 0) and a -0 follow the
    # oracle in both forms; a feature below -1 makes the candidate's cost NaN
    q = draw_query(np.random.default_rng(60), 9, 70)
    sched = q.sched.copy()
    sched[3, 5, 7] = -0.5
    sched[6, 9, 33] = -0.0
    sched[2, 11, 1] = -3.0
    q2 = Query(q.pipe, sched, q.terms)
    ok = np.ones(70, bool)
    ok[11] = False
    for prec, tol in (("fp32", FP32_TOL), ("bf16", BF16_TOL)):
        (c,), _, _ = gc.gpu_costs(cm, model, [q2], prec)
        assert np.isnan(c[11]), prec
        qq = q2 if prec == "fp32" else gc.quantized(q2)
        ref = oracle_mod.eval_query(params, qq.pipe, qq.sched, qq.terms)
        assert np.isnan(ref[11])
        assert gc.rel_err(c[ok], ref[ok]).max() <= tol, prec


def test_bf16_long_query_reads_hoisted_rows_from_memory(cm, oracle_mod, model, params):
    # more stages than the evaluator keeps in LDS
    q = draw_query(np.random.default_rng(61), 300, 40)
    (c,), _, _ = gc.gpu_costs(cm, model, [q], "bf16")
    qq = gc.quantized(q)
    ref = oracle_mod.eval_query(params, qq.pipe, qq.sched, qq.terms)
    assert gc.rel_err(c, ref).max() <= BF16_TOL


def test_bf16_log_table_equals_computed_log(cm, oracle_mod):
    # The bf16 evaluator looks the log transform of a feature code up in a
    # table unless a stage of the wave holds a code outside it (2^40 and up,
    # infinities, NaNs, negatives); then it computes it.  Both must give the
    # same bits.  Feature 5 walks every finite non-negative bf16 code; feature
    # 6 has zero weight, and in the second query it is 2^50 everywhere, which
    # sends every stage down the computed path without changing the cost.
    from synth import bf16_bits_to_f32
    from synth.workloads import PARAM_LAYOUT
    params = model_params(bias=True).copy()
    off = 0
    for name, shape in PARAM_LAYOUT:
        if name == "W_s":
            ws = params[off:off + shape[0] * shape[1]].reshape(shape)
            ws[:, 6] = 0.0
            break
        off += int(np.prod(shape))
    m = cm.cm_model_create(params)
    S, N = 8, 4096
    q = draw_query(np.random.default_rng(62), S, N)
    codes = (np.arange(S * N) % 0x7f80).astype(np.uint16).reshape(S, N)
    sched = q.sched.copy()
    sched[:, :, 5] = bf16_bits_to_f32(codes)
    sched[:, :, 6] = 1.0
    a = Query(q.pipe, sched, q.terms)
    sched_b = sched.copy()
    sched_b[:, :, 6] = 2.0 ** 50
    b = Query(q.pipe, sched_b, q.terms)
    (ca,), _, _ = gc.gpu_costs(cm, m, [a], "bf16")
    (cb,), _, _ = gc.gpu_costs(cm, m, [b], "bf16")
    m.close()
    assert np.array_equal(ca.view(np.uint32), cb.view(np.uint32))
    ref = oracle_mod.eval_query(params, a.pipe, gc.quantized(a).sched, a.terms)
    assert gc.rel_err(ca, ref).max() <= BF16_TOL
