"""The persistent beam step (cm_step_*) through the C ABI.

The step evaluates with the same arithmetic as cm_eval_batch (CM_BF16) and
selects like cm_topk_per_query, so its costs and beams must be bit-identical
to theirs for every launch configuration, whether the step hoists itself or
reads hoisted rows, and whether it runs as plain launches or graph replays.
Against the FP64 oracle: costs within the bf16 tolerance on bf16-rounded
inputs; beams bit-exact against the oracle's selection of the GPU's scores.
"""
import numpy as np
import pytest

from synth import Query, draw_query, model_params, workload
from tests import gpucase as gc

pytestmark = pytest.mark.gpu

BF16_TOL = 5e-4


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


def _outs(batch, k):
    import torch
    nq = max(1, batch.n_queries)
    cost = torch.full((max(1, batch.n_cands),), -5.0, dtype=torch.float32, device="cuda")
    idx = torch.full((nq * k,), -7, dtype=torch.int32, device="cuda")
    val = torch.full((nq * k,), 7.0, dtype=torch.float32, device="cuda")
    return cost, idx, val


def _step_for(cm, model, queries, k, slots=2):
    S = sum(q.n_stages for q in queries)
    N = sum(q.n_cands for q in queries)
    return cm.cm_step_create(model, "bf16", max_queries=max(1, len(queries)), max_stages=max(1, S),
                             max_cands=max(1, N), max_k=k, slots=slots)


def _eager(cm, model, queries, k):
    """cm_eval_batch + cm_topk_per_query: the per-call path."""
    import torch
    batch, cost = cm.pack_queries(queries, "bf16")
    ws = gc.workspace_for(cm, queries, k)
    cm.cm_eval_batch(model, "bf16", batch, ws, cost)
    nq = max(1, batch.n_queries)
    idx = torch.full((nq * k,), -7, dtype=torch.int32, device="cuda")
    val = torch.full((nq * k,), 7.0, dtype=torch.float32, device="cuda")
    cm.cm_topk_per_query(cost, batch, k, ws, idx, val)
    torch.cuda.synchronize()
    ws.close()
    return batch, cost.cpu().numpy(), idx.cpu().numpy(), val.cpu().numpy()


def _same_bits(a, b):
    return np.array_equal(np.asarray(a).view(np.uint32), np.asarray(b).view(np.uint32))


def _check_against(batch, cost_np, idx_np, val_np, ref):
    _, rc, ri, rv = ref
    n = batch.n_cands
    assert _same_bits(cost_np[:n], rc[:n])
    nk = len(ri) if batch.n_queries else 0
    assert np.array_equal(idx_np[:nk], ri[:nk])
    assert _same_bits(val_np[:nk], rv[:nk])


CONFIGS = [(0, 1, 1), (0, 1, 0), (64, 1, 1), (512, 2, 1), (1024, 4, 1), (97, 4, 0), (2048, 2, 1),
           (0, 8, 1), (300, 8, 0)]


@pytest.mark.parametrize("own_hoist", [True, False])
def test_step_equals_eval_and_topk_for_every_config(cm, model, own_hoist):
    import torch
    W = workload("ragged_17q")
    k = W.k
    ref = _eager(cm, model, W.queries, k)
    batch = ref[0]
    step = _step_for(cm, model, W.queries, k)
    U = None
    if not own_hoist:
        U = torch.empty(sum(q.n_stages for q in W.queries) * 32, dtype=torch.float32,
                        device="cuda")
        cm.cm_hoist_stages(model, "bf16", batch, U)
    for grid, gt, graph in CONFIGS:
        cm.cm_step_set_config(step, grid, gt, graph)
        cost, idx, val = _outs(batch, k)
        cm.cm_step_run(step, batch, U, k, cost, idx, val)
        torch.cuda.synchronize()
        _check_against(batch, cost.cpu().numpy(), idx.cpu().numpy(), val.cpu().numpy(), ref)
    step.close()


def test_step_graph_replays_match_eager(cm, model):
    """Several batches of different shapes replayed through the captured
    graphs of two slots, with eager work and synchronisations in between;
    every replay equals the per-call path."""
    import torch
    rng = np.random.default_rng(404)
    # the second, fourth and sixth groups together straddle every change of the
    # bf16 stage split (16/17, 32/33, 64/65 stages)
    shapes = [[(5, 100), (40, 700)], [(120, 33), (1, 4096), (17, 17)], [(9, 3000)],
              [(64, 257), (3, 0), (33, 900), (2, 5)], [(5, 100), (40, 700)],
              [(16, 300), (32, 129), (65, 150), (8, 64)]]
    k = 32
    step = cm.cm_step_create(model, "bf16", max_queries=8, max_stages=512, max_cands=1 << 14,
                             max_k=k, slots=2)
    assert cm.cm_step_get_config(step)["use_graph"] == 1
    for rep in range(3):
        for sh in shapes:
            qs = [draw_query(rng, S, N) for S, N in sh]
            ref = _eager(cm, model, qs, k)
            batch = ref[0]
            cost, idx, val = _outs(batch, k)
            cm.cm_step_run(step, batch, None, k, cost, idx, val)
            # eager work of the program between replays
            junk = torch.randn(4096, device="cuda")
            junk = (junk * 2).sum()
            torch.cuda.synchronize()
            _check_against(batch, cost.cpu().numpy(), idx.cpu().numpy(), val.cpu().numpy(), ref)
    step.close()


@pytest.mark.parametrize("k", [1, 32, 256])
def test_step_large_queries_merge_tiles(cm, model, oracle_mod, k):
    """Queries of several selection tiles (N > 4096): the last tile to finish
    merges the per-tile lists inside the step."""
    import torch
    rng = np.random.default_rng(900 + k)
    qs = [draw_query(rng, 6, 20000), draw_query(rng, 40, 9000), draw_query(rng, 3, 4097)]
    ref = _eager(cm, model, qs, k)
    batch = ref[0]
    step = _step_for(cm, model, qs, k)
    for gt in (1, 4):
        cm.cm_step_set_config(step, 0, gt, 1)
        cost, idx, val = _outs(batch, k)
        cm.cm_step_run(step, batch, None, k, cost, idx, val)
        torch.cuda.synchronize()
        c, i, v = cost.cpu().numpy(), idx.cpu().numpy(), val.cpu().numpy()
        _check_against(batch, c, i, v, ref)
        for j, d in enumerate(batch.queries):
            gc.assert_select_bit_exact(oracle_mod, c[d[5]:d[5] + d[1]], i[j * k:(j + 1) * k],
                                       v[j * k:(j + 1) * k], k)
    step.close()


def test_step_edge_queries(cm, model, oracle_mod):
    """No candidates, fewer candidates than k, one stage, the longest
    stages, all-equal costs (ties to the lowest index) in one step."""
    import torch
    rng = np.random.default_rng(5150)
    k = 40
    tie = draw_query(rng, 7, 300)
    tie = Query(tie.pipe, tie.sched, np.zeros_like(tie.terms))  # every cost is +0
    qs = [draw_query(rng, 3, 0), draw_query(rng, 1, 1), draw_query(rng, 1, 39),
          draw_query(rng, 120, 64), tie, draw_query(rng, 16, 41), draw_query(rng, 8, 0)]
    ref = _eager(cm, model, qs, k)
    batch = ref[0]
    step = _step_for(cm, model, qs, k)
    cost, idx, val = _outs(batch, k)
    cm.cm_step_run(step, batch, None, k, cost, idx, val)
    torch.cuda.synchronize()
    c, i, v = cost.cpu().numpy(), idx.cpu().numpy(), val.cpu().numpy()
    _check_against(batch, c, i, v, ref)
    for j, d in enumerate(batch.queries):
        n = d[1]
        bi, bv = i[j * k:(j + 1) * k], v[j * k:(j + 1) * k]
        gc.assert_select_bit_exact(oracle_mod, c[d[5]:d[5] + n], bi, bv, k)
        assert np.all(bi[n:] == -1) and np.all(np.isposinf(bv[n:]))
    assert np.array_equal(i[4 * k:5 * k], np.arange(k))
    step.close()


def test_step_against_oracle(cm, model, params, oracle_mod):
    import torch
    rng = np.random.default_rng(2024)
    qs = [draw_query(rng, int(rng.integers(1, 121)), int(rng.integers(0, 1500)))
          for _ in range(24)]
    k = 32
    batch, _ = cm.pack_queries(qs, "bf16")
    step = _step_for(cm, model, qs, k)
    cost, idx, val = _outs(batch, k)
    cm.cm_step_run(step, batch, None, k, cost, idx, val)
    torch.cuda.synchronize()
    c, i, v = cost.cpu().numpy(), idx.cpu().numpy(), val.cpu().numpy()
    for j, (q, d) in enumerate(zip(qs, batch.queries)):
        g = c[d[5]:d[5] + d[1]]
        if d[1]:
            qq = gc.quantized(q)
            ref = oracle_mod.eval_query(params, qq.pipe, qq.sched, qq.terms)
            assert gc.rel_err(g, ref).max() <= BF16_TOL, j
        gc.assert_select_bit_exact(oracle_mod, g, i[j * k:(j + 1) * k], v[j * k:(j + 1) * k], k)
    step.close()


def test_step_many_queries_and_slots_in_flight(cm, model):
    """200 queries in one step, then several steps queued on one stream with
    no synchronisation between them (slots reused in turn)."""
    import torch
    rng = np.random.default_rng(8)
    k = 8
    many = [draw_query(rng, int(rng.integers(1, 12)), int(rng.integers(0, 60))) for _ in range(200)]
    ref = _eager(cm, model, many, k)
    step = cm.cm_step_create(model, "bf16", max_queries=256, max_stages=4096, max_cands=1 << 15,
                             max_k=k, slots=3)
    cost, idx, val = _outs(ref[0], k)
    cm.cm_step_run(step, ref[0], None, k, cost, idx, val)
    torch.cuda.synchronize()
    _check_against(ref[0], cost.cpu().numpy(), idx.cpu().numpy(), val.cpu().numpy(), ref)

    sets = [[draw_query(rng, int(rng.integers(1, 50)), int(rng.integers(1, 2000)))
             for _ in range(int(rng.integers(1, 9)))] for _ in range(7)]
    refs = [_eager(cm, model, qs, k) for qs in sets]
    outs = []
    for r in refs:
        o = _outs(r[0], k)
        cm.cm_step_run(step, r[0], None, k, *o)
        outs.append(o)
    torch.cuda.synchronize()
    for r, (cost, idx, val) in zip(refs, outs):
        _check_against(r[0], cost.cpu().numpy(), idx.cpu().numpy(), val.cpu().numpy(), r)
    step.close()


def test_step_autotune_keeps_results(cm, model, tmp_path, monkeypatch):
    """The autotuner's pick leaves the results unchanged, is stored in the
    tuning cache (and its file, CM_TUNE_CACHE), is found again by
    cm_step_tuned_config and is applied by a server created afterwards."""
    import torch
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("CM_TUNE_CACHE", str(cache))
    rng = np.random.default_rng(31337)
    qs = [draw_query(rng, int(rng.integers(3, 121)), int(rng.integers(16, 2000)))
          for _ in range(6)]
    k = 32
    ref = _eager(cm, model, qs, k)
    batch = ref[0]
    step = _step_for(cm, model, qs, k)
    cost, idx, val = _outs(batch, k)
    cfg, us = cm.cm_step_autotune(step, batch, None, k, cost, idx, val, reps=3)
    assert cfg["group_tiles"] in (1, 2, 4, 8) and cfg["grid"] > 0 and us > 0
    assert cm.cm_step_get_config(step) == cfg
    rows = sum(q.n_stages * q.n_cands for q in qs)
    assert cm.cm_step_tuned_config(step, len(qs), rows) == cfg
    assert cm.cm_step_tuned_config(step, len(qs)) is not None
    line = [l.split() for l in cache.read_text().splitlines()]
    assert any(int(f[4]) == cfg["grid"] and int(f[5]) == cfg["group_tiles"] and
               int(f[6]) == cfg["use_graph"] for f in line), line
    srv = cm.cm_server_create(model, k=k, max_slots=1, max_sessions=2, max_batch_queries=len(qs),
                              max_batch_cands=1 << 14)
    assert srv.get_step_config() == cm.cm_step_tuned_config(step, len(qs))
    srv.close()
    torch.cuda.synchronize()
    _check_against(batch, cost.cpu().numpy(), idx.cpu().numpy(), val.cpu().numpy(), ref)
    cost, idx, val = _outs(batch, k)
    cm.cm_step_run(step, batch, None, k, cost, idx, val)
    torch.cuda.synchronize()
    _check_against(batch, cost.cpu().numpy(), idx.cpu().numpy(), val.cpu().numpy(), ref)
    step.close()


def test_step_errors(cm, model):
    import torch
    from paper_2012_07145_amd import _lib
    rng = np.random.default_rng(3)
    qs = [draw_query(rng, 4, 50), draw_query(rng, 5, 60)]
    batch, _ = cm.pack_queries(qs, "bf16")
    step = cm.cm_step_create(model, "bf16", max_queries=1, max_stages=100, max_cands=1000,
                             max_k=16, slots=1)
    cost, idx, val = _outs(batch, 16)
    with pytest.raises(cm.CmError) as e:
        cm.cm_step_run(step, batch, None, 16, cost, idx, val)
    assert e.value.status == _lib.CM_E2BIG
    one = cm.Batch(batch.queries[:1], batch.pipe, batch.sched, batch.terms)
    with pytest.raises(cm.CmError) as e:
        cm.cm_step_run(step, one, None, 17, cost, idx, val)
    assert e.value.status == _lib.CM_EINVAL
    bad = cm.Batch([(4, 50, 0, 4, 0, 0)], batch.pipe, batch.sched, batch.terms)
    with pytest.raises(cm.CmError) as e:
        cm.cm_step_run(step, bad, None, 16, cost, idx, val)
    assert e.value.status == _lib.CM_EINVAL
    with pytest.raises(cm.CmError) as e:
        cm.cm_step_set_config(step, 0, 3, 1)
    assert e.value.status == _lib.CM_EINVAL
    with pytest.raises(cm.CmError) as e:
        cm.cm_step_create(model, "fp32")
    assert e.value.status == _lib.CM_EUNSUPPORTED
    torch.cuda.synchronize()
    step.close()


def test_step_matches_per_call_with_out_of_table_features(cm, model):
    # Features of 2^40 and more, infinities and negative values are outside the
    # evaluator's log table; stages of waves that hold one take the computed
    # log transform.  The step kernel and the per-call kernels must still agree
    # bit for bit, selection included (NaN costs sort last).
    import torch
    rng = np.random.default_rng(63)
    queries = [draw_query(rng, S, N) for S, N in ((7, 300), (40, 129), (19, 1000))]
    big = queries[0].sched.copy()
    big[2, 17, 5] = 2.0 ** 41
    big[5, 250, 39] = np.inf
    queries[0] = Query(queries[0].pipe, big, queries[0].terms)
    neg = queries[1].sched.copy()
    neg[33, 64, 0] = -0.25
    neg[10, 3, 12] = 3.0e38
    queries[1] = Query(queries[1].pipe, neg, queries[1].terms)
    k = 32
    ref = _eager(cm, model, queries, k)
    batch = ref[0]
    assert not np.isfinite(ref[1][250])  # the infinite feature reaches its cost
    step = _step_for(cm, model, queries, k)
    cost, idx, val = _outs(batch, k)
    cm.cm_step_run(step, batch, None, k, cost, idx, val)
    torch.cuda.synchronize()
    _check_against(batch, cost.cpu().numpy(), idx.cpu().numpy(), val.cpu().numpy(), ref)
    step.close()
