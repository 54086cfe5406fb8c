"""The persistent step and the serving loop in the FP8 form, through the C
ABI: costs and beams bit-identical to the per-call FP8 path (cm_eval_batch
CM_FP8 + cm_topk_per_query) for every launch configuration, with the step's
own hoist following the model's FP8 form when it is prepared again, and
every served beam equal to its request evaluated alone.  The FP8 arithmetic
itself is held to the oracle in test_gpu_fp8.py."""
import numpy as np
import pytest

from synth import Query, draw_query, model_params, workload
from tests import gpucase as gc

pytestmark = pytest.mark.gpu

IN_SCALE = 16.0
CONFIGS = [(0, 1, 1), (0, 1, 0), (64, 1, 1), (512, 2, 1), (1024, 4, 1), (97, 4, 0)]


@pytest.fixture(scope="module")
def cm():
    import torch
    assert torch.cuda.is_available()
    import paper_2012_07145_amd as cm
    return cm


@pytest.fixture(scope="module")
def model(cm):
    m = cm.cm_model_create(model_params(bias=True))
    cm.cm_model_prepare_fp8(m, IN_SCALE, 8.0)
    yield m
    m.close()


def _eager(cm, model, batch, queries, k):
    import torch
    cost = torch.zeros(max(1, batch.n_cands), device="cuda")
    ws = gc.workspace_for(cm, queries, k)
    cm.cm_eval_batch(model, "fp8", batch, ws, cost)
    nq = max(1, batch.n_queries)
    idx = torch.full((nq * k,), -7, dtype=torch.int32, device="cuda")
    val = torch.full((nq * k,), 7.0, device="cuda")
    cm.cm_topk_per_query(cost, batch, k, ws, idx, val)
    torch.cuda.synchronize()
    ws.close()
    return cost.cpu().numpy(), idx.cpu().numpy(), val.cpu().numpy()


def _bits(a):
    return np.asarray(a).view(np.uint32)


def test_fp8_step_equals_per_call_path(cm, model):
    import torch
    W = workload("ragged_17q")
    k = W.k
    batch, _ = cm.pack_queries(W.queries, "fp8", in_scale=IN_SCALE)
    ref = _eager(cm, model, batch, W.queries, k)
    S = sum(q.n_stages for q in W.queries)
    step = cm.cm_step_create(model, "fp8", max_queries=len(W.queries), max_stages=S,
                             max_cands=W.n_cands, max_k=k, slots=2)
    U = torch.empty(S * 32, device="cuda")
    cm.cm_hoist_stages(model, "fp8", batch, U)
    for own_hoist in (True, False):
        for grid, gt, graph in CONFIGS:
            cm.cm_step_set_config(step, grid, gt, graph)
            cost = torch.full((W.n_cands,), -5.0, device="cuda")
            idx = torch.full((len(W.queries) * k,), -7, dtype=torch.int32, device="cuda")
            val = torch.full((len(W.queries) * k,), 7.0, device="cuda")
            cm.cm_step_run(step, batch, None if own_hoist else U, k, cost, idx, val)
            torch.cuda.synchronize()
            assert np.array_equal(_bits(cost.cpu().numpy()), _bits(ref[0][:W.n_cands])), (own_hoist, grid)
            assert np.array_equal(idx.cpu().numpy(), ref[1]), (own_hoist, grid)
            assert np.array_equal(_bits(val.cpu().numpy()), _bits(ref[2])), (own_hoist, grid)
    # a new FP8 form (other hidden scale): the captured step's own hoist
    # follows it, as the per-call path does
    cm.cm_model_prepare_fp8(model, IN_SCALE, 2.0)
    ref2 = _eager(cm, model, batch, W.queries, k)
    assert not np.array_equal(_bits(ref2[0]), _bits(ref[0]))
    cm.cm_step_set_config(step, 0, 1, 1)
    cost = torch.zeros(W.n_cands, device="cuda")
    idx = torch.zeros(len(W.queries) * k, dtype=torch.int32, device="cuda")
    val = torch.zeros(len(W.queries) * k, device="cuda")
    cm.cm_step_run(step, batch, None, k, cost, idx, val)
    torch.cuda.synchronize()
    assert np.array_equal(_bits(cost.cpu().numpy()), _bits(ref2[0][:W.n_cands]))
    assert np.array_equal(idx.cpu().numpy(), ref2[1])
    cm.cm_model_prepare_fp8(model, IN_SCALE, 8.0)
    step.close()


def test_fp8_step_needs_the_fp8_form(cm):
    m = cm.cm_model_create(model_params())
    with pytest.raises(cm.CmError) as e:
        cm.cm_step_create(m, "fp8", max_queries=2, max_stages=10, max_cands=100, max_k=8)
    assert e.value.status == -1
    with pytest.raises(cm.CmError):
        cm.cm_server_create(m, k=8, precision="fp8")
    m.close()


def test_fp8_serve_results_equal_alone(cm, model):
    import torch
    rng = np.random.default_rng(71)
    k = 32
    srv = cm.cm_server_create(model, k=k, max_slots=3, max_sessions=16, max_batch_queries=8,
                              max_batch_cands=1 << 15, precision="fp8")
    sess = []
    for _ in range(10):
        S = int(np.floor(np.exp(rng.uniform(np.log(3), np.log(121)))))
        pipe = draw_query(rng, S, 0).pipe
        sess.append((srv.session_open(pipe), pipe))
    reqs = []
    for r in range(40):
        sid, pipe = sess[int(rng.integers(len(sess)))]
        base = draw_query(rng, pipe.shape[0], int(rng.integers(0, 3000)))
        q = Query(pipe, base.sched, base.terms)
        kk = int(rng.integers(1, k + 1))
        x = torch.from_numpy(np.ascontiguousarray(q.sched, np.float32).ravel()).cuda()
        codes = cm.cm_fp8_encode(x, IN_SCALE) if x.numel() else torch.zeros(16, dtype=torch.uint8, device="cuda")
        terms = torch.from_numpy(np.ascontiguousarray(q.terms, np.float32).ravel()).cuda()
        if terms.numel() == 0:
            terms = torch.zeros(4, device="cuda")
        torch.cuda.synchronize()
        reqs.append((srv.submit(sid, q.n_cands, codes, terms, kk), q, kk, codes, terms))
    for t, q, kk, codes, terms in reqs:
        idx, val, _ = srv.wait(t, 20000)
        b, _ = cm.pack_queries([q], "fp8", in_scale=IN_SCALE)
        _, ri, rv = _eager(cm, model, b, [q], kk)
        assert np.array_equal(idx, ri[:kk]) and np.array_equal(_bits(val), _bits(rv[:kk])), t
    st = srv.stats()
    assert st["completed"] == 40
    # FP8 requests are priced at 72 bytes per row
    assert st["kernel_bytes"] > 0
    srv.close()
