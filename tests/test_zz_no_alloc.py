"""cm_eval_batch_static (the entry point for callers that cannot allocate)
against cm_eval_batch on the same seeded inputs: two calls in a row, the
second on a smaller batch, for every precision.  Both run the same kernels in
the same order, so the costs must agree bit for bit; the second call also
shows that nothing of the first call's scratch contents leaks into it."""
import numpy as np
import pytest

from synth import draw_query, model_params

pytestmark = pytest.mark.gpu


def _queries(seed, sizes):
    rng = np.random.default_rng(seed)
    return [draw_query(rng, S, N) for S, N in sizes]


def _fp8_model(cm, model, q):
    """Give the model its FP8 form, calibrated on 64 candidates of q."""
    s_in, s_h = cm.cm_fp8_calibrate(model, np.repeat(q.pipe, 64, axis=0),
                                    q.sched[:, :64].reshape(-1, 40))
    cm.cm_model_prepare_fp8(model, s_in, s_h)
    return s_in


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
def test_static_scratch_equals_workspace_path(prec):
    import torch

    import paper_2012_07145_amd as cm
    from tests.gpucase import workspace_for

    torch.cuda.set_device(0)
    model = cm.cm_model_create(model_params(bias=True))
    big = _queries(71, [(120, 700), (3, 16), (37, 2049), (9, 33), (64, 4096)])
    small = _queries(72, [(5, 100), (17, 31)])
    in_scale = _fp8_model(cm, model, big[0]) if prec == "fp8" else None
    for qs in (big, small):
        print(f"static scratch: {prec}, queries {[(q.n_stages, q.n_cands) for q in qs]}", flush=True)
        batch, cost_ws = cm.pack_queries(qs, prec, in_scale=in_scale)
        ws = workspace_for(cm, qs)
        cm.cm_eval_batch(model, prec, batch, ws, cost_ws)
        cost_st = torch.full_like(cost_ws, float("nan"))
        cm.cm_eval_batch_static(model, prec, batch, cost_st)
        torch.cuda.synchronize()
        a = cost_ws.cpu().numpy().view(np.uint32)
        b = cost_st.cpu().numpy().view(np.uint32)
        n = sum(q.n_cands for q in qs)
        assert np.array_equal(a[:n], b[:n]), (prec, int(np.sum(a[:n] != b[:n])))
        assert np.all(np.isfinite(cost_st.cpu().numpy()[:n]))
        ws.close()
    model.close()


def test_static_scratch_rejects_batches_above_its_limit():
    import torch

    import paper_2012_07145_amd as cm
    from paper_2012_07145_amd import _lib

    torch.cuda.set_device(0)
    model = cm.cm_model_create(model_params())
    q = _queries(73, [(8, 16)])[0]
    per = _lib.CM_STATIC_MAX_STAGES // 8 + 1  # one query too many of 8 stages
    batch, cost = cm.pack_queries([q] * per, "bf16")
    with pytest.raises(cm.CmError) as e:
        cm.cm_eval_batch_static(model, "bf16", batch, cost)
    assert e.value.status == _lib.CM_E2BIG
    model.close()
