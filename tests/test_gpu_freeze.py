"""Per-stage costs (cm_eval_stages) and freezing of the lowest-cost stages
(cm_freeze_stages, Sec. 3.2) on the GPU, through the C ABI.

Per-stage costs: against the oracle's FP64 per-stage costs (bf16: on the
bf16-rounded inputs; FP8: the FP8 form's per-stage costs on the same codes,
under each stage's share of the oracle's error bound).  A single stage lacks the averaging of the stage sum: a
stage whose cost comes from one coefficient near cancellation (b_2 against
W_2 h) carries that coefficient's relative error, so the per-stage bar is 10x
the cost bar at the maximum (float32 1e-4, bf16 5e-3) while the median is
held to the cost-level figure (float32 1e-6, bf16 2e-5).  The costs
themselves are bit-identical to cm_eval_batch.
Freezing: bit-exact against the oracle's rule on the same seeded stage costs
(ties, NaN, signed zeros, out-of-range candidates).  End to end (evaluate,
select the beam's best, freeze), the frozen set must be one the oracle's
per-stage costs allow: identical where the cost gap at the freeze boundary
exceeds the per-stage error bar, and otherwise a valid freezing within it.
"""
import numpy as np
import pytest

from synth import Query, draw_query, model_params, workload
from tests import gpucase as gc

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-4, "bf16": 5e-3}
MEDIAN_TOL = {"fp32": 1e-6, "bf16": 2e-5}
FP8_ACC_TOL = 2e-3  # as test_gpu_fp8.py: ACC_TOL
FP8_TOL = 1e-5      # as test_gpu_fp8.py: FP8_TOL


@pytest.fixture(scope="module")
def cm():
    import torch
    assert torch.cuda.is_available()
    import paper_2012_07145_amd as cm
    return cm


def _stage_view(stage_t, batch):
    st = stage_t.cpu().numpy()
    return [st[d[4] // 8: d[4] // 8 + d[0] * d[1]].reshape(d[0], d[1]) for d in batch.queries]


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
def test_eval_stages_against_oracle(cm, oracle_mod, prec):
    import torch
    params = model_params(bias=True)
    m = cm.cm_model_create(params)
    cm.cm_model_prepare_fp8(m, 16.0, 8.0)
    rng = np.random.default_rng(41)
    qs = [draw_query(rng, S, N) for S, N in ((1, 5), (7, 33), (17, 100), (40, 70))]
    ws = gc.workspace_for(cm, qs)
    if prec == "fp8":  # both sides read the oracle's input codes
        codes = [oracle_mod.fp8_codes(q.sched, 16.0) for q in qs]
        batch, cost = gc.pack_fp8(cm, qs, codes)
    else:
        batch, cost = cm.pack_queries(qs, prec)
    stage = torch.full((sum(q.n_stages * q.n_cands for q in qs) + 8,), -7.0, device="cuda")
    cm.cm_eval_stages(m, prec, batch, ws, cost, stage)
    cost2 = torch.zeros_like(cost)
    cm.cm_eval_batch(m, prec, batch, ws, cost2)
    torch.cuda.synchronize()
    assert torch.equal(cost.view(torch.int32), cost2.view(torch.int32))
    for j, (q, d, sv) in enumerate(zip(qs, batch.queries, _stage_view(stage, batch))):
        c = cost.cpu().numpy()[d[5]:d[5] + d[1]]
        assert np.allclose(sv.astype(np.float64).sum(0), c, rtol=1e-5)
        if prec == "fp8":
            # against the FP8 form's per-stage costs, under each stage's share
            # of the oracle's bound (test_gpu_fp8.py: product sums off by
            # ACC_TOL of their largest product, hoisted rows by 1e-5) plus
            # FP8_TOL for the stage's float32 dot product; the typical stage
            # takes no rounding flip and agrees to float32
            _, _, ref_stage, sbound = oracle_mod.eval_query_fp8(
                params, 16.0, 8.0, q.pipe, codes[j], q.terms, acc_tol=FP8_ACC_TOL,
                stage_costs=True)
            dev = np.abs(sv - ref_stage)
            assert np.all(dev <= sbound + FP8_TOL * np.abs(ref_stage)), (q.n_stages, dev.max())
            rel = np.where(ref_stage != 0, dev / np.where(ref_stage != 0, np.abs(ref_stage), 1.0),
                           dev)
            assert np.mean(rel <= FP8_TOL) >= 0.8 and np.median(rel) <= 2e-6, \
                (q.n_stages, np.mean(rel <= FP8_TOL), np.median(rel))
            continue
        qq = gc.quantized(q) if prec == "bf16" else q
        ref, ref_stage = oracle_mod.eval_query(params, qq.pipe, qq.sched, qq.terms,
                                               stage_costs=True)
        err = np.abs(sv - ref_stage) / np.abs(ref_stage)
        assert err.max() <= TOL[prec], (prec, q.n_stages, err.max())
        assert np.median(err) <= MEDIAN_TOL[prec], (prec, q.n_stages, np.median(err))
    assert np.all(stage.cpu().numpy()[-8:] == -7.0)  # nothing written past the last query
    ws.close()
    m.close()


def test_freeze_matches_oracle_on_seeded_costs(cm, oracle_mod):
    """Stage costs drawn with ties, NaN, +-0 and inf; kept candidates in and
    out of range; 40 queries (two launches of descriptors)."""
    import torch
    rng = np.random.default_rng(42)
    sizes = [(int(rng.integers(1, 200)), int(rng.integers(0, 9))) for _ in range(40)]
    sizes[0] = (1, 1)
    sizes[1] = (2500, 3)   # more stages than one LDS chunk of keys
    descs, off, arrays = [], 0, []
    for S, N in sizes:
        v = rng.choice([0.0, -0.0, 1.0, 2.0, np.nan, np.inf, 3.5], size=(S, N))
        v = np.where(rng.random((S, N)) < 0.6, rng.normal(size=(S, N)), v).astype(np.float32)
        arrays.append(v)
        descs.append((S, N, 0, 0, off * 8, 0))
        off += S * N
    flat = np.concatenate([a.ravel() for a in arrays] + [np.zeros(1, np.float32)])
    cand = np.array([int(rng.integers(-1, N + 1)) if N else 0 for _, N in sizes], np.int32)
    stride = 3
    cand_s = np.full(len(sizes) * stride, 99, np.int32)
    cand_s[::stride] = cand
    batch = cm.Batch(descs, torch.zeros(1, device="cuda"), torch.zeros(1, device="cuda"),
                     torch.zeros(1, device="cuda"))
    total = sum(S for S, _ in sizes)
    frozen = torch.full((total + 5,), 7, dtype=torch.uint8, device="cuda")
    cm.cm_freeze_stages(torch.from_numpy(flat).cuda(), batch, torch.from_numpy(cand_s).cuda(),
                        stride, frozen)
    torch.cuda.synchronize()
    got = frozen.cpu().numpy()
    r = 0
    for (S, N), v, c in zip(sizes, arrays, cand):
        want = (oracle_mod.freeze(v[:, c].astype(np.float64)) if 0 <= c < N
                else np.zeros(S, np.uint8))
        assert np.array_equal(got[r:r + S], want), (S, N, c)
        r += S
    assert np.all(got[total:] == 7)


def test_freeze_end_to_end(cm, oracle_mod):
    """Evaluate the ragged batch with per-stage costs (bf16), take every
    query's best candidate from the beam, freeze its stages."""
    import torch
    W = workload("ragged_17q")
    params = model_params()
    m = cm.cm_model_create(params)
    ws = gc.workspace_for(cm, W.queries)
    batch, cost = cm.pack_queries(W.queries, "bf16")
    stage = torch.empty(W.n_rows + 1, device="cuda")
    cm.cm_eval_stages(m, "bf16", batch, ws, cost, stage)
    k = 32
    idx, val = gc.gpu_topk(cm, cost, batch, k, ws)
    idx_t = torch.from_numpy(idx.ravel().copy()).cuda()
    frozen = torch.empty(sum(q.n_stages for q in W.queries), dtype=torch.uint8, device="cuda")
    cm.cm_freeze_stages(stage, batch, idx_t, k, frozen)
    torch.cuda.synchronize()
    got = frozen.cpu().numpy()
    gpu_stage = _stage_view(stage, batch)
    r, exact = 0, 0
    for j, q in enumerate(W.queries):
        S, c = q.n_stages, int(idx[j, 0])
        qq = gc.quantized(Query(q.pipe, q.sched[:, c:c + 1], q.terms[:, c:c + 1]))
        _, ref_stage = oracle_mod.eval_query(params, qq.pipe, qq.sched, qq.terms, stage_costs=True)
        v = ref_stage[:, 0]
        dev = np.abs(gpu_stage[j][:, c] - v)
        assert np.all(dev <= TOL["bf16"] * np.abs(v)), j
        g = got[r:r + S].astype(bool)
        r += S
        nfree = int(np.ceil(np.log2(S))) if S > 1 else 0
        assert g.sum() == S - nfree
        # two stages can swap order only if their oracle costs differ by less
        # than the two GPU deviations
        bar = 2 * dev.max()
        srt = np.sort(v)
        if S - nfree < S and srt[S - nfree] - srt[S - nfree - 1] > bar:
            assert np.array_equal(g, oracle_mod.freeze(v).astype(bool)), j
            exact += 1
        elif 0 < S - nfree < S:
            assert v[g].max() <= v[~g].min() + bar, j  # a valid freezing within the bar
    assert exact >= len(W.queries) - 2, exact
    ws.close()
    m.close()


def test_freeze_errors(cm):
    import torch
    batch = cm.Batch([(3, 2, 0, 0, 4, 0)], torch.zeros(1, device="cuda"),
                     torch.zeros(1, device="cuda"), torch.zeros(1, device="cuda"))
    st = torch.zeros(16, device="cuda")
    c = torch.zeros(1, dtype=torch.int32, device="cuda")
    f = torch.zeros(3, dtype=torch.uint8, device="cuda")
    with pytest.raises(cm.CmError):  # terms_off 4 is not a multiple of 8
        cm.cm_freeze_stages(st, batch, c, 1, f)
    batch = cm.Batch([(3, 2, 0, 0, 8, 0)], torch.zeros(1, device="cuda"),
                     torch.zeros(1, device="cuda"), torch.zeros(1, device="cuda"))
    with pytest.raises(cm.CmError):
        cm.cm_freeze_stages(st, batch, c, 0, f)
    with pytest.raises(cm.CmError):
        cm.cm_freeze_stages(st, batch, None, 1, f)
    cm.cm_freeze_stages(st, batch, c, 1, f)
    torch.cuda.synchronize()
