"""Memoized feature rows (cm_eval_indexed, Sec. 3.3) on the GPU: costs over a
row table with row numbers per (stage, candidate) are bit-identical to
cm_eval_batch on the materialized rows, and within the usual bars of the
oracle on those rows; a row number outside the table poisons only its
candidate."""
import numpy as np
import pytest

from synth import Query, draw_query, f32_to_bf16_bits, model_params
from tests import gpucase as gc

pytestmark = pytest.mark.gpu

IN_SCALE = 16.0


@pytest.fixture(scope="module")
def cm():
    import torch
    assert torch.cuda.is_available()
    import paper_2012_07145_amd as cm
    return cm


def _memo_case(seed, sizes, table_rows):
    """A table of distinct feature rows and ragged queries whose rows repeat:
    each stage draws its candidates' rows from a small pool (Zipf-like)."""
    rng = np.random.default_rng(seed)
    table = draw_query(rng, 1, table_rows).sched[0]   # [rows][40] raw features
    queries, ridx = [], []
    for S, N in sizes:
        q = draw_query(rng, S, N)
        pool = rng.integers(0, table_rows, size=(S, max(1, N // 8)))
        pick = np.minimum(rng.zipf(1.5, size=(S, N)) - 1, pool.shape[1] - 1)
        r = np.take_along_axis(pool, pick, axis=1).astype(np.int32)
        queries.append(Query(q.pipe, table[r], q.terms))
        ridx.append(r)
    return table, queries, ridx


def _indexed_batch(cm, queries, ridx, table_dev):
    import torch
    descs, pipes, terms, rows = [], [], [], []
    po = ro = to = co = 0
    for q, r in zip(queries, ridx):
        S, N = r.shape
        descs.append((S, N, po, ro, to, co))
        pipes.append(q.pipe.ravel())
        terms.append(q.terms.ravel())
        rows.append(r.ravel())
        po += S * 56
        ro += (S * N + 7) // 8 * 8
        rows.append(np.zeros((S * N + 7) // 8 * 8 - S * N, np.int32))
        to += S * N * 8
        co += N
    b = cm.Batch(descs, torch.from_numpy(np.concatenate(pipes)).cuda(), table_dev,
                 torch.from_numpy(np.concatenate(terms)).cuda())
    return b, torch.from_numpy(np.concatenate(rows)).cuda(), torch.zeros(co, device="cuda")


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_indexed_equals_materialized(cm, oracle_mod, prec):
    import torch
    params = model_params(bias=True)
    m = cm.cm_model_create(params)
    cm.cm_model_prepare_fp8(m, IN_SCALE, 8.0)
    sizes = [(1, 1), (5, 31), (17, 65), (40, 700), (120, 97), (9, 2000)]
    table, queries, ridx = _memo_case(7, sizes, 5000)
    ws = gc.workspace_for(cm, queries)
    if prec == "bf16":
        table_dev = torch.from_numpy(f32_to_bf16_bits(table).view(np.int16).copy()).cuda()
    else:
        table_dev = torch.from_numpy(oracle_mod.fp8_codes(table, IN_SCALE).ravel()).cuda()
    b, rows_t, cost = _indexed_batch(cm, queries, ridx, table_dev)
    cm.cm_eval_indexed(m, prec, b, rows_t, table.shape[0], ws, cost)
    # the same rows materialized
    if prec == "bf16":
        mb, mcost = cm.pack_queries(queries, "bf16")
    else:
        mb, mcost = gc.pack_fp8(cm, queries, [oracle_mod.fp8_codes(q.sched, IN_SCALE) for q in queries])
    cm.cm_eval_batch(m, prec, mb, ws, mcost)
    torch.cuda.synchronize()
    assert torch.equal(cost.view(torch.int32), mcost[:cost.numel()].view(torch.int32))
    if prec == "bf16":   # and the materialized rows against the oracle
        c = cost.cpu().numpy()
        for q, d in zip(queries, b.queries):
            qq = gc.quantized(q)
            ref = oracle_mod.eval_query(params, qq.pipe, qq.sched, qq.terms)
            assert gc.rel_err(c[d[5]:d[5] + d[1]], ref).max() <= 5e-4
    ws.close()
    m.close()


def test_indexed_row_outside_table_is_nan(cm, oracle_mod):
    import torch
    params = model_params()
    m = cm.cm_model_create(params)
    table, queries, ridx = _memo_case(8, [(6, 50), (30, 40)], 300)
    ridx[0][2, 7] = 300          # one past the end
    ridx[1][29, 39] = -1         # negative
    ridx[1][0, 0] = 2 ** 31 - 1  # far outside
    ws = gc.workspace_for(cm, queries)
    table_dev = torch.from_numpy(f32_to_bf16_bits(table).view(np.int16).copy()).cuda()
    b, rows_t, cost = _indexed_batch(cm, queries, ridx, table_dev)
    cm.cm_eval_indexed(m, "bf16", b, rows_t, table.shape[0], ws, cost)
    good = [np.where((r >= 0) & (r < 300), r, 0) for r in ridx]
    b2, rows2, cost2 = _indexed_batch(cm, queries, good, table_dev)
    cm.cm_eval_indexed(m, "bf16", b2, rows2, table.shape[0], ws, cost2)
    torch.cuda.synchronize()
    c, c2 = cost.cpu().numpy(), cost2.cpu().numpy()
    bad = np.zeros(c.size, bool)
    bad[[7, 50 + 39, 50 + 0]] = True
    assert np.all(np.isnan(c[bad]))
    assert np.array_equal(c[~bad].view(np.uint32), c2[~bad].view(np.uint32))
    ws.close()
    m.close()


def test_indexed_errors(cm):
    import torch
    m = cm.cm_model_create(model_params())
    table, queries, ridx = _memo_case(9, [(3, 10)], 20)
    ws = gc.workspace_for(cm, queries)
    b, rows_t, cost = _indexed_batch(cm, queries, ridx, torch.zeros(20 * 40, dtype=torch.int16,
                                                                     device="cuda"))
    with pytest.raises(cm.CmError) as e:
        cm.cm_eval_indexed(m, "fp32", b, rows_t, 20, ws, cost)
    assert e.value.status == -8
    with pytest.raises(cm.CmError):
        cm.cm_eval_indexed(m, "bf16", b, rows_t, 0, ws, cost)
    with pytest.raises(cm.CmError):
        cm.cm_eval_indexed(m, "bf16", b, None, 20, ws, cost)
    with pytest.raises(cm.CmError):
        cm.cm_eval_indexed(m, "bf16", b, rows_t, 2 ** 27, ws, cost)   # > 4 GiB of rows
    with pytest.raises(cm.CmError):
        cm.cm_eval_indexed(m, "fp8", b, rows_t, 20, ws, cost)        # no FP8 form yet
    cm.cm_eval_indexed(m, "bf16", b, rows_t, 20, ws, cost)
    torch.cuda.synchronize()
    ws.close()
    m.close()
