"""Helpers of the GPU tests: run the library through its C ABI on seeded
inputs and compare with the FP64 oracle."""
from __future__ import annotations

import numpy as np

from synth import Query, bf16_bits_to_f32, f32_to_bf16_bits


def quantized(q: Query) -> Query:
    """The same query with its schedule features rounded to bfloat16 (what
    the bf16 form of the library reads)."""
    return Query(q.pipe, bf16_bits_to_f32(f32_to_bf16_bits(q.sched)), q.terms)


def workspace_for(cm, queries, k=32, extra=1.0):
    S = sum(q.n_stages for q in queries)
    N = sum(q.n_cands for q in queries)
    R = sum(q.n_stages * q.n_cands for q in queries)
    e = lambda v: max(1, int(v * extra) + 1)  # noqa: E731
    return cm.cm_workspace_create(max(1, len(queries)), e(S), e(N), e(R), k)


def gpu_costs(cm, model, queries, prec, ws=None):
    """Evaluate a batch; returns (cost per query as float32 arrays, batch, cost tensor)."""
    import torch
    own = ws is None
    if own:
        ws = workspace_for(cm, queries)
    batch, cost = cm.pack_queries(queries, prec)
    cm.cm_eval_batch(model, prec, batch, ws, cost)
    torch.cuda.synchronize()
    c = cost.cpu().numpy()
    out = [c[d[5]:d[5] + d[1]].copy() for d in batch.queries]
    if own:
        ws.close()
    return out, batch, cost


def gpu_topk(cm, cost_t, batch, k, ws=None):
    import torch
    own = ws is None
    if own:
        ws = cm.cm_workspace_create(max(1, batch.n_queries), 1, max(1, batch.n_cands), 1, k)
    nq = batch.n_queries
    idx = torch.full((max(1, nq * k),), -7, dtype=torch.int32, device="cuda")
    val = torch.full((max(1, nq * k),), 7.0, dtype=torch.float32, device="cuda")
    cm.cm_topk_per_query(cost_t, batch, k, ws, idx, val)
    torch.cuda.synchronize()
    if own:
        ws.close()
    return (idx.cpu().numpy()[:nq * k].reshape(nq, k),
            val.cpu().numpy()[:nq * k].reshape(nq, k))


def assert_select_bit_exact(oracle, cost_f32, idx, val, k):
    """GPU selection == oracle selection applied to the GPU's own scores."""
    oi, ov = oracle.select(np.asarray(cost_f32, np.float64), k)
    assert np.array_equal(idx, oi), (idx[:8], oi[:8])
    ov32 = ov.astype(np.float32)
    same = (val.view(np.uint32) == ov32.view(np.uint32)) | (np.isnan(val) & np.isnan(ov32))
    assert np.all(same), (val[:8], ov32[:8])


def rel_err(gpu, ref):
    gpu = np.asarray(gpu, np.float64)
    return np.abs(gpu - ref) / np.maximum(np.abs(ref), 1e-300)


def topk_agreement(gpu_costs_list, ref_costs_list, k):
    """Pooled |S_gpu & S_ref| / sum min(k, N) over queries."""
    hit = tot = 0
    for g, r in zip(gpu_costs_list, ref_costs_list):
        n = len(r)
        kk = min(k, n)
        sg = set(np.lexsort((np.arange(n), np.asarray(g, np.float64)))[:kk].tolist())
        sr = set(np.lexsort((np.arange(n), r))[:kk].tolist())
        hit += len(sg & sr)
        tot += kk
    return hit / max(tot, 1), hit, tot


def pack_fp8(cm, queries, codes_list, device="cuda"):
    """Lay queries out as for pack_queries, with the given e4m3 code arrays
    (uint8 [S][N][40], one per query) as the schedule features."""
    import torch
    descs, pipes, codes, terms = [], [], [], []
    po = so = to = co = 0
    for q, c in zip(queries, codes_list):
        S, N = c.shape[0], c.shape[1]
        descs.append((S, N, po, so, to, co))
        pipes.append(np.ascontiguousarray(q.pipe, np.float32).ravel())
        codes.append(np.ascontiguousarray(c, np.uint8).ravel())
        terms.append(np.ascontiguousarray(q.terms, np.float32).ravel())
        po += S * 56
        so += S * N * 40
        to += S * N * 8
        co += N
    cat = lambda xs, dt, n: torch.from_numpy(np.concatenate(xs) if xs else np.zeros(n, dt)).to(device)  # noqa: E731
    batch = cm.Batch(descs, cat(pipes, np.float32, 1), cat(codes, np.uint8, 16),
                     cat(terms, np.float32, 4))
    cost = torch.zeros(max(co, 1), dtype=torch.float32, device=device)
    return batch, cost


def gpu_costs_fp8(cm, model, queries, codes_list, ws=None):
    import torch
    own = ws is None
    if own:
        ws = workspace_for(cm, queries)
    batch, cost = pack_fp8(cm, queries, codes_list)
    cm.cm_eval_batch(model, "fp8", batch, ws, cost)
    torch.cuda.synchronize()
    c = cost.cpu().numpy()
    out = [c[d[5]:d[5] + d[1]].copy() for d in batch.queries]
    if own:
        ws.close()
    return out, batch, cost


_FULL = {}


def full_size_query(name="precision_65536x64"):
    """The named workload's single query, drawn once per test process."""
    from synth import workload
    if name not in _FULL:
        _FULL[name] = workload(name)
    return _FULL[name]


def sample_columns(n, idx_top, n_sample=512, seed=0):
    """Candidate indices to check one by one: a seeded random sample plus the
    GPU's own top-k."""
    rng = np.random.default_rng(seed)
    pick = rng.choice(n, size=min(n, n_sample), replace=False)
    return np.unique(np.concatenate([pick, np.asarray(idx_top)[np.asarray(idx_top) >= 0]]))
