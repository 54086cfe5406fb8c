"""Known-bad-state penalty (cm_penalize_known_bad, Sec. 4.5) followed by
selection on the GPU, bit-exact against the oracle's penalty and selection on
the same seeded costs and hashes."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cm():
    import torch
    assert torch.cuda.is_available()
    import paper_2012_07145_amd as cm
    return cm


def _case(seed, nq=40):
    rng = np.random.default_rng(seed)
    sizes = [int(rng.integers(0, 3000)) for _ in range(nq)]
    sizes[0], sizes[1] = 0, 1
    pool = rng.integers(0, 2 ** 64, size=600, dtype=np.uint64)
    pool[:5] = [0, 1, 2 ** 63, 2 ** 64 - 1, 2 ** 63 - 1]   # unsigned order edges
    costs, hashes, descs, off = [], [], [], 0
    for n in sizes:
        c = rng.lognormal(8, 1, n).astype(np.float32)
        c[rng.random(n) < 0.02] = np.nan
        c[rng.random(n) < 0.02] = 0.0
        c[rng.random(n) < 0.02] = -0.0
        costs.append(c)
        hashes.append(rng.choice(pool, size=n))
        descs.append((1, n, 0, 0, 0, off))
        off += n
    bad = np.sort(np.concatenate([rng.choice(pool, 150), pool[:5], pool[:3]]))  # duplicates too
    return sizes, costs, hashes, descs, bad


@pytest.mark.parametrize("penalty", [1e3, 0.0, float("inf"), -5.0])
def test_penalty_then_topk_matches_oracle(cm, oracle_mod, penalty):
    import torch
    sizes, costs, hashes, descs, bad = _case({1e3: 5, 0.0: 6, float("inf"): 7, -5.0: 8}[penalty])
    k = 32
    flat_c = np.concatenate(costs + [np.zeros(1, np.float32)])
    flat_h = np.concatenate(hashes + [np.zeros(1, np.uint64)])
    cost_t = torch.from_numpy(flat_c.copy()).cuda()
    hash_t = torch.from_numpy(flat_h.view(np.int64).copy()).cuda()
    bad_t = torch.from_numpy(bad.view(np.int64).copy()).cuda()
    batch = cm.Batch(descs, torch.zeros(1, device="cuda"), torch.zeros(1, device="cuda"),
                     torch.zeros(1, device="cuda"))
    ws = cm.cm_workspace_create(len(sizes), 1, max(1, sum(sizes)), 1, k)
    cm.cm_penalize_known_bad(batch, hash_t, bad_t, penalty, cost_t)
    idx = torch.empty(len(sizes) * k, dtype=torch.int32, device="cuda")
    val = torch.empty(len(sizes) * k, device="cuda")
    cm.cm_topk_per_query(cost_t, batch, k, ws, idx, val)
    torch.cuda.synchronize()
    got_c = cost_t.cpu().numpy()
    gi = idx.cpu().numpy().reshape(-1, k)
    gv = val.cpu().numpy().reshape(-1, k)
    for j, (n, c, h) in enumerate(zip(sizes, costs, hashes)):
        want = oracle_mod.penalize(c, h, bad, penalty)
        off = descs[j][5]
        g = got_c[off:off + n]
        same = (g.view(np.uint32) == want.view(np.uint32)) | (np.isnan(g) & np.isnan(want))
        assert np.all(same), j
        oi, ov = oracle_mod.select(want.astype(np.float64), k)
        assert np.array_equal(gi[j], oi), j
        ov32 = ov.astype(np.float32)
        assert np.all((gv[j].view(np.uint32) == ov32.view(np.uint32)) |
                      (np.isnan(gv[j]) & np.isnan(ov32))), j
    assert got_c[-1] == 0.0
    ws.close()


def test_penalty_errors_and_empty_set(cm):
    import torch
    batch = cm.Batch([(1, 4, 0, 0, 0, 0)], torch.zeros(1, device="cuda"),
                     torch.zeros(1, device="cuda"), torch.zeros(1, device="cuda"))
    c = torch.arange(4, dtype=torch.float32, device="cuda")
    h = torch.arange(4, dtype=torch.int64, device="cuda")
    with pytest.raises(cm.CmError):
        cm.cm_penalize_known_bad(batch, h, h[:2], float("nan"), c)
    cm.cm_penalize_known_bad(batch, h, None, 5.0, c)   # empty set: nothing to do
    cm.cm_penalize_known_bad(batch, h, h[2:3], 5.0, c)
    torch.cuda.synchronize()
    assert c.cpu().tolist() == [0.0, 1.0, 7.0, 3.0]
