"""Hierarchical sampling (cm_sample_buckets, Sec. 3.1) on the GPU, bit-exact
against the oracle's sampling on the same seeded hashes and seeds: the same
representatives, in the same (ascending) order, for every query."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cm():
    import torch
    assert torch.cuda.is_available()
    import paper_2012_07145_amd as cm
    return cm


def bucket_hashes(rng, n):
    """n options in buckets of heavy-tailed sizes (many singletons, a few
    buckets of hundreds), hashed to random 64-bit values, shuffled."""
    sizes = []
    while sum(sizes) < n:
        sizes.append(int(min(rng.zipf(1.6), n - sum(sizes))))
    vals = rng.integers(0, 2 ** 64, size=len(sizes), dtype=np.uint64)
    vals[: min(4, len(vals))] = np.array([0, 2 ** 64 - 1, 2 ** 63, 2 ** 63 - 1],
                                         np.uint64)[: min(4, len(vals))]
    h = np.repeat(vals, sizes)
    rng.shuffle(h)
    return h


def run(cm, sampler, hashes_list, seeds):
    import torch
    descs, off = [], 0
    for h in hashes_list:
        descs.append((1, h.size, 0, 0, 0, off))
        off += h.size
    flat = np.concatenate(hashes_list + [np.zeros(1, np.uint64)])
    batch = cm.Batch(descs, torch.zeros(1, device="cuda"), torch.zeros(1, device="cuda"),
                     torch.zeros(1, device="cuda"))
    h_t = torch.from_numpy(flat.view(np.int64).copy()).cuda()
    sel = torch.full((off + 1,), -5, dtype=torch.int32, device="cuda")
    cnt = torch.full((len(hashes_list),), -5, dtype=torch.int32, device="cuda")
    cm.cm_sample_buckets(sampler, batch, h_t, seeds, sel, cnt)
    torch.cuda.synchronize()
    return sel.cpu().numpy(), cnt.cpu().numpy(), descs


def check(oracle_mod, hashes_list, seeds, sel, cnt, descs):
    for j, (h, sd, d) in enumerate(zip(hashes_list, seeds, descs)):
        want = oracle_mod.sample(h, int(sd))
        assert cnt[j] == want.size, (j, cnt[j], want.size)
        assert np.array_equal(sel[d[5]:d[5] + want.size], want), j


def test_sample_matches_oracle_ragged(cm, oracle_mod):
    rng = np.random.default_rng(17)
    sizes = [0, 1, 2, 3, 17, 100, 1000, 4096, 0, 5000, 333] + \
        [int(rng.integers(1, 4000)) for _ in range(40)]
    hashes = [bucket_hashes(rng, n) if n else np.zeros(0, np.uint64) for n in sizes]
    seeds = rng.integers(0, 2 ** 64, size=len(sizes), dtype=np.uint64)
    seeds[:2] = [0, 2 ** 64 - 1]
    sp = cm.cm_sampler_create(64, 200_000)
    sel, cnt, descs = run(cm, sp, hashes, seeds)
    check(oracle_mod, hashes, seeds, sel, cnt, descs)
    assert sel[-1] == -5   # nothing written past the last query's options
    # the sampler is reused: a second, different batch
    hashes2 = [bucket_hashes(rng, n) for n in (5, 70_000, 9)]
    seeds2 = np.array([3, 4, 5], np.uint64)
    sel2, cnt2, descs2 = run(cm, sp, hashes2, seeds2)
    check(oracle_mod, hashes2, seeds2, sel2, cnt2, descs2)
    sp.close()


def test_sample_large_query_and_reduction(cm, oracle_mod):
    """300,000 options in one query; the representatives are a few percent
    of the options, as in the paper's searches."""
    rng = np.random.default_rng(18)
    h = bucket_hashes(rng, 300_000)
    sp = cm.cm_sampler_create(1, 300_000)
    sel, cnt, descs = run(cm, sp, [h], np.array([99], np.uint64))
    check(oracle_mod, [h], [99], sel, cnt, descs)
    assert cnt[0] < 0.5 * h.size
    sp.close()


def test_sample_errors(cm):
    import torch
    sp = cm.cm_sampler_create(2, 100)
    z = torch.zeros(1, device="cuda")
    big = cm.Batch([(1, 101, 0, 0, 0, 0)], z, z, z)
    h = torch.zeros(128, dtype=torch.int64, device="cuda")
    sel = torch.zeros(128, dtype=torch.int32, device="cuda")
    cnt = torch.zeros(4, dtype=torch.int32, device="cuda")
    with pytest.raises(cm.CmError) as e:
        cm.cm_sample_buckets(sp, big, h, [1], sel, cnt)
    assert e.value.status == -5
    three = cm.Batch([(1, 5, 0, 0, 0, 0)] * 3, z, z, z)
    with pytest.raises(cm.CmError):
        cm.cm_sample_buckets(sp, three, h, [1, 2, 3], sel, cnt)
    ok = cm.Batch([(1, 5, 0, 0, 0, 0), (1, 0, 0, 0, 0, 5)], z, z, z)
    with pytest.raises(ValueError):
        cm.cm_sample_buckets(sp, ok, h, [1], sel, cnt)
    cm.cm_sample_buckets(sp, ok, h, [1, 2], sel, cnt)
    torch.cuda.synchronize()
    assert cnt.cpu().tolist()[:2] == [3, 0]   # five equal hashes: ceil(log2 5) = 3 kept
    sp.close()
